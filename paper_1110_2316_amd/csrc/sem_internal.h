// Internal data structures of the spectral element library (host side).
#pragma once
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/sem.h"

namespace sem {

constexpr int REG = 0, VTX = 1, VE = 2, EDGE = 3;
constexpr int REAL = 0, CORNER_CONST = 1, CORNER_POLY = 2;
constexpr int AFFINE = 0, VTX_BOX = 1, VE_BOX = 2, EDGE_BOX = 3, VTX_PATCH = 4, COLUMN = 5;
constexpr int BC_INTERIOR = 0, BC_DIRICHLET = 1, BC_SKIP = 2, BC_NEUMANN = 3;
constexpr int NFIELD = 10;  // u11 u22 u33 u12 u13 u23 u1 u2 u3 u
constexpr int MAXQ = 4;     // quantities per face term

// One face term of the functional (an interior pair or a Dirichlet face).
struct FaceHost {
    int eA, fA, eB, fB, orient;
    int region;
    int nq;                         // quantities
    double wts[MAXQ][3];            // alpha, beta, gamma per quantity
    int pmodeA, pmodeB;             // 0: constant 4x4 block, 1: per point
    std::vector<double> PA, PB;     // [nq][4][P] or [nq][4]
    // Dirichlet data directions: kind 0 value, 1 gradient dotted with dir
    int dkind[MAXQ];
    std::vector<double> ddir;       // [nq][P][3]
    std::vector<double> xA;         // [P][3]
    std::vector<double> nuv;        // [P][3] outward unit normal (Neumann face terms)
};

struct HostSetup {
    int W = 0, n = 0, m = 0;
    int E = 0, Ereal = 0, ncd = 0;
    int64_t ndof = 0, nreal_dof = 0;
    std::vector<int> region, kind, chart, cdof, cdir, real_index;
    std::vector<double> box, frame, mframe, origin, patch;
    std::vector<int> nbr, nbr_face, orient, bc;

    // 1D data
    std::vector<double> xn, wn, xm, wm;
    std::vector<double> Im, D1m, D2m;   // [m][n] fine-grid values of l_j, l_j', l_j''
    std::vector<double> Dn;             // [n][n] l_j'(xn_i)
    std::vector<double> K;              // [m][m] discrete H^{1/2} double sum

    // volume
    std::vector<double> coef;           // [Ereal][NFIELD][m^3]
    std::vector<uint32_t> fmask;        // [Ereal]
    std::vector<double> svol;           // [Ereal][m^3] sqrt(w |J|) omega
    std::vector<double> xvol;           // [Ereal][m^3][3]

    // faces
    std::vector<FaceHost> faces;
    std::vector<int> dir_faces;         // indices of Dirichlet face terms
    std::vector<int> neu_faces;         // indices of Neumann face terms
    std::vector<double> neu_wfac;       // [neu_faces][P] factor of the Neumann datum (1, rho^2/r or r)
    std::vector<uint8_t> slot_active;   // [E][6]

    // preconditioner
    std::vector<double> pbasis;         // [nb][n][n] Phi (column j = eigenvector j)
    std::vector<double> peig;           // [nb][n]
    std::vector<int> pidx;              // [Ereal][3]
    std::vector<double> pscale;         // [Ereal]
    std::vector<double> pg;             // [Ereal][3] 1D scale g_d of the element's separable form
    std::vector<int> deg;               // [Ereal][3] polynomial degree per lambda direction (W: ungraded)
    std::vector<double> cinv;           // [ncd] inverse diagonal of the corner blocks

    // corner reduction: for each corner DOF, list of (virtual element slot, index)
    std::vector<int> virt_elems;        // element ids of corner elements
    std::vector<int> cptr, cidx;        // CSR over corner dofs into virtual partial array

    // error quadrature
    int nq = 0;
    std::vector<double> xg, wg;         // Gauss nodes/weights
    std::vector<double> Lg, Lg1;        // [nq][n]
    std::vector<double> err_x;          // [Ereal][nq^3][3]
    std::vector<double> err_ji;         // [Ereal][nq^3][9] J^{-1}
    std::vector<double> err_w;          // [Ereal][nq^3] w |J|
};

// Builds everything; throws std::runtime_error on invalid input.
void build_host_setup(const sem_mesh* mesh, HostSetup& S);
// (Re)computes the volume coefficient fields for the operator with
// coefficients a [npts][6] (a11 a22 a33 a12 a13 a23), beta [npts][3], c [npts]
// at the volume points (NULL: -Laplace's a = I, beta = 0, c = 0).
void volume_fields(HostSetup& S, const double* a, const double* beta, const double* c);
// (Re)builds the separable preconditioner's 1D bases (pbasis, peig, pidx)
// from pg and deg: per element and direction the pencil (g^4 S2 + g^2 S1, F)
// restricted to the polynomials of degree deg (Sec. 5.2 forms on the graded
// space of Sec. 2.3), its eigenvectors padded with zero columns to n.
void separable_bases(HostSetup& S);
// Orthogonal projector (n x n, row-major) onto the polynomials of degree <= w
// in the values at the n = W+1 GLL nodes.
std::vector<double> degree_projector(const HostSetup& S, int w);

}  // namespace sem
