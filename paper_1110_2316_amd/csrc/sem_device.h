// Device-side data of the spectral element library (shared by kernels and API).
#pragma once
#include <cstdint>

#include <hip/hip_runtime.h>

namespace sem {

// Scalars of the device-resident PCG loop.
struct Scalars {
    double rho;       // r^T z
    double alpha;
    double beta;
    double pq;        // p^T X p
    double rr;        // r^T r
    double bb;        // b^T b
    double relres;    // sqrt(rr / bb)
    double tol;
    int iter;
    int maxit;
    int done;
    int status;
};

struct DevData {
    int W, n, m, E, Ereal, ncd, nfaces, nvirt;
    long long nreal_dof, ndof;
    const int* kind;            // [E]
    const int* real_index;      // [E]
    const int* cdof;            // [E]
    const int* cdir;            // [E]
    const int* virt_index;      // [E] index among corner elements or -1
    const unsigned char* slot_active;  // [E][6]
    const unsigned* fmask;      // [Ereal]
    const double* Im;           // [m][n]
    const double* D1m;
    const double* D2m;
    const double* Dn;           // [n][n]
    const double* K;            // [m][m]
    const double* wm;           // [m]
    const double* coef;         // [Ereal][9][m^3]
    const double* dvol;         // [Ereal][m^3]
    double* trace;              // [E][6][4][n^2]
    double* slotres;            // [E][6][4][n^2]
    const int* face_int;        // [F][8] eA fA eB fB orient nq pmodeA pmodeB
    const double* face_w;       // [F][4][3]
    const long long* face_off;  // [F][3] PA offset, PB offset, data offset (-1 if none)
    const double* pcoef;
    const double* gdata;
    const double* pbasis;       // [nb][n][n]
    const double* peig;         // [nb][n]
    const int* pidx;            // [Ereal][3]
    const double* pscale;       // [Ereal]
    const double* cinv;         // [ncd]
    const int* cptr;            // [ncd+1]
    const int* cidx;
    double* cpart;              // [nvirt][n]
    double* part_a;             // [E+1] partial sums
    double* part_b;
    double* part_c;
};

// Launchers for one compile-time degree W.
struct Ops {
    void (*volume)(hipStream_t, const DevData&, const double*, double*, int, const double*, double*, const Scalars*);
    void (*face)(hipStream_t, const DevData&, int, const Scalars*);
    void (*gather)(hipStream_t, const DevData&, double*, const double*, Scalars*, int, int);
    void (*update)(hipStream_t, const DevData&, int, double*, double*, double*, double*, const double*, const double*,
                   Scalars*);
    void (*error)(hipStream_t, const DevData&, const double*, int, const double*, const double*, const double*,
                  const double*, const double*, const double*, double*);
};

bool get_ops(int W, Ops& ops);
void launch_sub(hipStream_t st, double* r, const double* a, const double* b, long long n);

}  // namespace sem
