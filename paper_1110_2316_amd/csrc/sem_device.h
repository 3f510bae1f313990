// Device-side data of the spectral element library (shared by kernels and API).
#pragma once
#include <cstdint>

#include <hip/hip_runtime.h>

namespace sem {

// Fields of the volume operator: u11 u22 u33 u12 u13 u23 u1 u2 u3 u (lambda
// derivatives at the fine GLL points), one coefficient array each.
constexpr int VFIELDS = 10;

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

// Operator data in one compute precision (double, or float for the inner
// solves of the mixed-precision path).
template <class T>
struct Dev {
    const T* Im = nullptr;      // [m][n]
    const T* D1m = nullptr;
    const T* D2m = nullptr;
    const T* Dn = nullptr;      // [n][n]
    const T* K = nullptr;       // [m][m]
    const T* wm = nullptr;      // [m]
    const T* coef = nullptr;    // [Ereal][VFIELDS][a][c][b] (fine-grid point (a, b, c), b fastest)
    const T* pcoef = nullptr;   // face coefficients
    const T* face_w = nullptr;  // [F][4][3]
    T* trace = nullptr;         // [E][6][4][n^2]
    T* slotres = nullptr;       // [E][6][4][n^2]
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
    Dev<double> d64;
    Dev<float> d32;
    const double* Dn;           // [n][n] (FP64, for the gather)
    const double* dvol;         // [Ereal][m^3]
    const int* face_int;        // [F][8] eA fA eB fB orient nq pmodeA pmodeB
    const long long* face_off;  // [F][3] PA offset, PB offset, data offset (-1 if none)
    const double* gdata;
    const double* pbasis;       // [nb][n][n]
    const double* peig;         // [nb][n]
    const int* pidx;            // [Ereal][3]
    const double* pscale;       // [Ereal]
    const double* cinv;         // [ncd]
    // an operator apply restricted to some elements (the element-block
    // assembly): the volume and gather kernels run on sub_elem (element
    // ids), the face kernel on sub_face (face term indices), the corner
    // reduction not at all; null: every element and face term
    const int* sub_elem;
    int nsub_elem;
    const int* sub_face;
    int nsub_face;
    // graded degrees: the real elements with a degree below W in some
    // direction, their degrees (w1 | w2 << 8 | w3 << 16) and the projector
    // table [W+1][n][n] (0 elements: ungraded)
    int nproj;
    const int* proj_elem;
    const int* proj_deg;
    const double* projtab;
    int pk;                     // preconditioner: 0 separable; element blocks: 1 FP64 inverse,
                                // 2 float factor G, 3 float inverse
    const double* B64;          // [stored blocks][n3][ldb] X_ee^-1, full symmetric, by columns
    const float* B32;           // the same rounded to float
    int ldb;                    // column stride: n3 + 3 rounded up to a multiple of 32
    const int* bidx;            // [Ereal] stored block of each element (equal blocks are stored once)
    const int* bflip;           // [Ereal] lambda axes reversed between the element and its stored block
                                // (bit d: lambda_d; X_ee[a][b] = B[f(a)][f(b)], f the reversal)
    const int* uorder;          // [Ereal] elements grouped by stored block (schedule of k_update)
    // tasks of the grouped update: up to G elements (uorder[first .. first + count)) of one stored block
    int ntasks;
    const int* task_first;
    const int* task_count;
    const int* task_block;
    const float* G32;           // [Ereal][n3 (n3 + 1) / 2] G = L^-1 by columns (float)
    const float* G32r;          // the same by rows
    const double* Gc64;         // [ncd (ncd + 1) / 2] corner block, same layout
    const float* Gc32;
    double* cscratch;           // [ncd]
    const int* cptr;            // [ncd+1]
    const int* cidx;
    double* cpart;              // [nvirt][n]
    double* part_a;             // [E+1] partial sums
    double* part_b;
    double* part_c;
    // several right-hand sides in one launch (1 otherwise): item = blockIdx.x / nrhs,
    // right-hand side = blockIdx.x % nrhs; per right-hand side buffers follow
    // each other at these strides (elements of their type)
    int nrhs;
    long long vstride;          // vectors: ndof
    long long tstride;          // traces / face results: E 6 4 n^2
    long long pstride;          // partial sums
    long long cpstride;         // corner partials
    long long csstride;         // corner scratch
};

// offsets the per right-hand side buffers of D to right-hand side rh
__host__ __device__ inline void bind_rhs(DevData& D, int rh) {
    if (rh == 0) return;
    if (D.d64.trace) { D.d64.trace += rh * D.tstride; D.d64.slotres += rh * D.tstride; }
    if (D.d32.trace) { D.d32.trace += rh * D.tstride; D.d32.slotres += rh * D.tstride; }
    D.part_a += rh * D.pstride;
    D.part_b += rh * D.pstride;
    D.part_c += rh * D.pstride;
    D.cpart += rh * D.cpstride;
    D.cscratch += rh * D.csstride;
}

template <class T>
__host__ __device__ inline const Dev<T>& dev_of(const DevData& D);
template <>
__host__ __device__ inline const Dev<double>& dev_of<double>(const DevData& D) { return D.d64; }
template <>
__host__ __device__ inline const Dev<float>& dev_of<float>(const DevData& D) { return D.d32; }

// Launchers for one compile-time degree W and compute precision.
using VolumeFn = void (*)(hipStream_t, const DevData&, const double*, double*, int, const double*, double*,
                          const Scalars*);
struct Ops {
    VolumeFn volume;            // the selected tile of the element kernel
    VolumeFn volume_tile[3];    // tile candidates (lam1-slab widths, see tile_slab)
    int tile_slab[3];
    int tile;                   // index of the selected candidate
    void (*face)(hipStream_t, const DevData&, int, const Scalars*);
    void (*gather)(hipStream_t, const DevData&, double*, const double*, Scalars*, int, int);
    void (*update)(hipStream_t, const DevData&, int, double*, double*, double*, double*, const double*, const double*,
                   Scalars*);
    void (*error)(hipStream_t, const DevData&, const double*, int, const double*, const double*, const double*,
                  const double*, const double*, const double*, double*);
    void (*conform)(hipStream_t, const DevData&, const double*, double*, const int*, const double*);
    void (*project)(hipStream_t, const DevData&, double*);          // graded space: u <- Q u in place
    // element blocks: B <- Q B Q + s (I - Q), s = tr(B) / n3 per graded element (scale: [nproj] work)
    void (*block_project)(hipStream_t, const DevData&, double*, double*);
};

bool get_ops(int W, Ops& ops);        // FP64 operator
bool get_ops_f32(int W, Ops& ops);    // FP32 contractions (update / error stay FP64)
int volume_lds_bytes(int W, int fp32);
void update_shape(int W, int* G, int* parts);   // elements per task, row parts of the element-block update
void launch_flag_ops(hipStream_t st, Scalars* sc, const int* op, int R);
void launch_axpy_alpha_multi(hipStream_t st, double* u, const double* p, const Scalars* sc, long long n, int R);
void launch_sub(hipStream_t st, double* r, const double* a, const double* b, long long n);
void launch_unit_vector(hipStream_t st, double* v, const int* elems, int ne, int n3, int j0, int R, long long vs);
void launch_unit_clear(hipStream_t st, double* v, const int* elems, int ne, int n3, int j0, int R, long long vs);
void launch_extract_column(hipStream_t st, double* B, const double* y, const int* elems, int ne, int n3, int j0, int R,
                           long long vs);
void launch_block_sig(hipStream_t st, const double* A, int n3, int nblk, double* sig);
void launch_block_cmp(hipStream_t st, const double* A, const double* const* R, int n, const int* trip, int ntrip,
                      double* out);
void launch_pack_lower(hipStream_t st, const double* A, double* B64, float* G32, float* G32r, int n3, int nblk);
void launch_pack_full64(hipStream_t st, const double* A, double* B, int ld, int n3, int nblk);
void launch_pack_full32(hipStream_t st, const double* A, float* B, int ld, int n3, int nblk);
void launch_unpack_full(hipStream_t st, const float* B, int ld, double* A, int n3, int nblk);
void launch_unpack_lower(hipStream_t st, const float* P32, double* A, int n3, int nblk);
void launch_sum_rows(hipStream_t st, const double* part, int nrows, int K, double* out);
constexpr int SOURCE_MAXDEG = 12;
void launch_source_eval(hipStream_t st, const double* xv, const double* svol, const double* theta, int deg,
                        long long npts, double* dvol);
void launch_source_fourier(hipStream_t st, const double* xv, const double* svol, const double* coef, int nmodes,
                           long long npts, double* dvol);
void launch_source_project(hipStream_t st, const double* xv, const double* svol, const double* z, int deg, int m3,
                           int nelem, double* part, double* out);

}  // namespace sem
