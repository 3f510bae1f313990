// HIP kernels (gfx950) of the least-squares h-p spectral element operator.
//
// One PCG iteration on the normal equations X U = b (thesis Sec. 5.3) is four
// launches:
//   k_volume  per element: (fused p = z + beta p), weighted PDE residual on the
//             (2W+1)^3 GLL grid and its exact discrete adjoint (sum-factorised
//             1D contractions, LDS-staged), traces of u and grad_lam u on the
//             element faces;
//   k_face    per face term: jumps / boundary quantities on the (2W+1)^2 face
//             grid, weighting by the separable L2 / H^{1/2} face matrices,
//             transposed traces;
//   k_gather  per element: adds the transposed face traces, partial p^T q,
//             corner partial sums; k_corner_q sums them per corner unknown;
//             k_fin_gather (one block) finishes p^T q and alpha;
//   k_update  per element: u += alpha p, r -= alpha q, z = W^{-1} r (separable
//             preconditioner, Sec. 5.2), partial r^T z, r^T r; k_fin_update
//             (one block) computes beta and the stopping test.
// All reductions are fixed-order (no floating-point atomics), so runs are
// bit-reproducible.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <type_traits>

#include "sem_device.h"

namespace sem {

constexpr int BLOCK = 256;

__device__ inline double block_sum(double v, double* red) {
    // fixed-order tree reduction over the block (blockDim.x == BLOCK)
    const int t = threadIdx.x;
    red[t] = v;
    __syncthreads();
    for (int s = BLOCK / 2; s > 0; s >>= 1) {
        if (t < s) red[t] += red[t + s];
        __syncthreads();
    }
    double r = red[0];
    __syncthreads();
    return r;
}

// ---------------------------------------------------------------------------
// k_volume: one element per block.
//   mode 0: u given; mode 1: right-hand side (z = d, FP64 only); mode 2:
//   fused p = z + beta p (u is p, overwritten); mode 3: as mode 0, and the
//   weighted pointwise residual z_q of u is also written to pw [Ereal][m^3].
// Stages 2, 3 and their transposes never mix different lam1-indices a, so
// they run over slabs of SLAB a-values: the stage-2 arrays of one slab sit in
// LDS, and the transposed stage-2 results overwrite the stage-1 arrays of the
// slab's a-values (already consumed).  Stage 3, the pointwise residual and
// the transposed stage 3 run per (a, b) column in one thread.
// ---------------------------------------------------------------------------
template <int N, int M, class T>
struct VolCfg {
    static constexpr int fixed = 3 * M * N + N * N + N * N * N + 3 * N * N * M;   // elements of T
    static constexpr int per_a = 6 * N * M;
    // the largest slab whose LDS fits `bytes` (at least 1, at most M)
    static constexpr int slab_for(int bytes) {
        const int s = (bytes / (int)sizeof(T) - fixed) / per_a;
        return s < 1 ? 1 : (s > M ? M : s);
    }
    static constexpr int full_fits = (fixed + per_a * M) * (int)sizeof(T) <= 80 * 1024;
    // slab candidates: the whole element in LDS when it fits 80 KB, else the
    // largest slab under 155 KB (one workgroup per CU); the largest under
    // 78 KB (two workgroups per CU); and the first capped to one pass of the
    // stage-3 lanes when 4 lanes share a column (128 columns per pass)
    static constexpr int SLAB0 = full_fits ? M : slab_for(155 * 1024);
    static constexpr int SLAB1 = slab_for(78 * 1024);
    static constexpr int SLABQ = SLAB0 < 128 / M ? SLAB0 : (128 / M < 1 ? 1 : 128 / M);
    static constexpr int lds_bytes(int slab) { return (fixed + per_a * slab) * (int)sizeof(T); }
    // stage-1 values per slab (PS): u and the 1D operators fixed, per slab
    // the stage-1 and stage-2 values; the widest such slab under 155 KB that
    // four lanes per column cover in one pass (128 columns)
    static constexpr int fixed_ps = 3 * M * N + N * N + N * N * N;
    static constexpr int per_a_ps = 3 * N * N + 6 * N * M;
    static constexpr int SLABP_raw = (155 * 1024 / (int)sizeof(T) - fixed_ps) / per_a_ps;
    static constexpr int SLABP = SLABP_raw < 1 ? 1 : (SLABP_raw > 128 / M ? (128 / M < 1 ? 1 : 128 / M) : SLABP_raw);
    // a lane's share of a column's k-range with LPC lanes per column
    static constexpr int KL(int lpc) { return (N + lpc - 1) / lpc; }
    // stage-2 values of a column kept in registers while they fit
    static constexpr bool BREG(int lpc) { return (12 * KL(lpc) * (int)sizeof(T) / 4) <= 224; }
};

// value of another lane of the same quad: DPP quad_perm [1,0,3,2] (CTRL
// 0xB1, the other lane of an adjacent pair) or [2,3,0,1] (0x4E, the other pair)
template <int CTRL> __device__ inline float quad_swap(float x) {
    return __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, x), CTRL, 0xF, 0xF, false));
}
template <int CTRL> __device__ inline double quad_swap(double x) {
    const unsigned long long v = __builtin_bit_cast(unsigned long long, x);
    const int lo = __builtin_amdgcn_mov_dpp((int)(unsigned)(v & 0xffffffffull), CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_mov_dpp((int)(unsigned)(v >> 32), CTRL, 0xF, 0xF, false);
    return __builtin_bit_cast(double, ((unsigned long long)(unsigned)hi << 32) | (unsigned long long)(unsigned)lo);
}
// sum over the LPC (2 or 4) lanes of a column; every lane adds the same
// partials in the same pairing, so all hold the same bits
template <int LPC, class T> __device__ inline T lane_sum(T x) {
    if constexpr (LPC >= 2) x += quad_swap<0xB1>(x);
    if constexpr (LPC == 4) x += quad_swap<0x4E>(x);
    return x;
}

// threads of the element kernel: 256 with one lane per column, else 128 LPC
// (LPC 0: the matrix-core form of stage 3, 256 threads)
template <int LPC> constexpr int vol_block() { return LPC <= 1 ? 256 : 128 * LPC; }

// Stage 3, the pointwise residual and the transposed stage 3 of one lam1-slab
// on the float matrix cores (v_mfma_f32_16x16x4f32; lane l: operand A row
// l % 16 and k-column l / 16, operand B k-row l / 16 and column l % 16,
// result rows 4 (l / 16) + i, column l % 16).  The slab's columns (a, b) are
// taken b fastest in tiles of 16 per wavefront; per tile
//   F_al[c][col] = sum_k Mx_al[c][k] B_arr(al)[k][col]   (Mx in I, D1, D2)
// with c in row tiles of 16 and k in steps of 4, the residual z = sum_al
// C_al F_al (- d) and g_al = C_al z at each point in the lane that holds it,
// then T_arr[k][col] += sum_c Mx_al[c][k] g_al[c][col] with the c-steps
// ordered (row tile, result register), so that each lane's g values are
// already operand B of that step.  T overwrites the column's stage-2 values.
template <int N, int M, int SLAB, int VB>
__device__ __forceinline__ void stage3_mfma(int r, int mode, unsigned mask, bool general, bool zeroth,
                                            const float* C, const double* dv, double* pw, int a0, int na,
                                            const float* sI, const float* sD1, const float* sD2,
                                            float (*sB)[N * M * SLAB]) {
    typedef float f4 __attribute__((ext_vector_type(4)));
    constexpr int RT = (M + 15) / 16;       // row tiles of c
    constexpr int KST = (N + 3) / 4;        // steps of k
    constexpr int M2 = M * M, M3 = M * M * M;
    static_assert(N <= 16 && RT <= 2, "one row tile of k, at most two of c");
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int lc = lane & 15, lq = lane >> 4;
    const float* Mx[3] = {sI, sD1, sD2};
    // operand A of the forward products (c = 16 rt + lc, k = 4 s + lq) and of
    // the transposed ones (k = lc, c = 16 rt + 4 lq + i)
    float Af[3][RT][KST], At[3][RT][4];
#pragma unroll
    for (int mt = 0; mt < 3; ++mt)
#pragma unroll
        for (int rt = 0; rt < RT; ++rt) {
#pragma unroll
            for (int st = 0; st < KST; ++st) {
                const int c = 16 * rt + lc, k = 4 * st + lq;
                Af[mt][rt][st] = (c < M && k < N) ? Mx[mt][c * N + k] : 0.0f;
            }
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int c = 16 * rt + 4 * lq + i, k = lc;
                At[mt][rt][i] = (c < M && k < N) ? Mx[mt][c * N + k] : 0.0f;
            }
        }
    const int ncol = na * M;                 // the slab's columns, b fastest
    const int ntile = (ncol + 15) / 16;
    for (int tile = wv; tile < ntile; tile += VB / 64) {
        const int col = tile * 16 + lc;
        const bool cv = col < ncol;
        const int as = cv ? col / M : 0, b = cv ? col - as * M : 0;
        const int sbc = as + SLAB * b;           // the column in the stage-2 layout
        float Bf[6][KST];
#pragma unroll
        for (int arr = 0; arr < 6; ++arr)
#pragma unroll
            for (int st = 0; st < KST; ++st) {
                const int k = 4 * st + lq;
                Bf[arr][st] = (cv && k < N) ? sB[arr][sbc + SLAB * M * k] : 0.0f;
            }
        const int qcol = (a0 + as) + M * b;      // fine point (a, b, 0)
        const int ccol = (a0 + as) * M2 + b;     // its coefficients ([a][c][b] storage)
        float cf[RT][4];                          // one field's coefficients at this lane's points
        f4 z[RT];
#pragma unroll
        for (int rt = 0; rt < RT; ++rt) z[rt] = f4{0.0f, 0.0f, 0.0f, 0.0f};
        // (the field steps are macros so that every array index is a constant)
        // the coefficients of field AL at this lane's points (zero off the element)
#define SEM_LOAD_CF(AL)                                                                                   \
    _Pragma("unroll") for (int rt = 0; rt < RT; ++rt) _Pragma("unroll") for (int i = 0; i < 4; ++i) {      \
        const int c = 16 * rt + 4 * lq + i;                                                                 \
        cf[rt][i] = (cv && c < M && (mask >> (AL) & 1u)) ? C[(size_t)(AL) * M3 + ccol + M * c] : 0.0f;      \
    }
        // F_AL = Mx_MT B_ARR, added into z with its coefficients
#define SEM_FORWARD(AL, MT, ARR)                                                                           \
    {                                                                                                       \
        SEM_LOAD_CF(AL)                                                                                     \
        _Pragma("unroll") for (int rt = 0; rt < RT; ++rt) {                                                 \
            f4 acc = {0.0f, 0.0f, 0.0f, 0.0f};                                                              \
            _Pragma("unroll") for (int st = 0; st < KST; ++st)                                              \
                acc = __builtin_amdgcn_mfma_f32_16x16x4f32(Af[MT][rt][st], Bf[ARR][st], acc, 0, 0, 0);       \
            _Pragma("unroll") for (int i = 0; i < 4; ++i) z[rt][i] += cf[rt][i] * acc[i];                    \
        }                                                                                                   \
    }
        // T_ARR += Mx_MT^T g_AL, g_AL = C_AL z (the coefficients loaded again:
        // cache hits, fewer registers than keeping all fields)
#define SEM_TRANSPOSED(AL, MT, ARR)                                                                        \
    {                                                                                                       \
        SEM_LOAD_CF(AL)                                                                                     \
        _Pragma("unroll") for (int rt = 0; rt < RT; ++rt) _Pragma("unroll") for (int i = 0; i < 4; ++i)     \
            Tacc[ARR] = __builtin_amdgcn_mfma_f32_16x16x4f32(At[MT][rt][i], cf[rt][i] * z[rt][i], Tacc[ARR], \
                                                             0, 0, 0);                                      \
    }
        if (mode == 1) {
            // data: d at the points
#pragma unroll
            for (int rt = 0; rt < RT; ++rt)
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int c = 16 * rt + 4 * lq + i;
                    z[rt][i] = (cv && c < M) ? (float)dv[qcol + M2 * c] : 0.0f;
                }
        } else {
            SEM_FORWARD(0, 0, 5)
            SEM_FORWARD(1, 0, 2)
            SEM_FORWARD(2, 2, 0)
            if (general) {
                SEM_FORWARD(3, 0, 4)
                SEM_FORWARD(4, 1, 3)
                SEM_FORWARD(5, 1, 1)
                SEM_FORWARD(6, 0, 3)
                SEM_FORWARD(7, 0, 1)
                SEM_FORWARD(8, 1, 0)
            }
            if (zeroth) SEM_FORWARD(9, 0, 0)
        }
        if (mode == 3) {
#pragma unroll
            for (int rt = 0; rt < RT; ++rt)
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int c = 16 * rt + 4 * lq + i;
                    if (cv && c < M) pw[(size_t)r * M3 + qcol + M2 * c] = (double)z[rt][i];
                }
        }
        f4 Tacc[6];
#pragma unroll
        for (int arr = 0; arr < 6; ++arr) Tacc[arr] = f4{0.0f, 0.0f, 0.0f, 0.0f};
        SEM_TRANSPOSED(0, 0, 5)
        SEM_TRANSPOSED(1, 0, 2)
        SEM_TRANSPOSED(2, 2, 0)
        if (general) {
            SEM_TRANSPOSED(3, 0, 4)
            SEM_TRANSPOSED(4, 1, 3)
            SEM_TRANSPOSED(6, 0, 3)
            SEM_TRANSPOSED(5, 1, 1)
            SEM_TRANSPOSED(7, 0, 1)
            SEM_TRANSPOSED(8, 1, 0)
        }
        if (zeroth) {
            SEM_TRANSPOSED(9, 0, 0)
        }
#undef SEM_TRANSPOSED
#undef SEM_FORWARD
#undef SEM_LOAD_CF
        // T rows k = 4 lq + i of this lane's column back into the stage-2 slots
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int k = 4 * lq + i;
            if (cv && k < N)
#pragma unroll
                for (int arr = 0; arr < 6; ++arr) sB[arr][sbc + SLAB * M * k] = Tacc[arr][i];
        }
    }
}

// PS: stage-1 values per lam1-slab (recomputed for each slab from u, the
// transposed stage 1 summed slab after slab in registers) instead of for the
// whole element, for degrees whose whole-element stage-1 arrays leave no LDS
// for more than a one-point slab (FP64 from n = 11 on)
template <int N, int M, class T, int SLAB, int LPC, bool PS = false>
__global__ __launch_bounds__(vol_block<LPC>()) void k_volume(DevData D, const double* u, double* out, int mode,
                                                  const double* zf, double* pw, const Scalars* sc) {
    const int item = blockIdx.x / D.nrhs;
    const int rh = blockIdx.x - item * D.nrhs;
    const int e = D.sub_elem ? D.sub_elem[item] : item;
    if (rh) {
        bind_rhs(D, rh);
        const long long o = rh * D.vstride;
        u += o;
        out += o;
        if (zf) zf += o;
        if (pw) pw += o;
    }
    if (sc) sc += rh;
    if (sc && sc->done) return;
    using Cfg = VolCfg<N, M, T>;
    constexpr int VB = vol_block<LPC>();            // threads of this workgroup
    constexpr int N2 = N * N, N3 = N * N * N, M2 = M * M, M3 = M * M * M;
    const Dev<T>& P = dev_of<T>(D);
    __shared__ T sI[M * N], sD1[M * N], sD2[M * N], sDn[N * N];
    __shared__ T su[N3];
    constexpr int AW = PS ? SLAB : M;                 // lam1 extent held in sA
    __shared__ T sA[3][N2 * AW];
    __shared__ T sB[6][N * M * SLAB];
    const int tid = threadIdx.x;
    for (int i = tid; i < M * N; i += VB) { sI[i] = P.Im[i]; sD1[i] = P.D1m[i]; sD2[i] = P.D2m[i]; }
    for (int i = tid; i < N2; i += VB) sDn[i] = P.Dn[i];
    const int kind = D.kind[e];
    const int r = D.real_index[e];
    if (mode == 1 && kind != 0) return;
    if (kind == 0) {
        const size_t base = (size_t)r * N3;
        for (int i = tid; i < N3; i += VB) {
            double v = (mode == 1) ? 0.0 : u[base + i];
            if (mode == 2) {
                v = zf[base + i] + sc->beta * v;
                pw[base + i] = v;
            }
            su[i] = (T)v;
        }
    } else {
        const double* uc = u + D.nreal_dof + D.cdof[e];
        const int cd = D.cdir[e];
        for (int i = tid; i < N3; i += VB) {
            int idx3[3] = {i % N, (i / N) % N, i / N2};
            su[i] = (T)((kind == 1) ? uc[0] : uc[idx3[cd]]);
        }
    }
    __syncthreads();
    // ---- traces of u and grad_lam u on the active faces
    if (mode != 1) {
        for (int t = tid; t < 6 * 4 * N2; t += VB) {
            const int node = t % N2, c = (t / N2) % 4, f = t / (4 * N2);
            if (!D.slot_active[6 * e + f]) continue;
            const int d = f >> 1, s = f & 1;
            const int t0 = (d == 0) ? 1 : 0, t1 = (d == 2) ? 1 : 2;
            int idx[3];
            idx[d] = s ? N - 1 : 0;
            idx[t0] = node % N;
            idx[t1] = node / N;
            T v;
            if (c == 0) {
                v = su[idx[0] + N * idx[1] + N2 * idx[2]];
            } else {
                const int cd = c - 1;
                const int row = idx[cd];
                v = 0;
                for (int l = 0; l < N; ++l) {
                    int j3[3] = {idx[0], idx[1], idx[2]};
                    j3[cd] = l;
                    v += sDn[row * N + l] * su[j3[0] + N * j3[1] + N2 * j3[2]];
                }
            }
            P.trace[(((size_t)e * 6 + f) * 4 + c) * N2 + node] = v;
        }
    }
    if (kind != 0) return;
    // ---- stage 1: contractions along lam1 (I, D1, D2): A_al[k][j][a]
    for (int t = tid; t < (PS ? 0 : N2 * M); t += VB) {
        const int a = t % M, jk = t / M;
        const T* ur = su + N * jk;
        T a0 = 0, a1 = 0, a2 = 0;
#pragma unroll
        for (int i = 0; i < N; ++i) {
            const T v = ur[i];
            a0 += sI[a * N + i] * v;
            a1 += sD1[a * N + i] * v;
            a2 += sD2[a * N + i] * v;
        }
        sA[0][t] = a0; sA[1][t] = a1; sA[2][t] = a2;
    }
    __syncthreads();
    const unsigned mask = D.fmask[r];
    const bool general = (mask & 0x1F8u) != 0;         // fields u12 .. u3 present
    const bool zeroth = (mask >> 9 & 1u) != 0;        // the value u itself (c u)
    const T* C = P.coef + (size_t)r * VFIELDS * M3;
    const double* dv = D.dvol + (size_t)r * M3;
    constexpr int NACC = PS ? (N3 + VB - 1) / VB : 1;
    T acc[NACC];
#pragma unroll
    for (int q = 0; q < NACC; ++q) acc[q] = (T)0;
    for (int a0 = 0; a0 < M; a0 += SLAB) {
        const int na = (M - a0 < SLAB) ? (M - a0) : SLAB;
        if constexpr (PS) {
            // ---- stage 1 for the slab: A_al[k][j][as]
            for (int t = tid; t < N2 * SLAB; t += VB) {
                const int as = t % SLAB, jk = t / SLAB;
                if (as >= na) continue;
                const int a = a0 + as;
                const T* ur = su + N * jk;
                T v0 = 0, v1 = 0, v2 = 0;
#pragma unroll
                for (int i = 0; i < N; ++i) {
                    const T v = ur[i];
                    v0 += sI[a * N + i] * v;
                    v1 += sD1[a * N + i] * v;
                    v2 += sD2[a * N + i] * v;
                }
                sA[0][t] = v0; sA[1][t] = v1; sA[2][t] = v2;
            }
            __syncthreads();
        }
        // ---- stage 2 for the slab: B_be[k][b][as]
        for (int t = tid; t < SLAB * M * N; t += VB) {
            const int as = t % SLAB, b = (t / SLAB) % M, k = t / (SLAB * M);
            if (as >= na) continue;
            const int a = a0 + as;
            T b00 = 0, b01 = 0, b02 = 0, b10 = 0, b11 = 0, b20 = 0;
#pragma unroll
            for (int j = 0; j < N; ++j) {
                const int ia = PS ? as + SLAB * (j + N * k) : a + M * (j + N * k);
                const T x0 = sA[0][ia], x1 = sA[1][ia], x2 = sA[2][ia];
                const T i_ = sI[b * N + j], d1 = sD1[b * N + j], d2 = sD2[b * N + j];
                b00 += i_ * x0; b01 += d1 * x0; b02 += d2 * x0;
                b10 += i_ * x1; b11 += d1 * x1; b20 += i_ * x2;
            }
            sB[0][t] = b00; sB[1][t] = b01; sB[2][t] = b02; sB[3][t] = b10; sB[4][t] = b11; sB[5][t] = b20;
        }
        __syncthreads();
        if constexpr (LPC == 0) {
            static_assert(sizeof(T) == 4, "the matrix-core stage 3 is the float form");
            stage3_mfma<N, M, SLAB, VB>(r, mode, mask, general, zeroth, C, dv, pw, a0, na, sI, sD1, sD2, sB);
        } else {
        // ---- stage 3 + pointwise residual + transposed stage 3: LPC (1, 2 or
        // 4) adjacent lanes per column, lane h owning k = h KH .. (KH each, the
        // last lane what remains).  The lanes' parts of the residual z are
        // summed across the column once (lane_sum, the same pairing in every
        // lane), so every lane holds the same z.
            constexpr int KH = Cfg::KL(LPC);
            const int h = tid % LPC;
            const int kb = h * KH;                       // first k of this lane
            const int kn = max(0, min(KH, N - kb));      // number of own k
            for (int col = tid / LPC; col < SLAB * M; col += VB / LPC) {
                const int as = col % SLAB, b = col / SLAB;
                if (as >= na) continue;
                const int qcol = (a0 + as) + M * b;
                constexpr int BN = Cfg::BREG(LPC) ? KH : 1;
                T B00[BN], B01[BN], B02[BN], B10[BN], B11[BN], B20[BN];
                T T00[KH], T01[KH], T02[KH], T10[KH], T11[KH], T20[KH];
#pragma unroll
                for (int kk = 0; kk < KH; ++kk) {
                    if constexpr (Cfg::BREG(LPC)) {
                        const int ib = col + SLAB * M * min(kb + kk, N - 1);
                        B00[kk] = sB[0][ib]; B01[kk] = sB[1][ib]; B02[kk] = sB[2][ib];
                        B10[kk] = sB[3][ib]; B11[kk] = sB[4][ib]; B20[kk] = sB[5][ib];
                    }
                    T00[kk] = T01[kk] = T02[kk] = T10[kk] = T11[kk] = T20[kk] = 0;
                }
                auto Bv = [&](int arr, int kk) -> T {
                    if constexpr (Cfg::BREG(LPC)) {
                        switch (arr) {
                        case 0: return B00[kk]; case 1: return B01[kk]; case 2: return B02[kk];
                        case 3: return B10[kk]; case 4: return B11[kk]; default: return B20[kk];
                        }
                    } else {
                        return sB[arr][col + SLAB * M * min(kb + kk, N - 1)];
                    }
                };
                // coefficients stored [a][c][b]: this column's values for c are
                // M apart, and a wavefront's columns of one a are contiguous,
                // so each line is used up within a few steps of c
                const int ccol = (a0 + as) * M2 + b;
                T cfn[VFIELDS];
#pragma unroll
                for (int al = 0; al < VFIELDS; ++al) cfn[al] = (mask >> al & 1u) ? C[(size_t)al * M3 + ccol] : (T)0;
                for (int c = 0; c < M; ++c) {
                    const int q = qcol + M2 * c;
                    // this lane's entries of row c of I, D1, D2 (zero past its
                    // k-range): preloaded into registers, except in FP64 with one
                    // lane per column, where reading them from LDS where used keeps
                    // the register count (and so the occupancy) lower
                    constexpr bool PRE = !(sizeof(T) == 8 && LPC == 1);
                    const int crow = c * N;
                    T IrA[PRE ? KH : 1], D1A[PRE ? KH : 1], D2A[PRE ? KH : 1];
                    if constexpr (PRE) {
#pragma unroll
                        for (int kk = 0; kk < KH; ++kk) {
                            const int kx = crow + min(kb + kk, N - 1);
                            const bool own = kk < kn;
                            IrA[kk] = own ? sI[kx] : (T)0;
                            D1A[kk] = own ? sD1[kx] : (T)0;
                            D2A[kk] = own ? sD2[kx] : (T)0;
                        }
                    }
                    auto Ir = [&](int kk) -> T {
                        if constexpr (PRE) return IrA[kk];
                        else return kk < kn ? sI[crow + min(kb + kk, N - 1)] : (T)0;
                    };
                    auto D1r = [&](int kk) -> T {
                        if constexpr (PRE) return D1A[kk];
                        else return kk < kn ? sD1[crow + min(kb + kk, N - 1)] : (T)0;
                    };
                    auto D2r = [&](int kk) -> T {
                        if constexpr (PRE) return D2A[kk];
                        else return kk < kn ? sD2[crow + min(kb + kk, N - 1)] : (T)0;
                    };
                    T cf[VFIELDS];
#pragma unroll
                    for (int al = 0; al < VFIELDS; ++al) cf[al] = cfn[al];
                    if (c + 1 < M) {
#pragma unroll
                        for (int al = 0; al < VFIELDS; ++al)
                            cfn[al] = (mask >> al & 1u) ? C[(size_t)al * M3 + ccol + M * (c + 1)] : (T)0;
                    }
                    T z;
                    if (mode == 1) {
                        z = (T)dv[q];
                    } else {
                        // this lane's part of every field (its k-range); the
                        // coefficients are the column's, the same in every lane,
                        // so z = sum_al cf_al f_al is summed over the lanes once
                        T f[VFIELDS] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
#pragma unroll
                        for (int kk = 0; kk < KH; ++kk) {
                            f[0] += Ir(kk) * Bv(5, kk);
                            f[1] += Ir(kk) * Bv(2, kk);
                            f[2] += D2r(kk) * Bv(0, kk);
                        }
                        if (general) {
#pragma unroll
                            for (int kk = 0; kk < KH; ++kk) {
                                f[3] += Ir(kk) * Bv(4, kk);
                                f[4] += D1r(kk) * Bv(3, kk);
                                f[5] += D1r(kk) * Bv(1, kk);
                                f[6] += Ir(kk) * Bv(3, kk);
                                f[7] += Ir(kk) * Bv(1, kk);
                                f[8] += D1r(kk) * Bv(0, kk);
                            }
                        }
                        if (zeroth) {
#pragma unroll
                            for (int kk = 0; kk < KH; ++kk) f[9] += Ir(kk) * Bv(0, kk);
                        }
                        z = 0;
#pragma unroll
                        for (int al = 0; al < VFIELDS; ++al) z += cf[al] * f[al];
                        z = lane_sum<LPC>(z);
                    }
                    if (mode == 3 && h == 0) pw[(size_t)r * M3 + q] = (double)z;
                    T g[VFIELDS];
#pragma unroll
                    for (int al = 0; al < VFIELDS; ++al) g[al] = cf[al] * z;
#pragma unroll
                    for (int kk = 0; kk < KH; ++kk) {
                        T20[kk] += Ir(kk) * g[0];
                        T02[kk] += Ir(kk) * g[1];
                        T00[kk] += D2r(kk) * g[2];
                    }
                    if (general) {
#pragma unroll
                        for (int kk = 0; kk < KH; ++kk) {
                            T11[kk] += Ir(kk) * g[3];
                            T10[kk] += D1r(kk) * g[4] + Ir(kk) * g[6];
                            T01[kk] += D1r(kk) * g[5] + Ir(kk) * g[7];
                            T00[kk] += D1r(kk) * g[8];
                        }
                    }
                    if (zeroth) {
#pragma unroll
                        for (int kk = 0; kk < KH; ++kk) T00[kk] += Ir(kk) * g[9];
                    }
                }
#pragma unroll
                for (int kk = 0; kk < KH; ++kk) {
                    if (kk < kn) {
                        const int ib = col + SLAB * M * (kb + kk);
                        sB[0][ib] = T00[kk]; sB[1][ib] = T01[kk]; sB[2][ib] = T02[kk];
                        sB[3][ib] = T10[kk]; sB[4][ib] = T11[kk]; sB[5][ib] = T20[kk];
                    }
                }
            }
        }
        __syncthreads();
        // ---- transposed stage 2 for the slab, into sA at the slab's a-values
        for (int t = tid; t < SLAB * N * N; t += VB) {
            const int as = t % SLAB, j = (t / SLAB) % N, k = t / (SLAB * N);
            if (as >= na) continue;
            T a0v = 0, a1v = 0, a2v = 0;
            for (int b = 0; b < M; ++b) {
                const int ib = as + SLAB * (b + M * k);
                const T i_ = sI[b * N + j], d1 = sD1[b * N + j], d2 = sD2[b * N + j];
                a0v += i_ * sB[0][ib] + d1 * sB[1][ib] + d2 * sB[2][ib];
                a1v += i_ * sB[3][ib] + d1 * sB[4][ib];
                a2v += i_ * sB[5][ib];
            }
            const int ia = PS ? as + SLAB * (j + N * k) : (a0 + as) + M * (j + N * k);
            sA[0][ia] = a0v; sA[1][ia] = a1v; sA[2][ia] = a2v;
        }
        __syncthreads();
        if constexpr (PS) {
            // ---- transposed stage 1, this slab's part
#pragma unroll
            for (int q = 0; q < NACC; ++q) {
                const int t = tid + q * VB;
                if (t < N3) {
                    const int i = t % N, jk = t / N;
                    T v = 0;
                    for (int as = 0; as < na; ++as) {
                        const int a = a0 + as, ia = as + SLAB * jk;
                        v += sI[a * N + i] * sA[0][ia] + sD1[a * N + i] * sA[1][ia] + sD2[a * N + i] * sA[2][ia];
                    }
                    acc[q] += v;
                }
            }
            __syncthreads();
        }
    }
    double* o = out + (size_t)r * N3;
    if constexpr (PS) {
#pragma unroll
        for (int q = 0; q < NACC; ++q) {
            const int t = tid + q * VB;
            if (t < N3) o[t] = (double)acc[q];
        }
        return;
    }
    // ---- transposed stage 1
    for (int t = tid; t < N3; t += VB) {
        const int i = t % N, jk = t / N;
        T v = 0;
        for (int a = 0; a < M; ++a) {
            const int ia = a + M * jk;
            v += sI[a * N + i] * sA[0][ia] + sD1[a * N + i] * sA[1][ia] + sD2[a * N + i] * sA[2][ia];
        }
        o[t] = (double)v;
    }
}

// ---------------------------------------------------------------------------
// k_face: one face term per block.  mode 0: homogeneous apply; mode 1: data
// (FP64 only).
// ---------------------------------------------------------------------------
// threads of the face kernel: one per face point, whole wavefronts, at least BLOCK
template <int M> constexpr int face_block() {
    constexpr int t = (M * M + 63) / 64 * 64;
    return t < BLOCK ? BLOCK : (t > 1024 ? 1024 : t);
}

template <int N, int M, class T>
__global__ __launch_bounds__(face_block<M>()) void k_face(DevData D, int mode, const Scalars* sc) {
    const int item = blockIdx.x / D.nrhs;
    const int rh = blockIdx.x - item * D.nrhs;
    const int fidx = D.sub_face ? D.sub_face[item] : item;
    bind_rhs(D, rh);
    if (sc) sc += rh;
    if (sc && sc->done) return;
    constexpr int N2 = N * N, M2 = M * M;
    constexpr int FB = face_block<M>();
    const Dev<T>& Pd = dev_of<T>(D);
    __shared__ T sI[M * N], sK[M * M], sw[M];
    __shared__ T sT[2][4][M2];
    __shared__ T sX[2][4][M * N];
    __shared__ T sQ[4][M2];
    __shared__ int sInt[8];
    __shared__ T sWt[4][3];
    const int tid = threadIdx.x;
    if (tid < 8) sInt[tid] = D.face_int[8 * fidx + tid];
    if (tid < 12) sWt[tid / 3][tid % 3] = Pd.face_w[12 * fidx + tid];
    for (int i = tid; i < M * N; i += FB) sI[i] = Pd.Im[i];
    for (int i = tid; i < M * M; i += FB) sK[i] = Pd.K[i];
    if (tid < M) sw[tid] = Pd.wm[tid];
    __syncthreads();
    const int eA = sInt[0], fA = sInt[1], eB = sInt[2], fB = sInt[3], orient = sInt[4], nq = sInt[5];
    const int pmA = sInt[6], pmB = sInt[7];
    const bool interior = eB >= 0;
    T* resA = Pd.slotres + ((size_t)eA * 6 + fA) * 4 * N2;
    T* resB = interior ? Pd.slotres + ((size_t)eB * 6 + fB) * 4 * N2 : nullptr;
    if (mode == 1 && interior) {
        for (int i = tid; i < 4 * N2; i += FB) { resA[i] = 0; resB[i] = 0; }
        return;
    }
    const long long offA = D.face_off[3 * fidx], offB = D.face_off[3 * fidx + 1], offG = D.face_off[3 * fidx + 2];
    const T* PA = Pd.pcoef + offA;
    const T* PB = interior ? Pd.pcoef + offB : nullptr;
    const int nsides = interior ? 2 : 1;
    // this thread's face point (one per thread) and its coefficients of both
    // sides, loaded once here so that the loads overlap the interpolation and
    // serve both the forward and the transposed weighting
    constexpr bool CREG = FB >= M2;
    T ca[CREG ? 4 : 1][4], cb[CREG ? 4 : 1][4];
    if constexpr (CREG) {
        const int p = tid < M2 ? tid : M2 - 1;
#pragma unroll
        for (int k = 0; k < 4; ++k)
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                ca[k][c] = cb[k][c] = (T)0;
                if (k < nq) {
                    ca[k][c] = pmA ? PA[(size_t)(k * 4 + c) * M2 + p] : PA[k * 4 + c];
                    if (interior) cb[k][c] = pmB ? PB[(size_t)(k * 4 + c) * M2 + p] : PB[k * 4 + c];
                }
            }
    }
    auto coefA = [&](int k, int c, int p) -> T {
        if constexpr (CREG) return ca[k][c];
        else return pmA ? PA[(size_t)(k * 4 + c) * M2 + p] : PA[k * 4 + c];
    };
    auto coefB = [&](int k, int c, int p) -> T {
        if constexpr (CREG) return cb[k][c];
        else return pmB ? PB[(size_t)(k * 4 + c) * M2 + p] : PB[k * 4 + c];
    };
    if (mode == 0) {
        // the traces of both sides into LDS (sT holds them until the second
        // interpolation overwrites it)
        for (int t = tid; t < nsides * 4 * N2; t += FB) {
            const int i = t % N2, c = (t / N2) % 4, s = t / (4 * N2);
            sT[s][c][i] = Pd.trace[(((size_t)(s ? eB : eA) * 6 + (s ? fB : fA)) * 4 + c) * N2 + i];
        }
        __syncthreads();
        // interpolate the traces n x n -> m x m (both directions)
        for (int t = tid; t < nsides * 4 * M * N; t += FB) {
            const int a = t % M, j = (t / M) % N, c = (t / (M * N)) % 4, s = t / (4 * M * N);
            const T* tr = sT[s][c];
            T v = 0;
#pragma unroll
            for (int i = 0; i < N; ++i) v += sI[a * N + i] * tr[i + N * j];
            sX[s][c][a + M * j] = v;
        }
        __syncthreads();
        for (int t = tid; t < nsides * 4 * M2; t += FB) {
            const int a = t % M, b = (t / M) % M, c = (t / M2) % 4, s = t / (4 * M2);
            T v = 0;
#pragma unroll
            for (int j = 0; j < N; ++j) v += sI[b * N + j] * sX[s][c][a + M * j];
            sT[s][c][a + M * b] = v;
        }
        __syncthreads();
    }
    // quantities at A's face points
    for (int p = tid; p < M2; p += FB) {
        const int a = p % M, b = p / M;
        int ia = a, ib = b;
        if (orient & 1) { ia = b; ib = a; }
        if (orient & 2) ia = M - 1 - ia;
        if (orient & 4) ib = M - 1 - ib;
        const int pB = ia + M * ib;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            if (k >= nq) break;
            T qv;
            if (mode == 1) {
                qv = (T)D.gdata[offG + (size_t)k * M2 + p];
            } else {
                qv = 0;
#pragma unroll
                for (int c = 0; c < 4; ++c) {
                    qv += coefA(k, c, p) * sT[0][c][p];
                    if (interior) qv -= coefB(k, c, p) * sT[1][c][pB];
                }
            }
            sQ[k][p] = qv;
        }
    }
    __syncthreads();
    // face norms: W = alpha Om x Om Q + beta (K x Om) Q + gamma (Om x K) Q
    T Wv[4][(M2 + FB - 1) / FB];
    {
        int slot = 0;
        for (int p = tid; p < M2; p += FB, ++slot) {
            const int a = p % M, b = p / M;
            for (int k = 0; k < nq; ++k) {
                const T al = sWt[k][0], be = sWt[k][1], ga = sWt[k][2];
                T v = al * sw[a] * sw[b] * sQ[k][p];
                if (be != (T)0) {
                    T acc = 0;
                    for (int a2 = 0; a2 < M; ++a2) acc += sK[a * M + a2] * sQ[k][a2 + M * b];
                    v += be * sw[b] * acc;
                }
                if (ga != (T)0) {
                    T acc = 0;
                    for (int b2 = 0; b2 < M; ++b2) acc += sK[b * M + b2] * sQ[k][a + M * b2];
                    v += ga * sw[a] * acc;
                }
                Wv[k][slot] = v;
            }
        }
    }
    __syncthreads();
    // back to trace components (reuse sT)
    {
        int slot = 0;
        for (int p = tid; p < M2; p += FB, ++slot) {
            const int a = p % M, b = p / M;
            int ia = a, ib = b;
            if (orient & 1) { ia = b; ib = a; }
            if (orient & 2) ia = M - 1 - ia;
            if (orient & 4) ib = M - 1 - ib;
            const int pB = ia + M * ib;
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                T va = 0, vb = 0;
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    if (k >= nq) break;
                    va += coefA(k, c, p) * Wv[k][slot];
                    if (interior) vb -= coefB(k, c, p) * Wv[k][slot];
                }
                sT[0][c][p] = va;
                if (interior) sT[1][c][pB] = vb;
            }
        }
    }
    __syncthreads();
    // transposed interpolation m x m -> n x n
    for (int t = tid; t < nsides * 4 * M * N; t += FB) {
        const int a = t % M, j = (t / M) % N, c = (t / (M * N)) % 4, s = t / (4 * M * N);
        T v = 0;
        for (int b = 0; b < M; ++b) v += sI[b * N + j] * sT[s][c][a + M * b];
        sX[s][c][a + M * j] = v;
    }
    __syncthreads();
    for (int t = tid; t < nsides * 4 * N2; t += FB) {
        const int i = t % N, j = (t / N) % N, c = (t / N2) % 4, s = t / (4 * N2);
        T v = 0;
        for (int a = 0; a < M; ++a) v += sI[a * N + i] * sX[s][c][a + M * j];
        (s ? resB : resA)[c * N2 + i + N * j] = v;
    }
}

// ---------------------------------------------------------------------------
// k_gather: q_e += sum over active faces of the transposed traces; partial
// p^T q per element (pdot != nullptr); corner partial sums per corner element.
// k_corner_q: corner q values; k_fin_gather (one block): total p^T q, alpha.
// Reductions finish in later kernels: the kernel boundary makes the partials
// visible without device-scope fences in every block.
// ---------------------------------------------------------------------------
template <int N, class T>
__global__ __launch_bounds__(BLOCK) void k_gather(DevData D, double* q, const double* pdot, const Scalars* sc,
                                                  int rhs) {
    const int item = blockIdx.x / D.nrhs;
    const int rh = blockIdx.x - item * D.nrhs;
    const int e = D.sub_elem ? D.sub_elem[item] : item;
    if (rh) {
        bind_rhs(D, rh);
        q += rh * D.vstride;
        if (pdot) pdot += rh * D.vstride;
    }
    if (sc) sc += rh;
    if (sc && sc->done) return;
    constexpr int N2 = N * N, N3 = N * N * N;
    __shared__ double sDn[N * N];
    __shared__ double sres[6][4 * N2];
    __shared__ double sr[N3];
    __shared__ double red[BLOCK];
    __shared__ unsigned char act[6];
    const int tid = threadIdx.x;
    const int kind = D.kind[e];
    const int r = D.real_index[e];
    if (rhs && kind != 0) {
        if (tid == 0) D.part_a[e] = 0.0;
        return;
    }
    for (int i = tid; i < N2; i += BLOCK) sDn[i] = D.Dn[i];
    if (tid < 6) act[tid] = D.slot_active[6 * e + tid];
    __syncthreads();
    // stage the face results of this element (coalesced)
    const T* res0 = dev_of<T>(D).slotres + (size_t)e * 6 * 4 * N2;
    for (int i = tid; i < 6 * 4 * N2; i += BLOCK) {
        const int f = i / (4 * N2);
        sres[f][i - f * 4 * N2] = act[f] ? (double)res0[i] : 0.0;
    }
    __syncthreads();
    double dot = 0.0;
    for (int t = tid; t < N3; t += BLOCK) {
        int idx[3] = {t % N, (t / N) % N, t / N2};
        double v = (kind == 0) ? q[(size_t)r * N3 + t] : 0.0;
#pragma unroll
        for (int f = 0; f < 6; ++f) {
            if (!act[f]) continue;
            const int d = f >> 1, s = f & 1;
            const int t0 = (d == 0) ? 1 : 0, t1 = (d == 2) ? 1 : 2;
            const int ld = s ? N - 1 : 0;
            const double* res = sres[f];
            const int fn = idx[t0] + N * idx[t1];
            // normal derivative: every node on the normal line
            v += sDn[ld * N + idx[d]] * res[(1 + d) * N2 + fn];
            if (idx[d] == ld) {
                v += res[fn];
                for (int i0 = 0; i0 < N; ++i0)
                    v += sDn[i0 * N + idx[t0]] * res[(1 + t0) * N2 + i0 + N * idx[t1]];
                for (int i1 = 0; i1 < N; ++i1)
                    v += sDn[i1 * N + idx[t1]] * res[(1 + t1) * N2 + idx[t0] + N * i1];
            }
        }
        if (kind == 0) {
            q[(size_t)r * N3 + t] = v;
            if (pdot) dot += pdot[(size_t)r * N3 + t] * v;
        } else {
            sr[t] = v;
        }
    }
    if (kind != 0) {
        __syncthreads();
        const int v_ = D.virt_index[e];
        if (kind == 1) {
            double sum = 0;
            for (int t = tid; t < N3; t += BLOCK) sum += sr[t];
            sum = block_sum(sum, red);
            if (tid == 0) D.cpart[(size_t)v_ * N] = sum;
        } else {
            const int cd = D.cdir[e];
            for (int l = 0; l < N; ++l) {
                double sum = 0;
                for (int t = tid; t < N2; t += BLOCK) {
                    int a = t % N, b = t / N;
                    int idx3[3];
                    idx3[cd] = l;
                    idx3[cd == 0 ? 1 : 0] = a;
                    idx3[cd == 2 ? 1 : 2] = b;
                    sum += sr[idx3[0] + N * idx3[1] + N2 * idx3[2]];
                }
                sum = block_sum(sum, red);
                if (tid == 0) D.cpart[(size_t)v_ * N + l] = sum;
            }
        }
    }
    dot = block_sum(dot, red);
    if (tid == 0) D.part_a[e] = dot;
}

// corner unknowns: one wavefront per unknown, lanes stride its segment of
// corner element partials, fixed-order butterfly sum; q = the sum, and the
// corner part of p^T q per unknown into the corner scratch
__global__ __launch_bounds__(BLOCK) void k_corner_q(DevData D, double* q, const double* pdot, const Scalars* sc,
                                                    int rhs) {
    constexpr int WPB = BLOCK / 64;
    const int nb = (D.ncd + WPB - 1) / WPB;
    const int blk = blockIdx.x / D.nrhs;
    const int rh = blockIdx.x - blk * D.nrhs;
    if (rh) {
        bind_rhs(D, rh);
        q += rh * D.vstride;
        if (pdot) pdot += rh * D.vstride;
    }
    if (sc) sc += rh;
    if ((sc && sc->done) || blk >= nb) return;
    const int lane = threadIdx.x & 63;
    const int c = blk * WPB + (threadIdx.x >> 6);
    if (c >= D.ncd) return;
    double s = 0;
    if (!rhs)   // corner elements carry no data terms
        for (int t = D.cptr[c] + lane; t < D.cptr[c + 1]; t += 64) s += D.cpart[D.cidx[t]];
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
    if (lane == 0) {
        q[D.nreal_dof + c] = s;
        D.cscratch[c] = pdot ? pdot[D.nreal_dof + c] * s : 0.0;
    }
}

// total p^T q (element partials, then corner partials, fixed order) and alpha
__global__ __launch_bounds__(BLOCK) void k_fin_gather(DevData D, Scalars* sc, int pcg) {
    const int rh = blockIdx.x;
    bind_rhs(D, rh);
    if (sc) sc += rh;
    if (sc && sc->done) return;
    if (!pcg) return;
    __shared__ double red[BLOCK];
    const int tid = threadIdx.x;
    double tot = 0.0;
    for (int i = tid; i < D.E; i += BLOCK) tot += D.part_a[i];
    for (int c = tid; c < D.ncd; c += BLOCK) tot += D.cscratch[c];
    tot = block_sum(tot, red);
    if (tid == 0) {
        sc->pq = tot;
        if (!(tot == tot) || tot > 1e300 || tot < -1e300) { sc->status = -6; sc->done = 1; }
        else if (tot <= 0.0) { sc->status = -5; sc->done = 1; }
        else sc->alpha = sc->rho / tot;
    }
}

// ---------------------------------------------------------------------------
// k_update: blocks 0..Ereal-1 elements, block Ereal the corner DOFs.
//   mode 0 INIT: r = b - q, z = W^-1 r, p = z, partials r.z, r.r, b.b
//   mode 1 ITER: u += alpha p, r -= alpha q, z = W^-1 r, partials
//   mode 2 PREC: z = W^-1 r only
//   mode 3 REPL: r = b - q (q = X u in FP64: residual replacement), z = W^-1 r,
//                partials; finished like ITER
// k_fin_update (one block): r^T z, r^T r, beta, stopping test, corner p.
// ---------------------------------------------------------------------------
// Element-block preconditioner: z = G^T (G r) with G = L^{-1}, L the
// Cholesky factor of the element's diagonal block of X.  G is lower
// triangular and stored twice: by columns (column j holds rows j..n3-1,
// starting at j n3 - j (j - 1) / 2) for y = G r, and by rows (row i holds
// columns 0..i, starting at i (i + 1) / 2) for z = G^T y.  Both sweeps are
// "scalar times contiguous vector" updates: a thread owns output indices,
// consecutive threads read consecutive entries, and U sweep steps are loaded
// before they are used so that enough loads are in flight.  Products
// accumulate in double.
__device__ inline long long packed_col(long long j, long long n3) { return j * n3 - j * (j - 1) / 2; }
__device__ inline long long packed_row(long long i) { return i * (i + 1) / 2; }

template <int N3, class GT>
__device__ void block_apply(const GT* Gc, const GT* Gr, const double* sr, double* sy, double* sz) {
    // wavefront w sweeps the steps k = w, w + NW, ... (a quarter of the
    // columns, then of the rows); each lane owns outputs lane + 64 s.  The NW
    // partial vectors are added in wavefront order through LDS.
    constexpr int NW = BLOCK / 64;
    constexpr int RL = (N3 + 63) / 64;
    constexpr int U = (16 / RL) > 1 ? 16 / RL : 1;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    double acc[RL];
    // ---- y = G r: step k adds column k (rows k..N3-1) times r_k
#pragma unroll
    for (int s = 0; s < RL; ++s) acc[s] = 0.0;
#pragma unroll 1
    for (int k0 = w; k0 < N3; k0 += NW * U) {
        GT g[U][RL];
        double rk[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int k = k0 + NW * u;
            const int kc = min(k, N3 - 1);        // steps past the end load in bounds, weigh zero
            rk[u] = (k < N3) ? sr[kc] : 0.0;
            const GT* col = Gc + packed_col(kc, N3) - kc;
#pragma unroll
            for (int s = 0; s < RL; ++s) {
                const int i = lane + 64 * s;
                const GT v = col[min(max(i, kc), N3 - 1)];
                g[u][s] = (i >= kc && i < N3) ? v : (GT)0;
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
            for (int s = 0; s < RL; ++s) acc[s] += (double)g[u][s] * rk[u];
    }
    for (int ww = 0; ww < NW; ++ww) {
        if (w == ww) {
#pragma unroll
            for (int s = 0; s < RL; ++s) {
                const int i = lane + 64 * s;
                if (i < N3) sy[i] = (ww == 0 ? 0.0 : sy[i]) + acc[s];
            }
        }
        __syncthreads();
    }
    // ---- z = G^T y: step k adds row k (columns 0..k) times y_k
#pragma unroll
    for (int s = 0; s < RL; ++s) acc[s] = 0.0;
#pragma unroll 1
    for (int k0 = w; k0 < N3; k0 += NW * U) {
        GT g[U][RL];
        double yk[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int k = k0 + NW * u;
            const int kc = min(k, N3 - 1);
            yk[u] = (k < N3) ? sy[kc] : 0.0;
            const GT* row = Gr + packed_row(kc);
#pragma unroll
            for (int s = 0; s < RL; ++s) {
                const int j = lane + 64 * s;
                const GT v = row[min(j, kc)];
                g[u][s] = (j <= kc) ? v : (GT)0;
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
            for (int s = 0; s < RL; ++s) acc[s] += (double)g[u][s] * yk[u];
    }
    for (int ww = 0; ww < NW; ++ww) {
        if (w == ww) {
#pragma unroll
            for (int s = 0; s < RL; ++s) {
                const int j = lane + 64 * s;
                if (j < N3) sz[j] = (ww == 0 ? 0.0 : sz[j]) + acc[s];
            }
        }
        __syncthreads();
    }
}

// Element-block inverse applied to the elements of one task at once on the
// FP64 matrix cores: Z = B [r_1 .. r_16] for up to 16 elements sharing the
// stored block B (full symmetric, column k at k ld, ld = n3 + 3 rounded up to
// a multiple of 32: row stripes start on 128-byte lines, and the last
// four-row load of a column stays inside it).  One v_mfma_f64_16x16x4 takes a
// 16 x 4 tile of B (rows x columns) as operand A and the 4 x 16 tile of
// residuals (columns x elements) as operand B.  A wavefront owns 64 rows, as 64 / (16 V) super-tiles of 16 V rows: each
// lane loads V consecutive rows of one column in one 16-byte load (a double2,
// V = 2, or a float4, V = 4), whose entries feed V tiles (rows congruent to
// h mod V).  The residuals pass through LDS in chunks of KC columns.
typedef double dbl4 __attribute__((ext_vector_type(4)));

template <int N3> struct MfmaSplit {
    // wavefronts per workgroup (the kernel takes 2..4); 4 measured fastest
    // at N = W = 10, also against 3, whose row parts pad n^3 less (13 idle
    // rows instead of 205: 2 % slower)
    static constexpr int NW = 4;
    static constexpr int RP = NW * 64;                 // rows per part
    static constexpr int P = (N3 + RP - 1) / RP;       // row parts per task
    static constexpr int KC = 64;                      // columns per LDS chunk
    static constexpr int NCH = (N3 + KC - 1) / KC;
    static constexpr int KS = KC / 4;                  // 4-column steps per chunk
};

// elements per task: the 16 columns of the matrix-core tile
template <int N3> constexpr int group_cap() { return 16; }

// corner unknowns: the same product with the dense corner block (one block)
template <class GT>
__device__ void corner_block_apply(const GT* G, int nc, const double* r, double* y, double* z) {
    const int tid = threadIdx.x, nt = blockDim.x;
    for (int i = tid; i < nc; i += nt) {
        double acc = 0.0;
        for (int j = 0; j <= i; ++j) acc += (double)G[packed_col(j, nc) + i - j] * r[j];
        y[i] = acc;
    }
    __syncthreads();
    for (int j = tid; j < nc; j += nt) {
        const GT* col = G + packed_col(j, nc) - j;
        double acc = 0.0;
        for (int i = j; i < nc; ++i) acc += (double)col[i] * y[i];
        z[j] = acc;
    }
    __syncthreads();
}

// local index t = i + N j + N^2 k of an element with the lambda axes of the
// bits of c reversed (the map between an element and its stored block)
template <int N>
__device__ inline int flip_index(int t, int c) {
    if (!c) return t;
    int i = t % N, j = (t / N) % N, k = t / (N * N);
    if (c & 1) i = N - 1 - i;
    if (c & 2) j = N - 1 - j;
    if (c & 4) k = N - 1 - k;
    return i + N * (j + N * k);
}

template <int N>
__global__ __launch_bounds__(BLOCK) void k_update(DevData D, int mode, double* u, double* r, double* z,
                                                  double* p, const double* q, const double* b, const Scalars* sc) {
    const int blk0 = blockIdx.x / D.nrhs;
    const int rh = blockIdx.x - blk0 * D.nrhs;
    if (rh) {
        bind_rhs(D, rh);
        const long long o = rh * D.vstride;
        if (u) u += o;
        if (r) r += o;
        if (z) z += o;
        if (p) p += o;
        if (q) q += o;
        if (b) b += o;
    }
    if (sc) sc += rh;
    if (sc && sc->done && mode != 2) return;
    // element blocks: elements that share a stored block run one after another
    const int blk = (D.pk != 0 && D.uorder && blk0 < D.Ereal) ? D.uorder[blk0] : blk0;
    constexpr int N2 = N * N, N3 = N * N * N;
    __shared__ double sP[3][N * N];
    __shared__ double sL[3][N];
    __shared__ double s0[N3], s1[N3], s2[N3];
    __shared__ double red[BLOCK];
    const int tid = threadIdx.x;
    const double alpha = (mode == 1) ? sc->alpha : 0.0;
    const int pk = D.pk;
    double prz = 0, prr = 0, pbb = 0;
    if (blk < D.Ereal) {
        const size_t base = (size_t)blk * N3;
        const int fl = (pk != 0 && D.bflip) ? D.bflip[blk] : 0;
        if (pk == 0) {
            for (int d = 0; d < 3; ++d) {
                const int bi = D.pidx[3 * blk + d];
                for (int i = tid; i < N2; i += BLOCK) sP[d][i] = D.pbasis[(size_t)bi * N2 + i];
                if (tid < N) sL[d][tid] = D.peig[(size_t)bi * N + tid];
            }
        }
        for (int t = tid; t < N3; t += BLOCK) {
            double rv;
            if (mode == 0 || mode == 3) {
                rv = b[base + t] - q[base + t];
                r[base + t] = rv;
                if (mode == 0) pbb += b[base + t] * b[base + t];
            } else if (mode == 1) { u[base + t] += alpha * p[base + t]; rv = r[base + t] - alpha * q[base + t]; r[base + t] = rv; }
            else rv = r[base + t];
            s0[t] = rv;
        }
        __syncthreads();
        if (pk != 0) {
            // exact element block, form 2 (the forms 1 and 3 run in
            // k_update_mfma): two sweeps over the float factor G = L^-1 of the
            // stored block, z into s2; an element stored as a reversal of its
            // block applies it to the reversed residual (s0 takes r[f(t)])
            const int bi = D.bidx[blk];
            if (fl) {
                for (int t = tid; t < N3; t += BLOCK) s1[t] = s0[flip_index<N>(t, fl)];
                __syncthreads();
                for (int t = tid; t < N3; t += BLOCK) s0[t] = s1[t];
                __syncthreads();
            }
            const size_t goff = (size_t)bi * ((size_t)N3 * (N3 + 1) / 2);
            block_apply<N3, float>(D.G32 + goff, D.G32r + goff, s0, s1, s2);
        } else {
            // separable form (Sec. 5.2): t = (Phi3^T x Phi2^T x Phi1^T) r,
            // scaled by the inverse eigenvalue sums, z = (Phi3 x Phi2 x Phi1) t
            for (int t = tid; t < N3; t += BLOCK) {
                const int a = t % N, jk = t / N;
                double v = 0;
#pragma unroll
                for (int i = 0; i < N; ++i) v += sP[0][i * N + a] * s0[i + N * jk];
                s1[t] = v;
            }
            __syncthreads();
            for (int t = tid; t < N3; t += BLOCK) {
                const int a = t % N, bb = (t / N) % N, k = t / N2;
                double v = 0;
#pragma unroll
                for (int j = 0; j < N; ++j) v += sP[1][j * N + bb] * s1[a + N * (j + N * k)];
                s2[t] = v;
            }
            __syncthreads();
            const double inv_s = 1.0 / D.pscale[blk];
            for (int t = tid; t < N3; t += BLOCK) {
                const int a = t % N, bb = (t / N) % N, c = t / N2;
                double v = 0;
#pragma unroll
                for (int k = 0; k < N; ++k) v += sP[2][k * N + c] * s2[a + N * (bb + N * k)];
                s1[t] = v * inv_s / (sL[0][a] + sL[1][bb] + sL[2][c] + 1.0);
            }
            __syncthreads();
            for (int t = tid; t < N3; t += BLOCK) {
                const int a = t % N, bb = (t / N) % N, k = t / N2;
                double v = 0;
#pragma unroll
                for (int c = 0; c < N; ++c) v += sP[2][k * N + c] * s1[a + N * (bb + N * c)];
                s2[t] = v;
            }
            __syncthreads();
            for (int t = tid; t < N3; t += BLOCK) {
                const int a = t % N, j = (t / N) % N, k = t / N2;
                double v = 0;
#pragma unroll
                for (int bb = 0; bb < N; ++bb) v += sP[1][j * N + bb] * s2[a + N * (bb + N * k)];
                s1[t] = v;
            }
            __syncthreads();
            for (int t = tid; t < N3; t += BLOCK) {
                const int i = t % N, jk = t / N;
                double v = 0;
#pragma unroll
                for (int a = 0; a < N; ++a) v += sP[0][i * N + a] * s1[a + N * jk];
                s2[t] = v;
            }
            __syncthreads();
        }
        for (int t = tid; t < N3; t += BLOCK) {
            const int tp = flip_index<N>(t, fl);     // z[t] = (B r_f)[f(t)]
            const double v = s2[tp];
            z[base + t] = v;
            if (mode == 0) p[base + t] = v;
            const double rv = s0[tp];
            prz += rv * v;
            prr += rv * rv;
        }
    } else {
        const size_t c0 = D.nreal_dof;
        for (int c = tid; c < D.ncd; c += BLOCK) {
            const size_t i = c0 + c;
            double rv;
            if (mode == 0 || mode == 3) {
                rv = b[i] - q[i];
                r[i] = rv;
                if (mode == 0) pbb += b[i] * b[i];
            } else if (mode == 1) { u[i] += alpha * p[i]; rv = r[i] - alpha * q[i]; r[i] = rv; }
            else rv = r[i];
            if (pk == 0) {
                const double zv = D.cinv[c] * rv;
                z[i] = zv;
                if (mode == 0) p[i] = zv;
                prz += rv * zv;
            }
            prr += rv * rv;
        }
        if (pk != 0 && D.ncd > 0) {
            __syncthreads();   // r of the corner unknowns is complete (this block wrote it)
            if (pk == 1) corner_block_apply<double>(D.Gc64, D.ncd, r + c0, D.cscratch, z + c0);
            else corner_block_apply<float>(D.Gc32, D.ncd, r + c0, D.cscratch, z + c0);
            for (int c = tid; c < D.ncd; c += BLOCK) {
                const double zv = z[c0 + c];
                if (mode == 0) p[c0 + c] = zv;
                prz += r[c0 + c] * zv;
            }
        }
    }
    if (mode == 2) return;
    prz = block_sum(prz, red);
    prr = block_sum(prr, red);
    pbb = block_sum(pbb, red);
    if (tid == 0) { D.part_a[blk] = prz; D.part_b[blk] = prr; D.part_c[blk] = pbb; }
}

// The CG vector step ahead of the row-split update: r = b - q (modes 0, 3) or
// u += alpha p, r -= alpha q (mode 1), over every unknown.
__global__ __launch_bounds__(BLOCK) void k_cg_vec(DevData D, int mode, double* u, double* r, const double* p,
                                                  const double* q, const double* b, const Scalars* sc) {
    const int rh = blockIdx.y;
    const long long o = rh * D.vstride;
    sc += rh;
    if (sc->done) return;
    const double alpha = sc->alpha;
    const long long n = D.ndof;
    for (long long i = (long long)blockIdx.x * BLOCK + threadIdx.x; i < n; i += (long long)gridDim.x * BLOCK) {
        if (mode == 1) {
            u[o + i] += alpha * p[o + i];
            r[o + i] = r[o + i] - alpha * q[o + i];
        } else {
            r[o + i] = b[o + i] - q[o + i];
        }
    }
}

// Element-block update for the forms 1 (FP64 inverse) and 3 (float inverse),
// after k_cg_vec: z = B r (and p = z in mode 0) for the rows of one part of
// one task (D.task_*: up to 16 elements sharing a stored block); workgroup
// index = task P + part, the last one takes the corner unknowns.  Partial
// sums r.z, r.r, b.b (mode 0) of the workgroup's rows go to part_*[index].
template <int N, int PK>
__global__ __launch_bounds__(256) void k_update_mfma(DevData D, int mode, const double* r, double* z, double* p,
                                                     const double* b, const Scalars* sc) {
    constexpr int N3 = N * N * N;
    constexpr bool F32 = PK == 3;
    using S = MfmaSplit<N3>;
    constexpr int KC = S::KC, KS = S::KS;
    constexpr int DP = 8;                             // steps of operand A in flight (divides KS)
    using GT = typename std::conditional<F32, float, double>::type;
    constexpr int V = F32 ? 4 : 2;                    // rows per lane per load (16 bytes)
    constexpr int T = 64 / (16 * V);                  // super-tiles per wavefront
    typedef GT VT __attribute__((ext_vector_type(V)));
    const int wg = blockIdx.x / D.nrhs;
    const int rh = blockIdx.x - wg * D.nrhs;
    if (rh) {
        bind_rhs(D, rh);
        const long long o = rh * D.vstride;
        r += o;
        z += o;
        if (p) p += o;
        if (b) b += o;
    }
    if (sc) sc += rh;
    if (sc && sc->done && mode != 2) return;
    __shared__ __align__(16) double sr[KC * 16];      // residual chunk [k][element]
    __shared__ double red[3 * 4];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    double prz = 0, prr = 0, pbb = 0;
    if (wg < D.ntasks * S::P) {
        const int task = wg / S::P, part = wg - task * S::P;
        const int first = D.task_first[task], cnt = D.task_count[task], bi = D.task_block[task];
        const int m = lane & 15, kq = lane >> 4;            // operand row / column index of this lane
        const int rowbase = part * S::RP + w * 64;           // first row of this wavefront
        const bool wact = rowbase < N3;
        constexpr int LASTG = (N3 - 1) & ~(V - 1);          // last V-aligned row (column padded past it)
        const GT* Bb = (F32 ? (const GT*)D.B32 : (const GT*)D.B64) + (size_t)bi * N3 * D.ldb;
        const size_t ld = D.ldb;
        int arow[T];
#pragma unroll
        for (int t = 0; t < T; ++t) arow[t] = min(rowbase + 16 * V * t + V * m, LASTG);
        auto loadA = [&](int s, VT (&a)[T]) {
            const GT* col = Bb + (size_t)min(4 * s + kq, N3 - 1) * ld;
#pragma unroll
            // streamed once per launch: non-temporal loads keep the caches for
            // the vectors (measured 15-20 % faster than plain loads)
            for (int t = 0; t < T; ++t) a[t] = __builtin_nontemporal_load(reinterpret_cast<const VT*>(col + arow[t]));
        };
        // residual staging: thread -> columns tid % 64 + 64 hh of the chunk,
        // elements tid / 64 + NW q (SQ per thread)
        constexpr int NW = S::NW, SQ = (16 + NW - 1) / NW;
        // staging source per q: element * 8 + reversal code, or -1 (no element)
        int esrc[SQ];
#pragma unroll
        for (int q = 0; q < SQ; ++q) {
            const int v = (tid >> 6) + NW * q;
            const int el = v < cnt ? D.uorder[first + v] : -1;
            esrc[q] = el >= 0 ? 8 * el + D.bflip[el] : -1;
        }
        // The next chunk's residuals are loaded at the start of a chunk (from
        // clamped addresses, no branches) and only used, masked, when the
        // chunk is stored at its end: a use right after the load would wait
        // for it, and with it for every operand load issued before it.
        double stv[SQ];
        auto stage_load = [&](int c) {
            const int kc = min(c * KC + (tid & 63), N3 - 1);
#pragma unroll
            for (int q = 0; q < SQ; ++q) {
                const int es = max(esrc[q], 0);
                stv[q] = r[(size_t)(es >> 3) * N3 + flip_index<N>(kc, es & 7)];
            }
        };
        auto stage_store = [&](int c) {
            const bool kin = c * KC + (tid & 63) < N3;
#pragma unroll
            for (int q = 0; q < SQ; ++q) {
                const int v = (tid >> 6) + NW * q;
                if (v < 16) sr[(tid & 63) * 16 + v] = (kin && esrc[q] >= 0) ? stv[q] : 0.0;
            }
        };
        dbl4 acc[T][V];
#pragma unroll
        for (int t = 0; t < T; ++t)
#pragma unroll
            for (int h = 0; h < V; ++h) acc[t][h] = dbl4{0.0, 0.0, 0.0, 0.0};
        // Every wavefront runs the whole sweep (one without rows reads a clamped
        // row, and its results are dropped); columns past n3 meet zero residuals.
        VT ring[DP][T];
#pragma unroll
        for (int d = 0; d < DP; ++d) loadA(d, ring[d]);
        stage_load(0);
        stage_store(0);
        __syncthreads();
#pragma unroll 1
        for (int c = 0; c < S::NCH; ++c) {
            stage_load(c + 1);
#pragma unroll
            for (int j = 0; j < KS; ++j) {
                VT a[T];
#pragma unroll
                for (int t = 0; t < T; ++t) a[t] = ring[j % DP][t];
                loadA(c * KS + j + DP, ring[j % DP]);
                const double bop = sr[(4 * j + kq) * 16 + m];
#pragma unroll
                for (int t = 0; t < T; ++t)
#pragma unroll
                    for (int h = 0; h < V; ++h)
                        acc[t][h] = __builtin_amdgcn_mfma_f64_16x16x4f64((double)a[t][h], bop, acc[t][h], 0, 0, 0);
                // steps stay in order: the ring's loads keep their distance
                __builtin_amdgcn_sched_barrier(0);
            }
            __syncthreads();
            stage_store(c + 1);
            __syncthreads();
        }
        // results: register q of lane (m, kq) holds tile row 4 q + kq, element m,
        // i.e. row rowbase + 16 V t + V (4 q + kq) + h of acc[t][h]
        if (wact && m < cnt) {
            const int el = D.uorder[first + m];
            const size_t base = (size_t)el * N3;
            const int fm = D.bflip[el];
#pragma unroll
            for (int t = 0; t < T; ++t)
#pragma unroll
                for (int h = 0; h < V; ++h)
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        const int i0 = rowbase + 16 * V * t + V * (4 * q + kq) + h;
                        if (i0 < N3) {
                            // row i0 of the stored block is local index f(i0) of the element
                            const int i = flip_index<N>(i0, fm);
                            const double zv = acc[t][h][q];
                            z[base + i] = zv;
                            if (mode == 0) {
                                p[base + i] = zv;
                                pbb += b[base + i] * b[base + i];
                            }
                            const double rv = r[base + i];
                            prz += rv * zv;
                            prr += rv * rv;
                        }
                    }
        }
    } else {
        // corner unknowns
        const size_t c0 = D.nreal_dof;
        for (int c = tid; c < D.ncd; c += blockDim.x) {
            const double rv = r[c0 + c];
            prr += rv * rv;
            if (mode == 0) pbb += b[c0 + c] * b[c0 + c];
        }
        if (D.ncd > 0) {
            if (PK == 1) corner_block_apply<double>(D.Gc64, D.ncd, r + c0, D.cscratch, z + c0);
            else corner_block_apply<float>(D.Gc32, D.ncd, r + c0, D.cscratch, z + c0);
            for (int c = tid; c < D.ncd; c += blockDim.x) {
                const double zv = z[c0 + c];
                if (mode == 0) p[c0 + c] = zv;
                prz += r[c0 + c] * zv;
            }
        }
    }
    if (mode == 2) return;
    // fixed-order workgroup sums: wavefront shuffles, then the wavefronts in order
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        prz += __shfl_xor(prz, off);
        prr += __shfl_xor(prr, off);
        pbb += __shfl_xor(pbb, off);
    }
    if (lane == 0) { red[3 * w] = prz; red[3 * w + 1] = prr; red[3 * w + 2] = pbb; }
    __syncthreads();
    if (tid == 0) {
        double a = 0, c = 0, d = 0;
        for (int ww = 0; ww < MfmaSplit<N3>::NW; ++ww) { a += red[3 * ww]; c += red[3 * ww + 1]; d += red[3 * ww + 2]; }
        D.part_a[wg] = a;
        D.part_b[wg] = c;
        D.part_c[wg] = d;
    }
}

__global__ __launch_bounds__(BLOCK) void k_fin_update(DevData D, int mode, int nblk, double* p, const double* z,
                                                      Scalars* sc) {
    const int rh = blockIdx.x;
    if (rh) {
        bind_rhs(D, rh);
        p += rh * D.vstride;
        z += rh * D.vstride;
    }
    sc += rh;
    if (sc->done) return;
    __shared__ double red[BLOCK];
    __shared__ double sbeta;
    __shared__ int sgo;
    const int tid = threadIdx.x;
    double trz = 0, trr = 0, tbb = 0;
    for (int i = tid; i < nblk; i += BLOCK) { trz += D.part_a[i]; trr += D.part_b[i]; tbb += D.part_c[i]; }
    trz = block_sum(trz, red);
    trr = block_sum(trr, red);
    tbb = block_sum(tbb, red);
    if (tid == 0) {
        if (mode == 0) { sc->bb = tbb; sc->iter = 0; sc->status = 0; }
        const double bb = sc->bb;
        sc->rr = trr;
        sc->relres = (bb > 0) ? sqrt(trr / bb) : 0.0;
        sgo = 0;
        if (!(trz == trz) || !(trr == trr)) { sc->status = -6; sc->done = 1; }
        else if (trr == 0.0 || sc->relres <= sc->tol) { sc->done = 1; }
        else if (trz <= 0.0) { sc->status = -5; sc->done = 1; }
        if (mode == 0) { sc->rho = trz; sc->beta = 0.0; }
        else {
            sc->iter += 1;
            sc->beta = trz / sc->rho;
            sc->rho = trz;
            sbeta = sc->beta;
            if (!sc->done && sc->iter >= sc->maxit) { sc->status = -4; sc->done = 1; }
            // the corner part of p is advanced even on convergence, so that a
            // solve resumed after a residual replacement continues consistently
            sgo = sc->status == 0;
        }
    }
    __syncthreads();
    // corner part of p = z + beta p (the element part is fused into k_volume)
    if (mode != 0 && sgo) {
        const double be = sbeta;
        for (int c = tid; c < D.ncd; c += BLOCK) {
            const size_t i = D.nreal_dof + c;
            p[i] = z[i] + be * p[i];
        }
    }
}

// ---------------------------------------------------------------------------
// Assembly of the element blocks of X for the element-block preconditioner:
// X is applied to v = sum over the elements e of one colour of the unit
// vector at local index j of e.  Elements of one colour share no face term,
// so the part of X v on e is column j of e's diagonal block.  R columns at
// once: right-hand side rh of a multi right-hand side apply (vectors vs
// apart) carries local index j0 + rh.
// ---------------------------------------------------------------------------
__global__ void k_unit_vector(double* v, const int* elems, int ne, int n3, int j0, int R, long long vs) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= ne * R) return;
    const int k = t / R, rh = t - k * R, j = j0 + rh;
    double* vr = v + rh * vs + (size_t)elems[k] * n3;   // real-element index
    if (j0 > 0) vr[j - R] = 0.0;                        // this slot's previous column
    if (j < n3) vr[j] = 1.0;
}

__global__ void k_unit_clear(double* v, const int* elems, int ne, int n3, int j0, int R, long long vs) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= ne * R) return;
    const int k = t / R, rh = t - k * R, j = j0 + rh;
    if (j < n3) v[rh * vs + (size_t)elems[k] * n3 + j] = 0.0;
}

// column j0 + rh of block k of B = y of right-hand side rh on element
// elems[k], for the elements of an assembly chunk (column-major n3 x n3
// blocks, one per list position)
__global__ void k_extract_column(double* B, const double* y, const int* elems, int ne, int n3, int j0, int R,
                                 long long vs) {
    const int k = blockIdx.y / R, rh = blockIdx.y - k * R, j = j0 + rh;
    if (k >= ne || j >= n3) return;
    const size_t ob = ((size_t)k * n3 + j) * n3;
    const double* yr = y + rh * vs + (size_t)elems[k] * n3;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n3; i += gridDim.x * blockDim.x) B[ob + i] = yr[i];
}

// per block: sum of entries, sum of magnitudes, trace (fixed-order sums);
// equal blocks have equal signatures
__global__ __launch_bounds__(BLOCK) void k_block_sig(const double* A, int n3, double* sig) {
    __shared__ double red[BLOCK];
    const double* a = A + (size_t)blockIdx.x * n3 * n3;
    double s1 = 0, s2 = 0, s3 = 0;
    for (size_t t = threadIdx.x; t < (size_t)n3 * n3; t += BLOCK) {
        const double v = a[t];
        s1 += v;
        s2 += fabs(v);
        if (t % (n3 + 1) == 0) s3 += v;
    }
    s1 = block_sum(s1, red);
    s2 = block_sum(s2, red);
    s3 = block_sum(s3, red);
    if (threadIdx.x == 0) { sig[3 * blockIdx.x] = s1; sig[3 * blockIdx.x + 1] = s2; sig[3 * blockIdx.x + 2] = s3; }
}

__device__ inline double block_max(double v, double* red) {
    const int t = threadIdx.x;
    red[t] = v;
    __syncthreads();
    for (int s = BLOCK / 2; s > 0; s >>= 1) {
        if (t < s) red[t] = fmax(red[t], red[t + s]);
        __syncthreads();
    }
    const double r = red[0];
    __syncthreads();
    return r;
}

// Batched comparison of element blocks with stored blocks up to a reversal
// of lambda axes: for triple i = (x, u, c) of trip, out[2 i] = max_ab
// |A_x[a][b] - R_u[f(a)][f(b)]| and out[2 i + 1] = max |R_u|, A_x block x of
// A, R_u = R[u], f reversing the local index along lambda_d when bit d of c
// is set (blocks column-major n3 x n3, n3 = n^3).
__global__ __launch_bounds__(BLOCK) void k_block_cmp(const double* A, const double* const* R, int n, const int* trip,
                                                     double* out) {
    __shared__ double red[BLOCK];
    const int n3 = n * n * n;
    const int x = trip[3 * blockIdx.x], u = trip[3 * blockIdx.x + 1], c = trip[3 * blockIdx.x + 2];
    const double* ae = A + (size_t)x * n3 * n3;
    const double* au = R[u];
    auto flip = [&](int t) {
        int i = t % n, j = (t / n) % n, k = t / (n * n);
        if (c & 1) i = n - 1 - i;
        if (c & 2) j = n - 1 - j;
        if (c & 4) k = n - 1 - k;
        return i + n * (j + n * k);
    };
    double d = 0, m = 0;
    for (int b = 0; b < n3; ++b) {
        const size_t cb = (size_t)flip(b) * n3;
        for (int a = threadIdx.x; a < n3; a += BLOCK) {
            const double vu = au[cb + flip(a)];
            d = fmax(d, fabs(ae[(size_t)b * n3 + a] - vu));
            m = fmax(m, fabs(vu));
        }
    }
    d = block_max(d, red);
    m = block_max(m, red);
    if (threadIdx.x == 0) { out[2 * blockIdx.x] = d; out[2 * blockIdx.x + 1] = m; }
}

void launch_block_cmp(hipStream_t st, const double* A, const double* const* R, int n, const int* trip, int ntrip,
                      double* out) {
    if (ntrip > 0) hipLaunchKernelGGL(k_block_cmp, dim3(ntrip), dim3(BLOCK), 0, st, A, R, n, trip, out);
}

void launch_block_sig(hipStream_t st, const double* A, int n3, int nblk, double* sig) {
    hipLaunchKernelGGL(k_block_sig, dim3(nblk), dim3(BLOCK), 0, st, A, n3, sig);
}


// packs the lower triangle of each column-major n3 x n3 block: by columns
// into B64 (double) or G32 (float), and by rows into G32r (float) when given
__global__ void k_pack_lower(const double* A, double* B64, float* G32, float* G32r, int n3, int nblk) {
    // (B64 and G32 may both be given: the same lower triangle in double and float)
    const int e = blockIdx.y;
    if (e >= nblk) return;
    const size_t P = (size_t)n3 * (n3 + 1) / 2;
    const double* a = A + (size_t)e * n3 * n3;
    for (size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x; t < (size_t)n3 * n3;
         t += (size_t)gridDim.x * blockDim.x) {
        const int i = (int)(t % n3), j = (int)(t / n3);
        if (i < j) continue;
        const size_t oc = (size_t)e * P + (size_t)packed_col(j, n3) + (i - j);
        const double v = a[t];
        if (B64) B64[oc] = v;
        if (G32) G32[oc] = (float)v;
        if (G32r) G32r[(size_t)e * P + (size_t)packed_row(i) + j] = (float)v;
    }
}

void launch_unit_vector(hipStream_t st, double* v, const int* elems, int ne, int n3, int j0, int R, long long vs) {
    hipLaunchKernelGGL(k_unit_vector, dim3((ne * R + 255) / 256), dim3(256), 0, st, v, elems, ne, n3, j0, R, vs);
}
void launch_unit_clear(hipStream_t st, double* v, const int* elems, int ne, int n3, int j0, int R, long long vs) {
    hipLaunchKernelGGL(k_unit_clear, dim3((ne * R + 255) / 256), dim3(256), 0, st, v, elems, ne, n3, j0, R, vs);
}
void launch_extract_column(hipStream_t st, double* B, const double* y, const int* elems, int ne, int n3, int j0, int R,
                           long long vs) {
    hipLaunchKernelGGL(k_extract_column, dim3((n3 + 255) / 256, ne * R), dim3(256), 0, st, B, y, elems, ne, n3, j0, R,
                       vs);
}
// the lower triangle of packed float blocks back into column-major double
// blocks (for the positive-definiteness check of the rounded inverses)
__global__ void k_unpack_lower(const float* P32, double* A, int n3, int nblk) {
    const int e = blockIdx.y;
    if (e >= nblk) return;
    const size_t P = (size_t)n3 * (n3 + 1) / 2;
    double* a = A + (size_t)e * n3 * n3;
    for (size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x; t < (size_t)n3 * n3;
         t += (size_t)gridDim.x * blockDim.x) {
        const int i = (int)(t % n3), j = (int)(t / n3);
        a[t] = (i < j) ? 0.0 : (double)P32[(size_t)e * P + (size_t)packed_col(j, n3) + (i - j)];
    }
}

// full symmetric storage of blocks whose lower triangle is valid (column-major
// n3 x n3 input): column k at k ld in B
template <class GT>
__global__ void k_pack_full(const double* A, GT* B, int ld, int n3, int nblk) {
    const int e = blockIdx.y;
    if (e >= nblk) return;
    const double* a = A + (size_t)e * n3 * n3;
    GT* bb = B + (size_t)e * n3 * ld;
    for (size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x; t < (size_t)n3 * n3;
         t += (size_t)gridDim.x * blockDim.x) {
        const int i = (int)(t % n3), j = (int)(t / n3);
        if (i < j) continue;
        const GT v = (GT)a[t];
        bb[(size_t)j * ld + i] = v;
        bb[(size_t)i * ld + j] = v;
    }
}

// a float full block back into a column-major double block (positive-definiteness check)
__global__ void k_unpack_full(const float* B, int ld, double* A, int n3, int nblk) {
    const int e = blockIdx.y;
    if (e >= nblk) return;
    double* a = A + (size_t)e * n3 * n3;
    const float* bb = B + (size_t)e * n3 * ld;
    for (size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x; t < (size_t)n3 * n3;
         t += (size_t)gridDim.x * blockDim.x) {
        const int i = (int)(t % n3), j = (int)(t / n3);
        a[t] = (double)bb[(size_t)j * ld + i];
    }
}

void launch_pack_full64(hipStream_t st, const double* A, double* B, int ld, int n3, int nblk) {
    const int gx = (int)std::min<long long>(((long long)n3 * n3 + 255) / 256, 4096);
    hipLaunchKernelGGL(k_pack_full<double>, dim3(gx, nblk), dim3(256), 0, st, A, B, ld, n3, nblk);
}

void launch_pack_full32(hipStream_t st, const double* A, float* B, int ld, int n3, int nblk) {
    const int gx = (int)std::min<long long>(((long long)n3 * n3 + 255) / 256, 4096);
    hipLaunchKernelGGL(k_pack_full<float>, dim3(gx, nblk), dim3(256), 0, st, A, B, ld, n3, nblk);
}

void launch_unpack_full(hipStream_t st, const float* B, int ld, double* A, int n3, int nblk) {
    const int gx = (int)std::min<long long>(((long long)n3 * n3 + 255) / 256, 4096);
    hipLaunchKernelGGL(k_unpack_full, dim3(gx, nblk), dim3(256), 0, st, B, ld, A, n3, nblk);
}

void launch_unpack_lower(hipStream_t st, const float* P32, double* A, int n3, int nblk) {
    const int gx = (int)std::min<long long>(((long long)n3 * n3 + 255) / 256, 4096);
    hipLaunchKernelGGL(k_unpack_lower, dim3(gx, nblk), dim3(256), 0, st, P32, A, n3, nblk);
}

void launch_pack_lower(hipStream_t st, const double* A, double* B64, float* G32, float* G32r, int n3, int nblk) {
    const int gx = (int)std::min<long long>(((long long)n3 * n3 + 255) / 256, 4096);
    hipLaunchKernelGGL(k_pack_lower, dim3(gx, nblk), dim3(256), 0, st, A, B64, G32, G32r, n3, nblk);
}

// ---------------------------------------------------------------------------
// Tensor Legendre source f(x) = sum_{a,b,c < deg} theta[a + deg (b + deg c)]
// P_a(x1) P_b(x2) P_c(x3) and its adjoint.
// ---------------------------------------------------------------------------
constexpr int MAXDEG = 12;

__device__ inline void legendre_values(double x, int deg, double* P) {
    P[0] = 1.0;
    if (deg > 1) P[1] = x;
    for (int k = 1; k + 1 < deg; ++k) P[k + 1] = ((2 * k + 1) * x * P[k] - k * P[k - 1]) / (k + 1);
}

// d_q = s_q f(x_q) at every volume point
__global__ __launch_bounds__(BLOCK) void k_source_eval(const double* xv, const double* svol, const double* theta,
                                                       int deg, long long npts, double* dvol) {
    __shared__ double sth[MAXDEG * MAXDEG * MAXDEG];
    const int K = deg * deg * deg;
    for (int k = threadIdx.x; k < K; k += BLOCK) sth[k] = theta[k];
    __syncthreads();
    const long long q = (long long)blockIdx.x * BLOCK + threadIdx.x;
    if (q >= npts) return;
    double P1[MAXDEG], P2[MAXDEG], P3[MAXDEG];
    legendre_values(xv[3 * q], deg, P1);
    legendre_values(xv[3 * q + 1], deg, P2);
    legendre_values(xv[3 * q + 2], deg, P3);
    double f = 0.0;
    for (int c = 0; c < deg; ++c) {
        double fb = 0.0;
        for (int b = 0; b < deg; ++b) {
            double fa = 0.0;
            for (int a = 0; a < deg; ++a) fa += sth[a + deg * (b + deg * c)] * P1[a];
            fb += fa * P2[b];
        }
        f += fb * P3[c];
    }
    dvol[q] = svol[q] * f;
}

// d_q = s_q f(x_q), f = sum_k a_k cos(pi (kappa_k . x) + phi_k); coef [nmodes][5]
// = (a, kappa_1, kappa_2, kappa_3, phi)
__global__ __launch_bounds__(BLOCK) void k_source_fourier(const double* xv, const double* svol, const double* coef,
                                                          int nmodes, long long npts, double* dvol) {
    const long long q = (long long)blockIdx.x * BLOCK + threadIdx.x;
    if (q >= npts) return;
    const double x0 = xv[3 * q], x1 = xv[3 * q + 1], x2 = xv[3 * q + 2];
    double f = 0.0;
    for (int k = 0; k < nmodes; ++k) {
        const double* c = coef + 5 * k;
        f += c[0] * cos(M_PI * (c[1] * x0 + c[2] * x1 + c[3] * x2) + c[4]);
    }
    dvol[q] = svol[q] * f;
}

void launch_source_fourier(hipStream_t st, const double* xv, const double* svol, const double* coef, int nmodes,
                           long long npts, double* dvol) {
    hipLaunchKernelGGL(k_source_fourier, dim3((unsigned)((npts + BLOCK - 1) / BLOCK)), dim3(BLOCK), 0, st, xv, svol,
                       coef, nmodes, npts, dvol);
}

// part[r][k] = sum over the points q of element r of s_q z_q P_a P_b P_c
__global__ __launch_bounds__(BLOCK) void k_source_project(const double* xv, const double* svol, const double* z,
                                                          int deg, int m3, double* part) {
    constexpr int CH = 64;
    __shared__ double sP[3][MAXDEG][CH];
    __shared__ double sw[CH];
    constexpr int KR = (MAXDEG * MAXDEG * MAXDEG + BLOCK - 1) / BLOCK;
    const int r = blockIdx.x;
    const int tid = threadIdx.x;
    const int K = deg * deg * deg;
    double acc[KR];
#pragma unroll
    for (int j = 0; j < KR; ++j) acc[j] = 0.0;
    const size_t base = (size_t)r * m3;
    for (int q0 = 0; q0 < m3; q0 += CH) {
        const int nq = min(CH, m3 - q0);
        if (tid < 3 * CH) {
            const int d = tid / CH, qq = tid % CH;
            double P[MAXDEG];
            const double x = (qq < nq) ? xv[3 * (base + q0 + qq) + d] : 0.0;
            legendre_values(x, deg, P);
            for (int a = 0; a < deg; ++a) sP[d][a][qq] = P[a];
            if (d == 0) sw[qq] = (qq < nq) ? svol[base + q0 + qq] * z[base + q0 + qq] : 0.0;
        }
        __syncthreads();
#pragma unroll
        for (int j = 0; j < KR; ++j) {
            const int k = tid + BLOCK * j;
            if (k < K) {
                const int a = k % deg, b = (k / deg) % deg, c = k / (deg * deg);
                double v = 0.0;
                for (int qq = 0; qq < nq; ++qq) v += sw[qq] * sP[0][a][qq] * sP[1][b][qq] * sP[2][c][qq];
                acc[j] += v;
            }
        }
        __syncthreads();
    }
#pragma unroll
    for (int j = 0; j < KR; ++j) {
        const int k = tid + BLOCK * j;
        if (k < K) part[(size_t)r * K + k] = acc[j];
    }
}

// out[k] = sum_r part[r][k] in element order
__global__ void k_sum_rows(const double* part, int nrows, int K, double* out) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= K) return;
    double s = 0.0;
    for (int r = 0; r < nrows; ++r) s += part[(size_t)r * K + k];
    out[k] = s;
}

void launch_source_eval(hipStream_t st, const double* xv, const double* svol, const double* theta, int deg,
                        long long npts, double* dvol) {
    hipLaunchKernelGGL(k_source_eval, dim3((unsigned)((npts + BLOCK - 1) / BLOCK)), dim3(BLOCK), 0, st, xv, svol,
                       theta, deg, npts, dvol);
}

void launch_sum_rows(hipStream_t st, const double* part, int nrows, int K, double* out) {
    hipLaunchKernelGGL(k_sum_rows, dim3((K + 255) / 256), dim3(256), 0, st, part, nrows, K, out);
}

void launch_source_project(hipStream_t st, const double* xv, const double* svol, const double* z, int deg, int m3,
                           int nelem, double* part, double* out) {
    hipLaunchKernelGGL(k_source_project, dim3(nelem), dim3(BLOCK), 0, st, xv, svol, z, deg, m3, part);
    const int K = deg * deg * deg;
    hipLaunchKernelGGL(k_sum_rows, dim3((K + 255) / 256), dim3(256), 0, st, part, nelem, K, out);
}


// per right-hand side flag operations of the batched mixed solver:
// op 1 re-opens a solve stopped by its recursive residual, op 2 stops it with
// status -4 (its true residual no longer decreases)
__global__ void k_flag_ops(Scalars* sc, const int* op, int R) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= R) return;
    if (op[k] == 1 && sc[k].status == 0) sc[k].done = 0;
    if (op[k] == 2) { sc[k].done = 1; sc[k].status = -4; }
}

// u_rh += alpha_rh p_rh for R right-hand sides of length n
__global__ void k_axpy_alpha_multi(double* u, const double* p, const Scalars* sc, long long n, int R) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n * R) return;
    const int rh = (int)(i / n);
    if (sc[rh].done) return;
    u[i] += sc[rh].alpha * p[i];
}

void launch_flag_ops(hipStream_t st, Scalars* sc, const int* op, int R) {
    hipLaunchKernelGGL(k_flag_ops, dim3((R + 63) / 64), dim3(64), 0, st, sc, op, R);
}

void launch_axpy_alpha_multi(hipStream_t st, double* u, const double* p, const Scalars* sc, long long n, int R) {
    hipLaunchKernelGGL(k_axpy_alpha_multi, dim3((unsigned)((n * R + 255) / 256)), dim3(256), 0, st, u, p, sc, n, R);
}

// r = a - b (vector)
__global__ void k_sub(double* r, const double* a, const double* b, long long n) {
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) r[i] = a[i] - b[i];
}

// ---------------------------------------------------------------------------
// k_error: per real element, partial sums of the H^1 error and norm.
// ---------------------------------------------------------------------------
template <int N>
__global__ __launch_bounds__(BLOCK) void k_error(DevData D, const double* u, int nq, const double* Lg,
                                                 const double* Lg1, const double* eji, const double* ew,
                                                 const double* uex, const double* gex, double* part) {
    (void)D;
    constexpr int N3 = N * N * N;
    __shared__ double su[N3];
    __shared__ double red[BLOCK];
    const int tid = threadIdx.x;
    const int r = blockIdx.x;
    for (int t = tid; t < N3; t += BLOCK) su[t] = u[(size_t)r * N3 + t];
    __syncthreads();
    const int nq3 = nq * nq * nq;
    double num = 0, den = 0;
    for (int q = tid; q < nq3; q += BLOCK) {
        const int a = q % nq, b = (q / nq) % nq, c = q / (nq * nq);
        double v = 0, g0 = 0, g1 = 0, g2 = 0;
        for (int k = 0; k < N; ++k)
            for (int j = 0; j < N; ++j)
                for (int i = 0; i < N; ++i) {
                    const double x = su[i + N * (j + N * k)];
                    const double li = Lg[a * N + i], lj = Lg[b * N + j], lk = Lg[c * N + k];
                    const double di = Lg1[a * N + i], dj = Lg1[b * N + j], dk = Lg1[c * N + k];
                    v += li * lj * lk * x;
                    g0 += di * lj * lk * x;
                    g1 += li * dj * lk * x;
                    g2 += li * lj * dk * x;
                }
        const size_t base = (size_t)r * nq3 + q;
        const double* Ji = eji + base * 9;
        double gx[3];
        for (int aa = 0; aa < 3; ++aa) gx[aa] = Ji[0 * 3 + aa] * g0 + Ji[1 * 3 + aa] * g1 + Ji[2 * 3 + aa] * g2;
        const double w = ew[base];
        const double du = v - uex[base];
        double e2 = du * du, n2 = uex[base] * uex[base];
        for (int aa = 0; aa < 3; ++aa) {
            const double dg = gx[aa] - gex[base * 3 + aa];
            e2 += dg * dg;
            n2 += gex[base * 3 + aa] * gex[base * 3 + aa];
        }
        num += w * e2;
        den += w * n2;
    }
    num = block_sum(num, red);
    den = block_sum(den, red);
    if (tid == 0) { part[2 * r] = num; part[2 * r + 1] = den; }
}

// ---------------------------------------------------------------------------
// Conforming correction (Appendix C.1): uc = u + nu on each real element,
// nu = sum over its interior faces of (1 -/+ lam_d)/2 c_f [u]_f, [u]_f the
// neighbour's value minus the element's own at the face nodes (c_f = 1/2, 1
// next to a corner element).  tab [Ereal][6][5]: code (-1 none, 0 real
// neighbour, 1 corner constant, 2 corner polynomial), the neighbour's first
// unknown (real: element offset; corner: corner offset), its face, the
// orientation code, the corner polynomial's direction.  One workgroup per
// real element; u and uc must not alias.
// ---------------------------------------------------------------------------
template <int N>
__global__ __launch_bounds__(BLOCK) void k_conform(const double* u, double* uc, const int* tab, const double* xn,
                                                   long long nreal_dof) {
    constexpr int N2 = N * N, N3 = N * N * N;
    const int e = blockIdx.x;
    const size_t base = (size_t)e * N3;
    __shared__ double jump[6][N2];
    __shared__ int code[6];
    const int tid = threadIdx.x;
    const int* te = tab + (size_t)e * 30;
    if (tid < 6) code[tid] = te[5 * tid];
    for (int t = tid; t < 6 * N2; t += BLOCK) {
        const int f = t / N2, pq = t - f * N2, ia = pq % N, ib = pq / N;
        const int* tf = te + 5 * f;
        if (tf[0] < 0) { jump[f][pq] = 0.0; continue; }
        const int d = f >> 1, s = f & 1;
        const int t0 = d == 0 ? 1 : 0, t1 = d == 2 ? 1 : 2;
        int idx[3];
        idx[d] = s ? N - 1 : 0;
        idx[t0] = ia;
        idx[t1] = ib;
        const double own = u[base + idx[0] + N * (idx[1] + N * idx[2])];
        // the neighbour's node: face coordinates mapped by the orientation
        // code (swap, then reversal of the first / second), GLL nodes being
        // symmetric about 0
        const int o = tf[3];
        int ja = ia, jb = ib;
        if (o & 1) { ja = ib; jb = ia; }
        if (o & 2) ja = N - 1 - ja;
        if (o & 4) jb = N - 1 - jb;
        const int f2 = tf[2], d2 = f2 >> 1, s2 = f2 & 1;
        const int u0 = d2 == 0 ? 1 : 0, u1 = d2 == 2 ? 1 : 2;
        int jdx[3];
        jdx[d2] = s2 ? N - 1 : 0;
        jdx[u0] = ja;
        jdx[u1] = jb;
        double nb;
        if (tf[0] == 0) nb = u[(size_t)tf[1] + jdx[0] + N * (jdx[1] + N * jdx[2])];
        else if (tf[0] == 1) nb = u[nreal_dof + tf[1]];
        else nb = u[nreal_dof + tf[1] + jdx[tf[4]]];
        jump[f][pq] = (tf[0] == 0 ? 0.5 : 1.0) * (nb - own);
    }
    __syncthreads();
    for (int t = tid; t < N3; t += BLOCK) {
        const int i = t % N, j = (t / N) % N, k = t / N2;
        const int id[3] = {i, j, k};
        double v = u[base + t];
#pragma unroll
        for (int f = 0; f < 6; ++f) {
            if (code[f] < 0) continue;
            const int d = f >> 1, s = f & 1;
            const int t0 = d == 0 ? 1 : 0, t1 = d == 2 ? 1 : 2;
            const double x = xn[id[d]];
            const double blend = s ? 0.5 * (1.0 + x) : 0.5 * (1.0 - x);
            v += blend * jump[f][id[t0] + N * id[t1]];
        }
        uc[base + t] = v;
    }
}

// ---------------------------------------------------------------------------
// Graded degrees (Sec. 2.3).  Q_w (projtab[w], N x N row-major) is the
// orthogonal projector onto the degree-w polynomials in the values at the
// GLL nodes; an element of degrees (w1, w2, w3) projects with
// Q = Q_w3 (x) Q_w2 (x) Q_w1 (w1 along i, the fastest index).
// ---------------------------------------------------------------------------
// y (in LDS, N^3, i fastest) <- Q y, with s as scratch
template <int N>
__device__ void project3(const double (*sQ)[N * N], double* y, double* s) {
    constexpr int N2 = N * N, N3 = N * N * N;
    const int tid = threadIdx.x, nt = blockDim.x;
    for (int t = tid; t < N3; t += nt) {
        const int a = t % N, jk = t / N;
        double v = 0;
#pragma unroll
        for (int i = 0; i < N; ++i) v += sQ[0][a * N + i] * y[i + N * jk];
        s[t] = v;
    }
    __syncthreads();
    for (int t = tid; t < N3; t += nt) {
        const int a = t % N, b = (t / N) % N, k = t / N2;
        double v = 0;
#pragma unroll
        for (int j = 0; j < N; ++j) v += sQ[1][b * N + j] * s[a + N * (j + N * k)];
        y[t] = v;
    }
    __syncthreads();
    for (int t = tid; t < N3; t += nt) {
        const int a = t % N, b = (t / N) % N, c = t / N2;
        double v = 0;
#pragma unroll
        for (int k = 0; k < N; ++k) v += sQ[2][c * N + k] * y[a + N * (b + N * k)];
        s[t] = v;
    }
    __syncthreads();
}

template <int N>
__device__ void load_projectors(const DevData& D, int code, double (*sQ)[N * N]) {
    for (int d = 0; d < 3; ++d) {
        const int w = (code >> (8 * d)) & 255;
        for (int i = threadIdx.x; i < N * N; i += blockDim.x) sQ[d][i] = D.projtab[(size_t)w * N * N + i];
    }
}

// q_e <- Q q_e for the graded elements (item = graded element x right-hand side)
template <int N>
__global__ __launch_bounds__(BLOCK) void k_project(DevData D, double* q, const Scalars* sc) {
    constexpr int N3 = N * N * N;
    const int it = blockIdx.x / D.nrhs;
    const int rh = blockIdx.x - it * D.nrhs;
    if (rh) q += rh * D.vstride;
    if (sc) {
        sc += rh;
        if (sc->done) return;
    }
    __shared__ double sQ[3][N * N];
    __shared__ double y[N3], s[N3];
    load_projectors<N>(D, D.proj_deg[it], sQ);
    const size_t base = (size_t)D.proj_elem[it] * N3;
    for (int t = threadIdx.x; t < N3; t += BLOCK) y[t] = q[base + t];
    __syncthreads();
    project3<N>(sQ, y, s);
    for (int t = threadIdx.x; t < N3; t += BLOCK) q[base + t] = s[t];
}

// element blocks of the graded space: B_e <- Q B_e Q + s_e (I - Q) for the
// graded elements (B: [Ereal][n3 columns][n3 rows]), s_e = tr(B_e) / n3 (the
// complement scaled like the block).  Pass 0 takes the traces (one workgroup
// per item, before anything changes), pass 1 projects the columns, pass 2
// the rows and adds s_e (I - Q); workgroup (column or row index, item).
__global__ __launch_bounds__(BLOCK) void k_block_trace(DevData D, const double* B, int n3, double* scale) {
    __shared__ double red[BLOCK];
    const int it = blockIdx.x;
    const double* blk = B + (size_t)D.proj_elem[it] * n3 * n3;
    double v = 0;
    for (int i = threadIdx.x; i < n3; i += BLOCK) v += blk[(size_t)i * n3 + i];
    v = block_sum(v, red);
    if (threadIdx.x == 0) scale[it] = v / n3;
}

template <int N>
__global__ __launch_bounds__(BLOCK) void k_block_project(DevData D, double* B, int pass, const double* scale) {
    constexpr int N3 = N * N * N;
    const int idx = blockIdx.x, it = blockIdx.y;
    __shared__ double sQ[3][N * N];
    __shared__ double y[N3], s[N3];
    load_projectors<N>(D, D.proj_deg[it], sQ);
    double* blk = B + (size_t)D.proj_elem[it] * N3 * N3;
    // pass 1: column idx (contiguous); pass 2: row idx (stride N3)
    const size_t off = pass == 1 ? (size_t)idx * N3 : (size_t)idx;
    const size_t stride = pass == 1 ? 1 : (size_t)N3;
    for (int t = threadIdx.x; t < N3; t += BLOCK) y[t] = blk[off + t * stride];
    __syncthreads();
    project3<N>(sQ, y, s);
    const double sc = scale[it];
    for (int t = threadIdx.x; t < N3; t += BLOCK) {
        double v = s[t];
        if (pass == 2) {
            // s_e (I - Q)[idx][t], Q[i][j] = prod_d Q_d[i_d][j_d]
            const int i1 = idx % N, i2 = (idx / N) % N, i3 = idx / (N * N);
            const int j1 = t % N, j2 = (t / N) % N, j3 = t / (N * N);
            v += sc * ((idx == t ? 1.0 : 0.0) - sQ[0][i1 * N + j1] * sQ[1][i2 * N + j2] * sQ[2][i3 * N + j3]);
        }
        blk[off + t * stride] = v;
    }
}

// ---------------------------------------------------------------------------
// host-side launch helpers, dispatching on the compile-time degree
// ---------------------------------------------------------------------------
template <int W, class T>
struct Launch {
    static constexpr int N = W + 1, M = 2 * W + 1;
    template <int SLAB, int LPC, bool PS = false>
    static void volume(hipStream_t st, const DevData& D, const double* u, double* out, int mode, const double* zf,
                       double* pw, const Scalars* sc) {
        const int ne = D.sub_elem ? D.nsub_elem : D.E;
        if (ne > 0)
            hipLaunchKernelGGL((k_volume<N, M, T, SLAB, LPC, PS>), dim3(ne * D.nrhs), dim3(vol_block<LPC>()), 0, st,
                               D, u, out, mode, zf, pw, sc);
    }
    static void face(hipStream_t st, const DevData& D, int mode, const Scalars* sc) {
        const int nf = D.sub_face ? D.nsub_face : D.nfaces;
        if (nf > 0)
            hipLaunchKernelGGL((k_face<N, M, T>), dim3(nf * D.nrhs), dim3(face_block<M>()), 0, st, D, mode, sc);
    }
    static void gather(hipStream_t st, const DevData& D, double* q, const double* pdot, Scalars* sc, int pcg, int rhs) {
        const int ne = D.sub_elem ? D.nsub_elem : D.E;
        if (ne > 0) hipLaunchKernelGGL((k_gather<N, T>), dim3(ne * D.nrhs), dim3(BLOCK), 0, st, D, q, pdot, sc, rhs);
        if (D.ncd > 0 && !D.sub_elem) {
            const int nb = (D.ncd + BLOCK / 64 - 1) / (BLOCK / 64);
            hipLaunchKernelGGL(k_corner_q, dim3(nb * D.nrhs), dim3(BLOCK), 0, st, D, q, pdot, sc, rhs);
        }
        // graded degrees: the result projected onto the graded space (the
        // partial p.q above is unchanged for p in that space)
        if (D.nproj > 0) hipLaunchKernelGGL((k_project<N>), dim3(D.nproj * D.nrhs), dim3(BLOCK), 0, st, D, q, sc);
        if (pcg) hipLaunchKernelGGL(k_fin_gather, dim3(D.nrhs), dim3(BLOCK), 0, st, D, sc, pcg);
    }
    static void project(hipStream_t st, const DevData& D, double* u) {
        if (D.nproj > 0)
            hipLaunchKernelGGL((k_project<N>), dim3(D.nproj * D.nrhs), dim3(BLOCK), 0, st, D, u, nullptr);
    }
    static void block_project(hipStream_t st, const DevData& D, double* B, double* scale) {
        constexpr int N3 = N * N * N;
        if (D.nproj <= 0) return;
        hipLaunchKernelGGL(k_block_trace, dim3(D.nproj), dim3(BLOCK), 0, st, D, B, N3, scale);
        for (int pass = 1; pass <= 2; ++pass)
            hipLaunchKernelGGL((k_block_project<N>), dim3(N3, D.nproj), dim3(BLOCK), 0, st, D, B, pass, scale);
    }
    static void update(hipStream_t st, const DevData& D, int mode, double* u, double* r, double* z, double* p,
                       const double* q, const double* b, Scalars* sc) {
        constexpr int N3 = N * N * N;
        int nblk = D.Ereal + 1;
        if (D.ntasks > 0 && (D.pk == 1 || D.pk == 3)) {
            if (mode != 2) {
                const int gx = (int)std::min<long long>((D.ndof + BLOCK - 1) / BLOCK, 2048);
                hipLaunchKernelGGL(k_cg_vec, dim3(gx, D.nrhs), dim3(BLOCK), 0, st, D, mode, u, r, p, q, b, sc);
            }
            nblk = D.ntasks * MfmaSplit<N3>::P + 1;
            if (D.pk == 1)
                hipLaunchKernelGGL((k_update_mfma<N, 1>), dim3(nblk * D.nrhs), dim3(64 * MfmaSplit<N3>::NW), 0, st, D,
                                   mode, r, z, p, b,
                                   sc);
            else
                hipLaunchKernelGGL((k_update_mfma<N, 3>), dim3(nblk * D.nrhs), dim3(64 * MfmaSplit<N3>::NW), 0, st, D,
                                   mode, r, z, p, b,
                                   sc);
        } else {
            hipLaunchKernelGGL((k_update<N>), dim3((D.Ereal + 1) * D.nrhs), dim3(BLOCK), 0, st, D, mode, u, r, z, p,
                               q, b, sc);
        }
        // graded degrees with a float form of the element blocks: the rounded
        // inverse leaves O(eps32) parts of z off the graded space, which the
        // projected operator cannot see (they would stay in u); z (and p = z
        // of the first step) are projected back.  r lies in the graded space,
        // so the partial r.z above is unchanged.
        if (D.nproj > 0 && (D.pk == 2 || D.pk == 3)) {
            const Scalars* psc = mode == 2 ? nullptr : sc;     // a lone apply ignores the stop flags
            hipLaunchKernelGGL((k_project<N>), dim3(D.nproj * D.nrhs), dim3(BLOCK), 0, st, D, z, psc);
            if (mode == 0) hipLaunchKernelGGL((k_project<N>), dim3(D.nproj * D.nrhs), dim3(BLOCK), 0, st, D, p, psc);
        }
        if (mode != 2)
            hipLaunchKernelGGL(k_fin_update, dim3(D.nrhs), dim3(BLOCK), 0, st, D, mode, nblk, p, z, sc);
    }
    static void conform(hipStream_t st, const DevData& D, const double* u, double* uc, const int* tab,
                        const double* xn) {
        if (D.Ereal > 0)
            hipLaunchKernelGGL((k_conform<N>), dim3(D.Ereal), dim3(BLOCK), 0, st, u, uc, tab, xn, D.nreal_dof);
    }
    static void error(hipStream_t st, const DevData& D, const double* u, int nq, const double* Lg, const double* Lg1,
                      const double* eji, const double* ew, const double* uex, const double* gex, double* part) {
        hipLaunchKernelGGL((k_error<N>), dim3(D.Ereal), dim3(BLOCK), 0, st, D, u, nq, Lg, Lg1, eji, ew, uex, gex, part);
    }
};

template <int W, class T>
Ops make_ops() {
    using L = Launch<W, T>;
    using C = VolCfg<W + 1, 2 * W + 1, T>;
    Ops o{};
    // candidates: the widest and the 78 KB slab with one lane per column (in
    // float the 78 KB slab with stage 3 on the matrix cores, in FP64 for the
    // degrees where that slab is one point the per-slab stage-1 tile), and
    // the capped slab with four lanes per column (workgroups of 512)
    o.volume_tile[0] = &L::template volume<C::SLAB0, 1>;
    // float: the 78 KB slab with stage 3 on the matrix cores; FP64 where the
    // 78 KB slab is a single point: stage-1 values per slab, four lanes
    constexpr bool ps = !std::is_same<T, float>::value && C::SLAB1 == 1;
    if constexpr (std::is_same<T, float>::value) o.volume_tile[1] = &L::template volume<C::SLAB1, 0>;
    else if constexpr (ps) o.volume_tile[1] = &L::template volume<C::SLABP, 4, true>;
    else o.volume_tile[1] = &L::template volume<C::SLAB1, 1>;
    o.volume_tile[2] = &L::template volume<C::SLABQ, 4>;
    o.tile_slab[0] = C::SLAB0;
    o.tile_slab[1] = ps ? C::SLABP : C::SLAB1;
    o.tile_slab[2] = C::SLABQ;
    o.tile = 0;
    o.volume = o.volume_tile[0];
    o.face = &L::face;
    o.gather = &L::gather;
    o.update = &L::update;
    o.error = &L::error;
    o.conform = &L::conform;
    o.project = &L::project;
    o.block_project = &L::block_project;
    return o;
}

template <class T>
bool get_ops_t(int W, Ops& ops) {
    switch (W) {
    case 1: ops = make_ops<1, T>(); return true;
    case 2: ops = make_ops<2, T>(); return true;
    case 3: ops = make_ops<3, T>(); return true;
    case 4: ops = make_ops<4, T>(); return true;
    case 5: ops = make_ops<5, T>(); return true;
    case 6: ops = make_ops<6, T>(); return true;
    case 7: ops = make_ops<7, T>(); return true;
    case 8: ops = make_ops<8, T>(); return true;
    case 9: ops = make_ops<9, T>(); return true;
    case 10: ops = make_ops<10, T>(); return true;
    case 11: ops = make_ops<11, T>(); return true;
    case 12: ops = make_ops<12, T>(); return true;
    default: return false;
    }
}

bool get_ops(int W, Ops& ops) { return get_ops_t<double>(W, ops); }
bool get_ops_f32(int W, Ops& ops) { return get_ops_t<float>(W, ops); }

template <class T>
int lds_t(int W) {
    switch (W) {
#define SEM_LDS_CASE(w) case w: return VolCfg<w + 1, 2 * w + 1, T>::lds_bytes(VolCfg<w + 1, 2 * w + 1, T>::SLAB0);
    SEM_LDS_CASE(1) SEM_LDS_CASE(2) SEM_LDS_CASE(3) SEM_LDS_CASE(4) SEM_LDS_CASE(5) SEM_LDS_CASE(6)
    SEM_LDS_CASE(7) SEM_LDS_CASE(8) SEM_LDS_CASE(9) SEM_LDS_CASE(10) SEM_LDS_CASE(11) SEM_LDS_CASE(12)
#undef SEM_LDS_CASE
    default: return -1;
    }
}
void update_shape(int W, int* G, int* parts) {
    switch (W) {
#define SEM_G_CASE(w)                                                                                    \
    case w:                                                                                              \
        *G = group_cap<(w + 1) * (w + 1) * (w + 1)>();                                                   \
        *parts = MfmaSplit<(w + 1) * (w + 1) * (w + 1)>::P;                                              \
        return;
        SEM_G_CASE(1) SEM_G_CASE(2) SEM_G_CASE(3) SEM_G_CASE(4) SEM_G_CASE(5) SEM_G_CASE(6)
        SEM_G_CASE(7) SEM_G_CASE(8) SEM_G_CASE(9) SEM_G_CASE(10) SEM_G_CASE(11) SEM_G_CASE(12)
#undef SEM_G_CASE
    default: *G = 1; *parts = 1;
    }
}

int volume_lds_bytes(int W, int fp32) { return fp32 ? lds_t<float>(W) : lds_t<double>(W); }


void launch_sub(hipStream_t st, double* r, const double* a, const double* b, long long n) {
    if (n > 0) hipLaunchKernelGGL(k_sub, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, r, a, b, n);
}

}  // namespace sem
