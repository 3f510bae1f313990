// C ABI of the least-squares h-p spectral element library (see include/sem.h).
#include <hip/hip_runtime.h>
#include <rocsolver/rocsolver.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <stdexcept>
#include <mutex>
#include <string>
#include <vector>

#include "sem_device.h"
#include "sem_internal.h"

using namespace sem;

static_assert(NFIELD == VFIELDS, "host and device field counts differ");

namespace {

thread_local std::string g_err;

sem_status fail(sem_status s, const std::string& msg) {
    g_err = msg;
    return s;
}

struct HipError : std::runtime_error {
    using std::runtime_error::runtime_error;
};

void hipcheck(hipError_t e, const char* what) {
    if (e != hipSuccess) throw HipError(std::string(what) + ": " + hipGetErrorString(e));
}

}  // namespace

struct sem_ctx {
    HostSetup S;
    DevData D{};
    Ops ops{};
    Scalars* sc = nullptr;          // device scalars
    Scalars* sc_host = nullptr;     // pinned mirror
    std::vector<void*> allocs;
    void release(void* p) {
        for (auto it = allocs.begin(); it != allocs.end(); ++it)
            if (*it == p) {
                (void)hipFree(p);
                allocs.erase(it);
                return;
            }
    }
    double* d_q = nullptr;          // [ndof] work: X p
    double* d_r = nullptr;
    double* d_z = nullptr;
    double* d_p = nullptr;
    double* d_b = nullptr;          // stored right-hand side
    double* d_gdata = nullptr;
    double* d_dvol = nullptr;
    bool have_data = false;
    bool have_blocks = false;       // element-block preconditioner built
    int64_t graded_ndof = 0;        // unknowns of the graded space (sem_set_degrees)
    // work buffers of multi right-hand side solves (sem_pcg_solve_batch)
    int multi_R = 0;
    std::vector<void*> multi_mem;
    double *m_q = nullptr, *m_r = nullptr, *m_z = nullptr, *m_p = nullptr;
    double *m_trace = nullptr, *m_slotres = nullptr, *m_pa = nullptr, *m_pb = nullptr, *m_pc = nullptr;
    double *m_cpart = nullptr, *m_cs = nullptr;
    float *m_trace32 = nullptr, *m_slotres32 = nullptr;
    int* m_op = nullptr;            // [R] flag operations (batched mixed solver)
    int* m_op_host = nullptr;
    Scalars* m_sc = nullptr;
    Scalars* m_sc_host = nullptr;
    int mixed_pk = 2;               // float form of the element blocks used by the mixed solver
    int n_stored_blocks = 0;        // distinct element blocks stored
    std::vector<int> proj_elem_host, proj_deg_host;   // graded elements and their degree codes
    double* d_xvol = nullptr;       // [Ereal][m^3][3] volume points (source evaluation)
    double* d_svol = nullptr;       // [Ereal][m^3] data weights s_q
    double* d_zq = nullptr;         // [Ereal][m^3] pointwise residual (adjoint)
    double* d_spart = nullptr;      // [Ereal][deg^3] per-element source projections
    Ops ops32{};                    // FP32 operator launchers (mixed precision)
    bool have32 = false;            // FP32 operator data uploaded
    std::vector<double> face_w_host, pcoef_host;   // kept for the FP32 copies
    // error quadrature
    double *d_Lg = nullptr, *d_Lg1 = nullptr, *d_eji = nullptr, *d_ew = nullptr, *d_epart = nullptr;
    int device = 0;
    // conforming correction: neighbour table and the GLL nodes, built on first use
    int* d_conf_tab = nullptr;
    double* d_xn = nullptr;
    // boundary data of the face terms without a neighbour: host copy of the
    // device array, and each face term's offset in it (-1: interior)
    std::vector<double> gdata_host;
    std::vector<long long> face_goff;

    template <class T>
    T* alloc(size_t count) {
        void* p = nullptr;
        size_t bytes = std::max<size_t>(count, 1) * sizeof(T);
        hipcheck(hipMalloc(&p, bytes), "hipMalloc");
        allocs.push_back(p);
        hipcheck(hipMemset(p, 0, bytes), "hipMemset");
        return static_cast<T*>(p);
    }
    // volume coefficient fields in the element kernel's order: per element
    // and field [a][c][b] (b fastest) instead of the host's [c][b][a], so
    // that a lam1-slab pass reads whole lines (a thread owns column (a, b)
    // and walks c)
    template <class T>
    std::vector<T> coef_device_order(const std::vector<double>& v) const {
        const int m = S.m;
        const size_t m3 = (size_t)m * m * m, nf = v.size() / m3;
        std::vector<T> out(v.size());
        for (size_t f = 0; f < nf; ++f) {
            const double* src = v.data() + f * m3;
            T* dst = out.data() + f * m3;
            for (int c = 0; c < m; ++c)
                for (int b = 0; b < m; ++b)
                    for (int a = 0; a < m; ++a) dst[((size_t)a * m + c) * m + b] = (T)src[((size_t)c * m + b) * m + a];
        }
        return out;
    }
    template <class T>
    T* upload(const std::vector<T>& v) {
        T* p = alloc<T>(v.size());
        if (!v.empty()) hipcheck(hipMemcpy(p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice), "hipMemcpy");
        return p;
    }
    // float copy of FP64 operator data (rounded to nearest)
    float* upload_f32(const std::vector<double>& v) {
        std::vector<float> f(v.size());
        for (size_t i = 0; i < v.size(); ++i) f[i] = (float)v[i];
        return upload(f);
    }
    // operator data of the FP32 contractions, built on first use
    void ensure_fp32() {
        if (have32) return;
        if (!get_ops_f32(S.W, ops32)) throw std::invalid_argument("no FP32 kernels for this W");
        const size_t n2 = (size_t)S.n * S.n;
        Dev<float>& P = D.d32;
        P.Im = upload_f32(S.Im); P.D1m = upload_f32(S.D1m); P.D2m = upload_f32(S.D2m);
        P.Dn = upload_f32(S.Dn); P.K = upload_f32(S.K); P.wm = upload_f32(S.wm);
        P.coef = upload(coef_device_order<float>(S.coef));
        P.face_w = upload_f32(face_w_host);
        P.pcoef = upload_f32(pcoef_host);
        P.trace = alloc<float>((size_t)S.E * 6 * 4 * n2);
        P.slotres = alloc<float>((size_t)S.E * 6 * 4 * n2);
        hipcheck(hipDeviceSynchronize(), "fp32 upload");
        have32 = true;
    }
    void free_multi() {
        for (void* p : multi_mem) (void)hipFree(p);
        multi_mem.clear();
        if (m_sc_host) (void)hipHostFree(m_sc_host);
        m_sc_host = nullptr;
        if (m_op_host) (void)hipHostFree(m_op_host);
        m_op_host = nullptr;
        multi_R = 0;
    }
    // buffers for R right-hand sides (kept for later calls with R or fewer)
    void ensure_multi(int R) {
        if (R <= multi_R) return;
        free_multi();
        auto get = [&](size_t bytes) {
            void* p = nullptr;
            if (hipMalloc(&p, std::max<size_t>(bytes, 8)) != hipSuccess) {
                (void)hipGetLastError();
                free_multi();
                throw std::bad_alloc();
            }
            multi_mem.push_back(p);
            return p;
        };
        const size_t nv = (size_t)R * S.ndof * sizeof(double);
        m_q = (double*)get(nv); m_r = (double*)get(nv); m_z = (double*)get(nv); m_p = (double*)get(nv);
        m_trace = (double*)get((size_t)R * D.tstride * sizeof(double));
        m_slotres = (double*)get((size_t)R * D.tstride * sizeof(double));
        m_pa = (double*)get((size_t)R * D.pstride * sizeof(double));
        m_pb = (double*)get((size_t)R * D.pstride * sizeof(double));
        m_pc = (double*)get((size_t)R * D.pstride * sizeof(double));
        m_cpart = (double*)get((size_t)R * D.cpstride * sizeof(double));
        m_cs = (double*)get((size_t)R * D.csstride * sizeof(double));
        m_sc = (Scalars*)get((size_t)R * sizeof(Scalars));
        hipcheck(hipHostMalloc((void**)&m_sc_host, (size_t)R * sizeof(Scalars), hipHostMallocDefault),
                 "hipHostMalloc");
        m_trace32 = (float*)get((size_t)R * D.tstride * sizeof(float));
        m_slotres32 = (float*)get((size_t)R * D.tstride * sizeof(float));
        m_op = (int*)get((size_t)R * sizeof(int));
        hipcheck(hipHostMalloc((void**)&m_op_host, (size_t)R * sizeof(int), hipHostMallocDefault), "hipHostMalloc");
        // the face results of inactive slots are read as zero: start cleared
        hipcheck(hipMemset(m_slotres, 0, (size_t)R * D.tstride * sizeof(double)), "hipMemset");
        hipcheck(hipMemset(m_trace, 0, (size_t)R * D.tstride * sizeof(double)), "hipMemset");
        hipcheck(hipMemset(m_slotres32, 0, (size_t)R * D.tstride * sizeof(float)), "hipMemset");
        hipcheck(hipMemset(m_trace32, 0, (size_t)R * D.tstride * sizeof(float)), "hipMemset");
        multi_R = R;
    }
    // device data viewing the multi right-hand side buffers (f32: the float
    // operator's traces and the float element blocks)
    DevData multi_view(int R, bool f32 = false) const {
        DevData Dr = D;
        Dr.nrhs = R;
        Dr.d64.trace = f32 ? nullptr : m_trace;
        Dr.d64.slotres = f32 ? nullptr : m_slotres;
        Dr.d32.trace = f32 ? m_trace32 : nullptr;
        Dr.d32.slotres = f32 ? m_slotres32 : nullptr;
        if (f32 && Dr.pk == 1) Dr.pk = mixed_pk;
        Dr.part_a = m_pa; Dr.part_b = m_pb; Dr.part_c = m_pc;
        Dr.cpart = m_cpart;
        Dr.cscratch = m_cs;
        return Dr;
    }
    ~sem_ctx() {
        free_multi();
        for (void* p : allocs) (void)hipFree(p);
        if (sc_host) (void)hipHostFree(sc_host);
    }
};

extern "C" {

const char* sem_last_error(void) { return g_err.c_str(); }

sem_status sem_setup(const sem_mesh* mesh, void* stream, sem_ctx** out) {
    if (!out) return fail(SEM_EINVAL, "sem_setup: out is NULL");
    *out = nullptr;
    sem_ctx* ctx = nullptr;
    try {
        ctx = new sem_ctx();
        build_host_setup(mesh, ctx->S);
        HostSetup& S = ctx->S;
        if (!get_ops(S.W, ctx->ops)) {
            delete ctx;
            return fail(SEM_EINVAL, "sem_setup: W=" + std::to_string(S.W) + " has no compiled kernels");
        }
        hipcheck(hipGetDevice(&ctx->device), "hipGetDevice");
        DevData& D = ctx->D;
        const int n = S.n, m = S.m, n2 = n * n;
        D.W = S.W; D.n = n; D.m = m; D.E = S.E; D.Ereal = S.Ereal; D.ncd = S.ncd;
        D.nfaces = (int)S.faces.size(); D.nvirt = (int)S.virt_elems.size();
        D.nreal_dof = S.nreal_dof; D.ndof = S.ndof;
        ctx->graded_ndof = S.ndof;
        D.kind = ctx->upload(S.kind);
        D.real_index = ctx->upload(S.real_index);
        D.cdof = ctx->upload(S.cdof);
        D.cdir = ctx->upload(S.cdir);
        std::vector<int> vidx(S.E, -1);
        for (size_t v = 0; v < S.virt_elems.size(); ++v) vidx[S.virt_elems[v]] = (int)v;
        D.virt_index = ctx->upload(vidx);
        D.slot_active = ctx->upload(S.slot_active);
        D.fmask = ctx->upload(S.fmask);
        Dev<double>& P64 = D.d64;
        P64.Im = ctx->upload(S.Im); P64.D1m = ctx->upload(S.D1m); P64.D2m = ctx->upload(S.D2m);
        P64.Dn = ctx->upload(S.Dn); P64.K = ctx->upload(S.K); P64.wm = ctx->upload(S.wm);
        P64.coef = ctx->upload(ctx->coef_device_order<double>(S.coef));
        D.Dn = P64.Dn;
        ctx->d_dvol = ctx->alloc<double>((size_t)S.Ereal * m * m * m);
        D.dvol = ctx->d_dvol;
        P64.trace = ctx->alloc<double>((size_t)S.E * 6 * 4 * n2);
        P64.slotres = ctx->alloc<double>((size_t)S.E * 6 * 4 * n2);
        // faces
        std::vector<int> fint;
        std::vector<double> fw, pco;
        std::vector<long long> foff;
        long long goff = 0;
        const int P = m * m;
        for (const FaceHost& F : S.faces) {
            int v[8] = {F.eA, F.fA, F.eB, F.fB, F.orient, F.nq, F.pmodeA, F.pmodeB};
            fint.insert(fint.end(), v, v + 8);
            for (int k = 0; k < MAXQ; ++k)
                for (int c = 0; c < 3; ++c) fw.push_back(k < F.nq ? F.wts[k][c] : 0.0);
            long long oa = (long long)pco.size();
            pco.insert(pco.end(), F.PA.begin(), F.PA.end());
            long long ob = (long long)pco.size();
            pco.insert(pco.end(), F.PB.begin(), F.PB.end());
            long long og = -1;
            if (F.eB < 0) { og = goff; goff += (long long)F.nq * P; }
            foff.push_back(oa); foff.push_back(ob); foff.push_back(og);
            ctx->face_goff.push_back(og);
        }
        ctx->gdata_host.assign((size_t)goff, 0.0);
        D.face_int = ctx->upload(fint);
        P64.face_w = ctx->upload(fw);
        D.face_off = ctx->upload(foff);
        P64.pcoef = ctx->upload(pco);
        ctx->face_w_host = std::move(fw);
        ctx->pcoef_host = std::move(pco);
        ctx->d_gdata = ctx->alloc<double>((size_t)goff);
        D.gdata = ctx->d_gdata;
        // preconditioner
        D.pbasis = ctx->upload(S.pbasis); D.peig = ctx->upload(S.peig);
        D.pidx = ctx->upload(S.pidx); D.pscale = ctx->upload(S.pscale); D.cinv = ctx->upload(S.cinv);
        D.cptr = ctx->upload(S.cptr); D.cidx = ctx->upload(S.cidx);
        D.cpart = ctx->alloc<double>((size_t)std::max(1, D.nvirt) * n);
        D.pk = 0;
        D.cscratch = ctx->alloc<double>((size_t)std::max(1, D.ncd));
        D.nrhs = 1;
        D.vstride = S.ndof;
        D.tstride = (long long)S.E * 6 * 4 * n2;
        // partial sums: one per element (or per workgroup of the row-split
        // block update, at most parts per element), plus the corner's
        int ugroup = 1, uparts = 1;
        update_shape(S.W, &ugroup, &uparts);
        (void)ugroup;
        D.pstride = (long long)(S.E + 2) * uparts;
        D.cpstride = (long long)std::max(1, D.nvirt) * n;
        D.csstride = std::max(1, D.ncd);
        D.part_a = ctx->alloc<double>((size_t)D.pstride);
        D.part_b = ctx->alloc<double>((size_t)D.pstride);
        D.part_c = ctx->alloc<double>((size_t)D.pstride);
        ctx->sc = ctx->alloc<Scalars>(1);
        hipcheck(hipHostMalloc((void**)&ctx->sc_host, sizeof(Scalars), hipHostMallocDefault), "hipHostMalloc");
        std::memset(ctx->sc_host, 0, sizeof(Scalars));
        ctx->d_q = ctx->alloc<double>(S.ndof);
        ctx->d_r = ctx->alloc<double>(S.ndof);
        ctx->d_z = ctx->alloc<double>(S.ndof);
        ctx->d_p = ctx->alloc<double>(S.ndof);
        ctx->d_b = ctx->alloc<double>(S.ndof);
        // error quadrature
        ctx->d_Lg = ctx->upload(S.Lg); ctx->d_Lg1 = ctx->upload(S.Lg1);
        ctx->d_eji = ctx->upload(S.err_ji); ctx->d_ew = ctx->upload(S.err_w);
        ctx->d_epart = ctx->alloc<double>(2 * (size_t)std::max(1, S.Ereal));
        (void)stream;
        hipcheck(hipDeviceSynchronize(), "sem_setup sync");
    } catch (const HipError& e) {
        delete ctx;
        return fail(SEM_EHIP, e.what());
    } catch (const std::bad_alloc&) {
        delete ctx;
        return fail(SEM_ENOMEM, "sem_setup: host allocation failed");
    } catch (const std::exception& e) {
        delete ctx;
        return fail(SEM_EINVAL, std::string("sem_setup: ") + e.what());
    }
    *out = ctx;
    return SEM_OK;
}

void sem_destroy(sem_ctx* ctx) { delete ctx; }

int64_t sem_ndof(const sem_ctx* ctx) { return ctx ? ctx->S.ndof : -1; }
int64_t sem_num_real_elements(const sem_ctx* ctx) { return ctx ? ctx->S.Ereal : -1; }
int64_t sem_num_volume_points(const sem_ctx* ctx) {
    return ctx ? (int64_t)ctx->S.Ereal * ctx->S.m * ctx->S.m * ctx->S.m : -1;
}
int64_t sem_num_dirichlet_points(const sem_ctx* ctx) {
    return ctx ? (int64_t)ctx->S.dir_faces.size() * ctx->S.m * ctx->S.m : -1;
}
int64_t sem_num_error_points(const sem_ctx* ctx) {
    return ctx ? (int64_t)ctx->S.Ereal * ctx->S.nq * ctx->S.nq * ctx->S.nq : -1;
}

sem_status sem_volume_points(const sem_ctx* ctx, double* xyz) {
    if (!ctx || !xyz) return fail(SEM_EINVAL, "sem_volume_points: NULL argument");
    std::memcpy(xyz, ctx->S.xvol.data(), ctx->S.xvol.size() * sizeof(double));
    return SEM_OK;
}

sem_status sem_dirichlet_points(const sem_ctx* ctx, double* xyz) {
    if (!ctx || !xyz) return fail(SEM_EINVAL, "sem_dirichlet_points: NULL argument");
    size_t o = 0;
    for (int fi : ctx->S.dir_faces) {
        const auto& x = ctx->S.faces[fi].xA;
        std::memcpy(xyz + o, x.data(), x.size() * sizeof(double));
        o += x.size();
    }
    return SEM_OK;
}

sem_status sem_error_points(const sem_ctx* ctx, double* xyz) {
    if (!ctx || !xyz) return fail(SEM_EINVAL, "sem_error_points: NULL argument");
    std::memcpy(xyz, ctx->S.err_x.data(), ctx->S.err_x.size() * sizeof(double));
    return SEM_OK;
}

sem_status sem_set_data(sem_ctx* ctx, const double* f, const double* g, const double* gradg) {
    if (!ctx || !f) return fail(SEM_EINVAL, "sem_set_data: NULL argument");
    HostSetup& S = ctx->S;
    const int P = S.m * S.m;
    if (!S.dir_faces.empty() && (!g || !gradg)) return fail(SEM_EINVAL, "sem_set_data: Dirichlet data missing");
    try {
        std::vector<double> d(S.svol.size());
        for (size_t i = 0; i < d.size(); ++i) d[i] = S.svol[i] * f[i];
        hipcheck(hipMemcpy(ctx->d_dvol, d.data(), d.size() * sizeof(double), hipMemcpyHostToDevice), "hipMemcpy");
        // each Dirichlet face term's data at its own offset (the Neumann
        // terms' data, sem_set_neumann_data, sits between them)
        std::vector<double>& gd = ctx->gdata_host;
        size_t pt = 0;
        for (int fi : S.dir_faces) {
            const FaceHost& F = S.faces[fi];
            const size_t og = (size_t)ctx->face_goff[fi];
            for (int k = 0; k < F.nq; ++k)
                for (int p = 0; p < P; ++p) {
                    const size_t gp = pt + p;
                    double v = 0;
                    if (F.dkind[k] == 0) v = g[gp];
                    else
                        for (int a = 0; a < 3; ++a) v += gradg[3 * gp + a] * F.ddir[((size_t)k * P + p) * 3 + a];
                    gd[og + (size_t)k * P + p] = v;
                }
            pt += P;
        }
        if (!gd.empty())
            hipcheck(hipMemcpy(ctx->d_gdata, gd.data(), gd.size() * sizeof(double), hipMemcpyHostToDevice), "hipMemcpy");
    } catch (const std::exception& e) {
        return fail(SEM_EHIP, e.what());
    }
    ctx->have_data = true;
    return SEM_OK;
}

int64_t sem_num_neumann_points(const sem_ctx* ctx) {
    return ctx ? (int64_t)ctx->S.neu_faces.size() * ctx->S.m * ctx->S.m : -1;
}

sem_status sem_neumann_points(const sem_ctx* ctx, double* xyz, double* normal) {
    if (!ctx || !xyz || !normal) return fail(SEM_EINVAL, "sem_neumann_points: NULL argument");
    const HostSetup& S = ctx->S;
    const int P = S.m * S.m;
    size_t pt = 0;
    for (int fi : S.neu_faces) {
        const FaceHost& F = S.faces[fi];
        std::memcpy(xyz + 3 * pt, F.xA.data(), (size_t)P * 3 * sizeof(double));
        std::memcpy(normal + 3 * pt, F.nuv.data(), (size_t)P * 3 * sizeof(double));
        pt += P;
    }
    return SEM_OK;
}

sem_status sem_set_neumann_data(sem_ctx* ctx, const double* h) {
    if (!ctx || !h) return fail(SEM_EINVAL, "sem_set_neumann_data: NULL argument");
    HostSetup& S = ctx->S;
    const int P = S.m * S.m;
    try {
        std::vector<double>& gd = ctx->gdata_host;
        size_t pt = 0;
        for (size_t i = 0; i < S.neu_faces.size(); ++i) {
            const size_t og = (size_t)ctx->face_goff[S.neu_faces[i]];
            for (int p = 0; p < P; ++p) gd[og + p] = S.neu_wfac[i * P + p] * h[pt + p];
            pt += P;
        }
        if (!gd.empty())
            hipcheck(hipMemcpy(ctx->d_gdata, gd.data(), gd.size() * sizeof(double), hipMemcpyHostToDevice), "hipMemcpy");
    } catch (const std::exception& e) {
        return fail(SEM_EHIP, e.what());
    }
    return SEM_OK;
}

namespace {

// q = X u (homogeneous apply): volume + faces + gather and corner reduction
void apply_X_with(const Ops& ops, sem_ctx* ctx, hipStream_t st, const double* u, double* q) {
    const DevData& D = ctx->D;
    ops.volume(st, D, u, q, 0, nullptr, nullptr, nullptr);
    ops.face(st, D, 0, nullptr);
    ops.gather(st, D, q, nullptr, ctx->sc, 0, 0);
}

void apply_X(sem_ctx* ctx, hipStream_t st, const double* u, double* q) { apply_X_with(ctx->ops, ctx, st, u, q); }

void clear_done(sem_ctx* ctx, hipStream_t st) {
    // done / status live in the scalars; zero them with a copy of a
    // host-side cleared struct (no memset nodes: safe under graph capture)
    std::memset(ctx->sc_host, 0, sizeof(Scalars));
    hipcheck(hipMemcpyAsync(ctx->sc, ctx->sc_host, sizeof(Scalars), hipMemcpyHostToDevice, st), "hipMemcpyAsync");
}

// device memory for the blocks of one assembly chunk, and for the vectors
// and traces of the columns applied at once
constexpr size_t kChunkBytes = size_t(2) << 30;
constexpr size_t kMultiBytes = size_t(3) << 29;

// Diagonal blocks of X for the element-block preconditioner, assembled with
// the operator kernels themselves (chunks of one colour's elements, one local
// index at a time), stored once per class of equal blocks, factored
// X_ee = L L^T and inverted on the device.  Temporary device memory: one
// chunk (kChunkBytes), the vectors and traces of the columns applied at once
// (kMultiBytes) and the stored blocks until they are factored.
void build_blocks(sem_ctx* ctx, hipStream_t st) {
    HostSetup& S = ctx->S;
    DevData& D = ctx->D;
    const int E = S.Ereal;
    const int n3 = S.n * S.n * S.n;
    const int ncd = S.ncd;
    // colouring of the real elements: no two elements of one colour share a face term
    std::vector<std::vector<int>> adj(E);
    for (const FaceHost& F : S.faces) {
        if (F.eB < 0) continue;
        const int a = S.real_index[F.eA], b = S.real_index[F.eB];
        if (a < 0 || b < 0) continue;
        adj[a].push_back(b);
        adj[b].push_back(a);
    }
    std::vector<int> colour(E, -1);
    int ncol = 0;
    for (int e = 0; e < E; ++e) {
        std::vector<char> used(ncol + 1, 0);
        for (int x : adj[e])
            if (colour[x] >= 0) used[colour[x]] = 1;
        int c = 0;
        while (used[c]) ++c;
        colour[e] = c;
        ncol = std::max(ncol, c + 1);
    }
    std::vector<int> order;
    std::vector<int> cptr(ncol + 1, 0);
    for (int c = 0; c < ncol; ++c) {
        for (int e = 0; e < E; ++e)
            if (colour[e] == c) order.push_back(e);
        cptr[c + 1] = (int)order.size();
    }
    std::vector<void*> tmp;
    auto talloc = [&](size_t bytes) {
        void* p = nullptr;
        if (hipMalloc(&p, std::max<size_t>(bytes, 8)) != hipSuccess) {
            (void)hipGetLastError();
            throw std::bad_alloc();            // the handler below frees tmp
        }
        tmp.push_back(p);
        return p;
    };
    const int nproj = D.nproj;
    auto tfree = [&](void* p) {
        for (auto it = tmp.begin(); it != tmp.end(); ++it)
            if (*it == p) { (void)hipFree(p); tmp.erase(it); return; }
    };
    try {
        const size_t bb = (size_t)n3 * n3;            // entries of one block
        // Assembly chunks: the elements of one colour, at most K at a time, so
        // that the temporary blocks stay within kChunkBytes (or the
        // environment's SEM_BLOCK_CHUNK_KB KiB).
        size_t chunk_bytes = kChunkBytes;
        if (const char* ev = std::getenv("SEM_BLOCK_CHUNK_KB")) {
            const long long kb = std::atoll(ev);
            if (kb > 0) chunk_bytes = (size_t)kb << 10;
        }
        const int K =
            (int)std::max<size_t>(1, std::min<size_t>((size_t)std::max(E, 1), chunk_bytes / (bb * sizeof(double))));
        std::vector<int> chb, che;                    // chunk ranges in `order`
        for (int c = 0; c < ncol; ++c)
            for (int s0 = cptr[c]; s0 < cptr[c + 1]; s0 += K) {
                chb.push_back(s0);
                che.push_back(std::min(s0 + K, cptr[c + 1]));
            }
        const int nch = (int)chb.size();
        int* d_order = (int*)talloc(order.size() * sizeof(int));
        hipcheck(hipMemcpy(d_order, order.data(), order.size() * sizeof(int), hipMemcpyHostToDevice), "copy");
        double* Bc = (double*)talloc((size_t)K * bb * sizeof(double));
        double* v = (double*)talloc((size_t)S.ndof * sizeof(double));
        double* y = (double*)talloc((size_t)S.ndof * sizeof(double));
        // the blocks of X itself: no graded projection in the applies
        D.nproj = 0;
        hipcheck(hipMemsetAsync(v, 0, (size_t)S.ndof * sizeof(double), st), "memset");
        // A column of the blocks of a chunk needs only the volume terms of the
        // chunk's elements and the face terms on their faces: the applies run
        // on those (element ids, face terms per chunk).  The other side of
        // such a face carries no unit vector, so its traces must be zero: one
        // full apply of v = 0 clears every trace first, and one restricted
        // apply of v = 0 clears a chunk's traces after it.
        std::vector<int> eid(E);
        for (int e = 0; e < S.E; ++e)
            if (S.real_index[e] >= 0) eid[S.real_index[e]] = e;
        std::vector<std::vector<int>> efaces(S.E);
        for (size_t f = 0; f < S.faces.size(); ++f) {
            efaces[S.faces[f].eA].push_back((int)f);
            if (S.faces[f].eB >= 0) efaces[S.faces[f].eB].push_back((int)f);
        }
        std::vector<int> sub_e, sub_f, fptr(nch + 1, 0);
        for (int k = 0; k < (int)order.size(); ++k) sub_e.push_back(eid[order[k]]);
        for (int h = 0; h < nch; ++h) {
            std::vector<int> fs;
            for (int k = chb[h]; k < che[h]; ++k) {
                const std::vector<int>& ef = efaces[eid[order[k]]];
                fs.insert(fs.end(), ef.begin(), ef.end());
            }
            std::sort(fs.begin(), fs.end());
            fs.erase(std::unique(fs.begin(), fs.end()), fs.end());
            sub_f.insert(sub_f.end(), fs.begin(), fs.end());
            fptr[h + 1] = (int)sub_f.size();
        }
        int* d_sube = (int*)talloc(std::max<size_t>(sub_e.size(), 1) * sizeof(int));
        int* d_subf = (int*)talloc(std::max<size_t>(sub_f.size(), 1) * sizeof(int));
        if (!sub_e.empty())
            hipcheck(hipMemcpy(d_sube, sub_e.data(), sub_e.size() * sizeof(int), hipMemcpyHostToDevice), "copy");
        if (!sub_f.empty())
            hipcheck(hipMemcpy(d_subf, sub_f.data(), sub_f.size() * sizeof(int), hipMemcpyHostToDevice), "copy");
        // graded elements: degree code per real element (-1: full degree)
        std::vector<int> gdeg(E, -1);
        for (size_t i = 0; i < ctx->proj_elem_host.size(); ++i) gdeg[ctx->proj_elem_host[i]] = ctx->proj_deg_host[i];
        int* d_pslot = (int*)talloc((size_t)K * sizeof(int));
        int* d_pdeg = (int*)talloc((size_t)K * sizeof(int));
        double* d_scale = (double*)talloc((size_t)K * sizeof(double));
        double* d_sig = (double*)talloc((size_t)K * 3 * sizeof(double));
        // Equal blocks are stored once.  Elements that are images of each
        // other under the mesh's symmetries (theta-sectors, the three edges,
        // mirror images across theta) have blocks that agree to rounding, up
        // to a reversal of some lambda axes: X_ee[a][b] = X_uu[f(a)][f(b)].
        // Each chunk's blocks are compared with the stored blocks of close
        // reversal-invariant signature (sum, sum of moduli, trace) under all
        // eight reversals at once; an unmatched block becomes a stored block
        // and the chunk's other unmatched blocks of close signature are
        // compared with it.  A match to 1e-9 relative takes the first
        // reversal that matches.  Stored blocks live in slabs of SB blocks
        // (factored slab by slab below).
        constexpr int SB = 32;
        std::vector<double*> slab;
        std::vector<double> rsig;                     // 3 per stored block
        std::vector<const double*> rptr((size_t)std::max(E, 1));
        const double** d_rptr = (const double**)talloc((size_t)std::max(E, 1) * sizeof(double*));
        int U = 0;
        std::vector<int> bidx(E, -1), bflip(E, 0);
        const double tol = 1e-9;
        std::vector<double> sig;
        auto close = [&](const double* a, const double* b2) {
            for (int k = 0; k < 3; ++k)
                if (std::fabs(a[k] - b2[k]) > tol * (std::fabs(b2[1]) + 1e-300)) return false;
            return true;
        };
        std::vector<int> trip;
        std::vector<double> cmp;
        int* d_trip = nullptr;
        double* d_cmp = nullptr;
        size_t cap_trip = 0;
        // compares the triples in trip; entry t matches when its difference is within tol
        auto run_cmp = [&]() {
            const int nt = (int)trip.size() / 3;
            if (nt == 0) return;
            if ((size_t)nt > cap_trip) {
                if (d_trip) tfree(d_trip);
                if (d_cmp) tfree(d_cmp);
                cap_trip = std::max<size_t>((size_t)nt, 2 * cap_trip);
                d_trip = (int*)talloc(cap_trip * 3 * sizeof(int));
                d_cmp = (double*)talloc(cap_trip * 2 * sizeof(double));
            }
            hipcheck(hipMemcpyAsync(d_trip, trip.data(), trip.size() * sizeof(int), hipMemcpyHostToDevice, st), "copy");
            launch_block_cmp(st, Bc, d_rptr, S.n, d_trip, nt, d_cmp);
            cmp.resize((size_t)nt * 2);
            hipcheck(hipMemcpyAsync(cmp.data(), d_cmp, cmp.size() * sizeof(double), hipMemcpyDeviceToHost, st), "copy");
            hipcheck(hipStreamSynchronize(st), "sync");
        };
        // assigns the first matching (u, c) of each chunk position in trip order
        auto take_matches = [&](int beg) {
            const int nt = (int)trip.size() / 3;
            for (int t = 0; t < nt; ++t) {
                const int e = order[beg + trip[3 * t]];
                if (bidx[e] < 0 && cmp[2 * t] <= tol * cmp[2 * t + 1]) {
                    bidx[e] = trip[3 * t + 1];
                    bflip[e] = trip[3 * t + 2];
                }
            }
        };
        // Several columns per apply: the applies of a chunk run as a multi
        // right-hand side apply, column j0 + rh in right-hand side rh, with
        // their own vectors, traces and partial sums (at most kMultiBytes),
        // about 1024 workgroups per kernel (one element apply is one
        // workgroup, so a chunk of a few hundred elements fills the GPU with
        // a few columns at once).
        const long long vs = D.vstride;
        const size_t per_rhs = (2 * (size_t)vs + 2 * (size_t)D.tstride + 3 * (size_t)D.pstride +
                                (size_t)D.cpstride + (size_t)D.csstride) * sizeof(double) + sizeof(Scalars);
        const int Rmax = (int)std::max<size_t>(1, std::min<size_t>(16, kMultiBytes / per_rhs));
        double* vR = (double*)talloc((size_t)Rmax * vs * sizeof(double));
        double* yR = (double*)talloc((size_t)Rmax * vs * sizeof(double));
        DevData Dm = D;
        Dm.d64.trace = (double*)talloc((size_t)Rmax * D.tstride * sizeof(double));
        Dm.d64.slotres = (double*)talloc((size_t)Rmax * D.tstride * sizeof(double));
        Dm.d32.trace = nullptr;
        Dm.d32.slotres = nullptr;
        Dm.part_a = (double*)talloc((size_t)3 * Rmax * D.pstride * sizeof(double));
        Dm.part_b = Dm.part_a + (size_t)Rmax * D.pstride;
        Dm.part_c = Dm.part_b + (size_t)Rmax * D.pstride;
        Dm.cpart = (double*)talloc((size_t)Rmax * std::max<long long>(D.cpstride, 1) * sizeof(double));
        Dm.cscratch = (double*)talloc((size_t)Rmax * std::max<long long>(D.csstride, 1) * sizeof(double));
        Scalars* scR = (Scalars*)talloc((size_t)Rmax * sizeof(Scalars));
        std::vector<Scalars> sc0((size_t)Rmax);
        std::memset(sc0.data(), 0, sc0.size() * sizeof(Scalars));
        hipcheck(hipMemcpyAsync(scR, sc0.data(), sc0.size() * sizeof(Scalars), hipMemcpyHostToDevice, st), "copy");
        hipcheck(hipMemsetAsync(vR, 0, (size_t)Rmax * vs * sizeof(double), st), "memset");
        auto apply_multi = [&](const DevData& Dv) {
            ctx->ops.volume(st, Dv, vR, yR, 0, nullptr, nullptr, scR);
            ctx->ops.face(st, Dv, 0, scR);
            ctx->ops.gather(st, Dv, yR, nullptr, scR, 0, 0);
        };
        Dm.nrhs = Rmax;
        apply_multi(Dm);                          // every trace of every right-hand side cleared
        for (int h = 0; h < nch; ++h) {
            const int beg = chb[h], ne = che[h] - chb[h];
            const int* el = d_order + beg;
            const int R = std::max(1, std::min(Rmax, (1024 + ne - 1) / ne));
            DevData Dc = Dm;
            Dc.nrhs = R;
            Dc.sub_elem = d_sube + beg;
            Dc.nsub_elem = ne;
            Dc.sub_face = d_subf + fptr[h];
            Dc.nsub_face = fptr[h + 1] - fptr[h];
            int j0 = 0;
            for (; j0 < n3; j0 += R) {
                launch_unit_vector(st, vR, el, ne, n3, j0, R, vs);
                apply_multi(Dc);
                launch_extract_column(st, Bc, yR, el, ne, n3, j0, R, vs);
            }
            launch_unit_clear(st, vR, el, ne, n3, j0 - R, R, vs);
            apply_multi(Dc);                      // this chunk's traces back to zero
            hipcheck(hipGetLastError(), "block assembly");
            // graded elements: the block of the projected operator on the
            // graded space, the identity scaled like the block on its
            // complement (Q X_ee Q + s (I - Q), s = tr X_ee / n3)
            std::vector<int> ps, pd;
            for (int x = 0; x < ne; ++x)
                if (gdeg[order[beg + x]] >= 0) {
                    ps.push_back(x);
                    pd.push_back(gdeg[order[beg + x]]);
                }
            if (!ps.empty()) {
                hipcheck(hipMemcpyAsync(d_pslot, ps.data(), ps.size() * sizeof(int), hipMemcpyHostToDevice, st), "copy");
                hipcheck(hipMemcpyAsync(d_pdeg, pd.data(), pd.size() * sizeof(int), hipMemcpyHostToDevice, st), "copy");
                DevData Dp = D;
                Dp.proj_elem = d_pslot;
                Dp.proj_deg = d_pdeg;
                Dp.nproj = (int)ps.size();
                ctx->ops.block_project(st, Dp, Bc, d_scale);
                hipcheck(hipGetLastError(), "graded blocks");
            }
            launch_block_sig(st, Bc, n3, ne, d_sig);
            sig.resize((size_t)ne * 3);
            hipcheck(hipMemcpyAsync(sig.data(), d_sig, sig.size() * sizeof(double), hipMemcpyDeviceToHost, st), "copy");
            hipcheck(hipStreamSynchronize(st), "sync");
            // against the stored blocks
            trip.clear();
            for (int x = 0; x < ne; ++x)
                for (int u = 0; u < U; ++u)
                    if (close(&sig[3 * x], &rsig[3 * u]))
                        for (int c = 0; c < 8; ++c) trip.insert(trip.end(), {x, u, c});
            run_cmp();
            take_matches(beg);
            // new stored blocks from the unmatched ones
            std::vector<int> pending;
            for (int x = 0; x < ne; ++x)
                if (bidx[order[beg + x]] < 0) pending.push_back(x);
            while (!pending.empty()) {
                const int x0 = pending[0];
                if (U % SB == 0) slab.push_back((double*)talloc((size_t)SB * bb * sizeof(double)));
                double* dst = slab[U / SB] + (size_t)(U % SB) * bb;
                hipcheck(hipMemcpyAsync(dst, Bc + (size_t)x0 * bb, bb * sizeof(double), hipMemcpyDeviceToDevice, st),
                         "copy");
                rptr[U] = dst;
                hipcheck(hipMemcpyAsync(d_rptr + U, &rptr[U], sizeof(double*), hipMemcpyHostToDevice, st), "copy");
                rsig.insert(rsig.end(), &sig[3 * x0], &sig[3 * x0] + 3);
                bidx[order[beg + x0]] = U;
                bflip[order[beg + x0]] = 0;
                trip.clear();
                for (size_t i = 1; i < pending.size(); ++i)
                    if (close(&sig[3 * pending[i]], &sig[3 * x0]))
                        for (int c = 0; c < 8; ++c) trip.insert(trip.end(), {pending[i], U, c});
                ++U;
                run_cmp();
                take_matches(beg);
                std::vector<int> rest;
                for (size_t i = 1; i < pending.size(); ++i)
                    if (bidx[order[beg + pending[i]]] < 0) rest.push_back(pending[i]);
                pending.swap(rest);
            }
        }
        for (void* q : {(void*)vR, (void*)yR, (void*)Dm.d64.trace, (void*)Dm.d64.slotres, (void*)Dm.part_a,
                        (void*)Dm.cpart, (void*)Dm.cscratch, (void*)scR})
            tfree(q);
        // corner block (dense, small): one unit vector per corner unknown
        std::vector<double> Xcc((size_t)ncd * ncd);
        const double one = 1.0, zero = 0.0;
        for (int c = 0; c < ncd; ++c) {
            double* vc = v + S.nreal_dof + c;
            hipcheck(hipMemcpyAsync(vc, &one, sizeof(double), hipMemcpyHostToDevice, st), "copy");
            apply_X(ctx, st, v, y);
            hipcheck(hipMemcpyAsync(Xcc.data() + (size_t)c * ncd, y + S.nreal_dof, ncd * sizeof(double),
                                    hipMemcpyDeviceToHost, st), "copy");
            hipcheck(hipMemcpyAsync(vc, &zero, sizeof(double), hipMemcpyHostToDevice, st), "copy");
            hipcheck(hipStreamSynchronize(st), "sync");
        }
        D.nproj = nproj;
        tfree(Bc);
        tfree(v);
        tfree(y);
        std::vector<int> uorder(E);
        for (int e = 0; e < E; ++e) uorder[e] = e;
        std::stable_sort(uorder.begin(), uorder.end(), [&](int a, int b2) { return bidx[a] < bidx[b2]; });
        D.bidx = ctx->upload(bidx);
        D.bflip = ctx->upload(bflip);
        D.uorder = ctx->upload(uorder);
        ctx->n_stored_blocks = U;
        {
            // tasks of the element-block update: the elements of one stored
            // block, in groups of at most G of about equal size
            int G = 1, parts = 1;
            update_shape(S.W, &G, &parts);
            std::vector<int> tf, tc, tb;
            for (int i = 0; i < E;) {
                int j = i;
                while (j < E && bidx[uorder[j]] == bidx[uorder[i]]) ++j;
                const int c = j - i, ng = (c + G - 1) / G;
                for (int g = 0, f = i; g < ng; ++g) {
                    const int cg = c / ng + (g < c % ng ? 1 : 0);
                    tf.push_back(f);
                    tc.push_back(cg);
                    tb.push_back(bidx[uorder[i]]);
                    f += cg;
                }
                i = j;
            }
            D.ntasks = (int)tf.size();
            D.task_first = ctx->upload(tf);
            D.task_count = ctx->upload(tc);
            D.task_block = ctx->upload(tb);
        }
        // Slab by slab: batched Cholesky of the stored blocks, X_ee^{-1}
        // (potri) in full symmetric storage, double and float, and from a copy
        // of the factor G = L^{-1} (trtri, the packed float fallback); then
        // whether the float-rounded inverse is still positive definite.
        // Column stride of the full storage: a multiple of 32 entries
        // (128-byte aligned stripes) with at least 3 rows past n3 (the last
        // float4 of a column).
        const int ldb = (n3 + 3 + 31) & ~31;
        D.ldb = ldb;
        const size_t P = (size_t)n3 * (n3 + 1) / 2;
        double* B64 = ctx->alloc<double>((size_t)U * n3 * ldb);
        float* B32 = ctx->alloc<float>((size_t)U * n3 * ldb);
        float* G32 = ctx->alloc<float>((size_t)U * P);
        float* G32r = ctx->alloc<float>((size_t)U * P);
        struct Handle {
            rocblas_handle h = nullptr;
            ~Handle() { if (h) rocblas_destroy_handle(h); }
        } handle;
        if (rocblas_create_handle(&handle.h) != rocblas_status_success) throw HipError("rocblas_create_handle failed");
        rocblas_handle h = handle.h;
        rocblas_set_stream(h, st);
        rocblas_int* info = (rocblas_int*)talloc((size_t)SB * sizeof(rocblas_int));
        double* L2 = (double*)talloc((size_t)SB * bb * sizeof(double));
        const rocblas_stride sa = (rocblas_stride)bb;
        std::vector<rocblas_int> hinfo(SB);
        int bad = 0;
        bool f32_spd = true, failed = false;
        // blocks of the last call whose info is nonzero; a call that failed
        // outright counts every block
        auto info_bad = [&](rocblas_status s, int nb, bool& call_failed) {
            if (s != rocblas_status_success) {
                call_failed = true;
                return nb;
            }
            hipcheck(hipMemcpyAsync(hinfo.data(), info, nb * sizeof(rocblas_int), hipMemcpyDeviceToHost, st), "copy");
            hipcheck(hipStreamSynchronize(st), "sync");
            int nz = 0;
            for (int i = 0; i < nb; ++i) nz += hinfo[i] != 0;
            return nz;
        };
        for (int sl = 0; sl < (int)slab.size() && !failed && !bad; ++sl) {
            const int u0 = sl * SB, nb = std::min(SB, U - u0);
            double* A = slab[sl];
            bad += info_bad(rocsolver_dpotrf_strided_batched(h, rocblas_fill_lower, n3, A, n3, sa, info, nb), nb, failed);
            if (failed || bad) break;
            hipcheck(hipMemcpyAsync(L2, A, (size_t)nb * bb * sizeof(double), hipMemcpyDeviceToDevice, st), "copy");
            bad += info_bad(rocsolver_dtrtri_strided_batched(h, rocblas_fill_lower, rocblas_diagonal_non_unit, n3, L2,
                                                             n3, sa, info, nb), nb, failed);
            if (failed || bad) break;
            bad += info_bad(rocsolver_dpotri_strided_batched(h, rocblas_fill_lower, n3, A, n3, sa, info, nb), nb, failed);
            if (failed || bad) break;
            const size_t of = (size_t)u0 * n3 * ldb;
            launch_pack_full64(st, A, B64 + of, ldb, n3, nb);
            launch_pack_full32(st, A, B32 + of, ldb, n3, nb);
            launch_pack_lower(st, L2, nullptr, G32 + (size_t)u0 * P, G32r + (size_t)u0 * P, n3, nb);
            launch_unpack_full(st, B32 + of, ldb, L2, n3, nb);
            hipcheck(hipGetLastError(), "pack");
            bool spd_call_failed = false;
            const int nz = info_bad(rocsolver_dpotrf_strided_batched(h, rocblas_fill_lower, n3, L2, n3, sa, info, nb),
                                    nb, spd_call_failed);
            f32_spd = f32_spd && nz == 0;
            tfree(A);
            slab[sl] = nullptr;
        }
        if (failed) throw HipError("rocsolver factorisation of the element blocks failed");
        if (bad) throw std::invalid_argument(std::to_string(bad) + " element blocks are not positive definite");
        hipcheck(hipStreamSynchronize(st), "sync");
        for (void* q : tmp) (void)hipFree(q);
        tmp.clear();
        // corner block on the host: Cholesky and inverse of its factor
        const size_t Pc = (size_t)ncd * (ncd + 1) / 2;
        std::vector<double> L((size_t)ncd * ncd, 0.0), Gi((size_t)ncd * ncd, 0.0);
        for (int j = 0; j < ncd; ++j) {
            double d = Xcc[(size_t)j * ncd + j];
            for (int k = 0; k < j; ++k) d -= L[(size_t)j * ncd + k] * L[(size_t)j * ncd + k];
            if (!(d > 0)) throw std::invalid_argument("corner block is not positive definite");
            const double ljj = std::sqrt(d);
            L[(size_t)j * ncd + j] = ljj;
            for (int i = j + 1; i < ncd; ++i) {
                double v2 = 0.5 * (Xcc[(size_t)j * ncd + i] + Xcc[(size_t)i * ncd + j]);
                for (int k = 0; k < j; ++k) v2 -= L[(size_t)i * ncd + k] * L[(size_t)j * ncd + k];
                L[(size_t)i * ncd + j] = v2 / ljj;
            }
        }
        for (int j = 0; j < ncd; ++j) {          // column j of L^{-1}: forward substitution
            for (int i = j; i < ncd; ++i) {
                double v2 = (i == j) ? 1.0 : 0.0;
                for (int k = j; k < i; ++k) v2 -= L[(size_t)i * ncd + k] * Gi[(size_t)k * ncd + j];
                Gi[(size_t)i * ncd + j] = v2 / L[(size_t)i * ncd + i];
            }
        }
        std::vector<double> gc(Pc);
        std::vector<float> gcf(Pc);
        size_t o = 0;
        for (int j = 0; j < ncd; ++j)
            for (int i = j; i < ncd; ++i, ++o) {
                gc[o] = Gi[(size_t)i * ncd + j];
                gcf[o] = (float)gc[o];
            }
        D.B64 = B64;
        D.B32 = B32;
        if (f32_spd) {
            // the float inverse serves the mixed path: its factor is not needed
            ctx->release(G32);
            ctx->release(G32r);
            G32 = G32r = nullptr;
        }
        D.G32 = G32;
        D.G32r = G32r;
        ctx->mixed_pk = f32_spd ? 3 : 2;
        D.Gc64 = ctx->upload(gc);
        D.Gc32 = ctx->upload(gcf);
    } catch (...) {
        D.nproj = nproj;
        D.sub_elem = nullptr;
        D.sub_face = nullptr;
        for (void* q : tmp) (void)hipFree(q);
        throw;
    }
    ctx->have_blocks = true;
}

}  // namespace

sem_status sem_set_preconditioner(sem_ctx* ctx, int kind, void* stream) {
    if (!ctx) return fail(SEM_EINVAL, "sem_set_preconditioner: NULL context");
    if (kind != SEM_PRECOND_SEPARABLE && kind != SEM_PRECOND_ELEMENT_BLOCK)
        return fail(SEM_EINVAL, "sem_set_preconditioner: unknown kind");
    hipStream_t st = (hipStream_t)stream;
    try {
        if (kind == SEM_PRECOND_ELEMENT_BLOCK && !ctx->have_blocks) {
            clear_done(ctx, st);
            build_blocks(ctx, st);
        }
        ctx->D.pk = (kind == SEM_PRECOND_ELEMENT_BLOCK) ? 1 : 0;
    } catch (const std::bad_alloc&) {
        return fail(SEM_ENOMEM, "sem_set_preconditioner: device memory for the element blocks");
    } catch (const std::invalid_argument& e) {
        return fail(SEM_EINVAL, std::string("sem_set_preconditioner: ") + e.what());
    } catch (const std::exception& e) {
        return fail(SEM_EHIP, e.what());
    }
    return SEM_OK;
}

sem_status sem_rhs(sem_ctx* ctx, double* b, void* stream) {
    if (!ctx || !b) return fail(SEM_EINVAL, "sem_rhs: NULL argument");
    if (!ctx->have_data) return fail(SEM_ENODATA, "sem_rhs: call sem_set_data first");
    hipStream_t st = (hipStream_t)stream;
    try {
        const DevData& D = ctx->D;
        clear_done(ctx, st);
        ctx->ops.volume(st, D, nullptr, b, 1, nullptr, nullptr, nullptr);
        ctx->ops.face(st, D, 1, nullptr);
        ctx->ops.gather(st, D, b, nullptr, ctx->sc, 0, 1);
        hipcheck(hipMemcpyAsync(ctx->d_b, b, D.ndof * sizeof(double), hipMemcpyDeviceToDevice, st), "copy b");
        hipcheck(hipGetLastError(), "sem_rhs launch");
    } catch (const std::exception& e) {
        return fail(SEM_EHIP, e.what());
    }
    return SEM_OK;
}

sem_status sem_residual(sem_ctx* ctx, const double* u, double* r, int homogeneous, void* stream) {
    return sem_residual_prec(ctx, u, r, homogeneous, SEM_FP64, stream);
}

sem_status sem_residual_prec(sem_ctx* ctx, const double* u, double* r, int homogeneous, int precision,
                             void* stream) {
    if (!ctx || !u || !r) return fail(SEM_EINVAL, "sem_residual: NULL argument");
    if (u == r) return fail(SEM_EINVAL, "sem_residual: u and r alias");
    if (precision != SEM_FP64 && precision != SEM_MIXED_FP32) return fail(SEM_EINVAL, "sem_residual: bad precision");
    if (!homogeneous && !ctx->have_data) return fail(SEM_ENODATA, "sem_residual: no data");
    hipStream_t st = (hipStream_t)stream;
    try {
        clear_done(ctx, st);
        if (precision == SEM_MIXED_FP32) {
            ctx->ensure_fp32();
            apply_X_with(ctx->ops32, ctx, st, u, r);
        } else {
            apply_X(ctx, st, u, r);
        }
        if (!homogeneous) launch_sub(st, r, r, ctx->d_b, ctx->D.ndof);
        hipcheck(hipGetLastError(), "sem_residual launch");
    } catch (const std::exception& e) {
        return fail(SEM_EHIP, e.what());
    }
    return SEM_OK;
}

sem_status sem_precond(sem_ctx* ctx, const double* r, double* z, void* stream) {
    if (!ctx || !r || !z) return fail(SEM_EINVAL, "sem_precond: NULL argument");
    hipStream_t st = (hipStream_t)stream;
    try {
        clear_done(ctx, st);
        ctx->ops.update(st, ctx->D, 2, nullptr, const_cast<double*>(r), z, nullptr, nullptr, nullptr, ctx->sc);
        hipcheck(hipGetLastError(), "sem_precond launch");
    } catch (const std::exception& e) {
        return fail(SEM_EHIP, e.what());
    }
    return SEM_OK;
}

namespace {
void ensure_source(sem_ctx* ctx) {
    if (ctx->d_xvol) return;
    ctx->d_xvol = ctx->upload(ctx->S.xvol);
    ctx->d_svol = ctx->upload(ctx->S.svol);
    ctx->d_zq = ctx->alloc<double>(ctx->S.svol.size());
    ctx->d_spart = ctx->alloc<double>((size_t)std::max(1, ctx->S.Ereal) * SOURCE_MAXDEG * SOURCE_MAXDEG * SOURCE_MAXDEG);
}
}  // namespace

sem_status sem_set_source_legendre(sem_ctx* ctx, int deg, const double* theta, void* stream) {
    if (!ctx || !theta) return fail(SEM_EINVAL, "sem_set_source_legendre: NULL argument");
    if (deg < 1 || deg > SOURCE_MAXDEG) return fail(SEM_EINVAL, "sem_set_source_legendre: deg must be 1..12");
    hipStream_t st = (hipStream_t)stream;
    try {
        ensure_source(ctx);
        const long long npts = (long long)ctx->S.svol.size();
        launch_source_eval(st, ctx->d_xvol, ctx->d_svol, theta, deg, npts, ctx->d_dvol);
        // homogeneous Dirichlet data
        size_t ng = 0;
        for (int fi : ctx->S.dir_faces) ng += (size_t)ctx->S.faces[fi].nq * ctx->S.m * ctx->S.m;
        if (ng) hipcheck(hipMemsetAsync(ctx->d_gdata, 0, ng * sizeof(double), st), "memset");
        hipcheck(hipGetLastError(), "source launch");
    } catch (const std::exception& e) {
        return fail(SEM_EHIP, e.what());
    }
    ctx->have_data = true;
    return SEM_OK;
}

sem_status sem_set_source_fourier(sem_ctx* ctx, int nmodes, const double* coef, void* stream) {
    if (!ctx || !coef || nmodes < 1) return fail(SEM_EINVAL, "sem_set_source_fourier: bad argument");
    hipStream_t st = (hipStream_t)stream;
    try {
        ensure_source(ctx);
        const long long npts = (long long)ctx->S.svol.size();
        launch_source_fourier(st, ctx->d_xvol, ctx->d_svol, coef, nmodes, npts, ctx->d_dvol);
        size_t ng = 0;
        for (int fi : ctx->S.dir_faces) ng += (size_t)ctx->S.faces[fi].nq * ctx->S.m * ctx->S.m;
        if (ng) hipcheck(hipMemsetAsync(ctx->d_gdata, 0, ng * sizeof(double), st), "memset");
        hipcheck(hipGetLastError(), "source launch");
    } catch (const std::exception& e) {
        return fail(SEM_EHIP, e.what());
    }
    ctx->have_data = true;
    return SEM_OK;
}

sem_status sem_source_adjoint(sem_ctx* ctx, int deg, const double* lambda, double* grad, void* stream) {
    if (!ctx || !lambda || !grad) return fail(SEM_EINVAL, "sem_source_adjoint: NULL argument");
    if (deg < 1 || deg > SOURCE_MAXDEG) return fail(SEM_EINVAL, "sem_source_adjoint: deg must be 1..12");
    hipStream_t st = (hipStream_t)stream;
    try {
        ensure_source(ctx);
        clear_done(ctx, st);
        const int m3 = ctx->S.m * ctx->S.m * ctx->S.m;
        ctx->ops.volume(st, ctx->D, lambda, ctx->d_q, 3, nullptr, ctx->d_zq, nullptr);
        launch_source_project(st, ctx->d_xvol, ctx->d_svol, ctx->d_zq, deg, m3, ctx->S.Ereal, ctx->d_spart, grad);
        hipcheck(hipGetLastError(), "adjoint launch");
    } catch (const std::exception& e) {
        return fail(SEM_EHIP, e.what());
    }
    return SEM_OK;
}

namespace {

// the status of a solve that did not converge, with its message
sem_status fail_pcg(sem_status s, bool floor) {
    if (s == SEM_ENOCONV && floor)
        return fail(s, "PCG: the true residual stopped decreasing above rtol (attainable accuracy)");
    if (s == SEM_ENOCONV) return fail(s, "PCG: maxit reached");
    if (s == SEM_EBREAKDOWN) return fail(s, "PCG: breakdown (non-positive curvature)");
    if (s == SEM_ENAN) return fail(s, "PCG: NaN or Inf");
    return fail(s, "PCG: failed");
}

// The batched PCG loop over contexts and right-hand sides (arguments checked
// by the caller).  f32: float operator contractions with the float element
// blocks (the inner solves of the mixed batch), else FP64.
sem_status batch_pcg(int nctx, sem_ctx* const* ctxs, const int* nrhs, const double* const* b, double* const* u,
                     double rtol, int maxit, int check, bool f32, sem_pcg_info* infos, hipStream_t st) {
    hipStream_t cs = nullptr;
    hipEvent_t ev = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    int sync_dev = -1;
    try {
        hipcheck(hipGetDevice(&sync_dev), "hipGetDevice");
        std::vector<DevData> Dv(nctx);
        for (int c = 0; c < nctx; ++c) {
            sem_ctx* x = ctxs[c];
            const int R = nrhs[c];
            x->ensure_multi(R);
            Dv[c] = x->multi_view(R, f32);
            std::memset(x->m_sc_host, 0, (size_t)R * sizeof(Scalars));
            for (int k = 0; k < R; ++k) { x->m_sc_host[k].tol = rtol; x->m_sc_host[k].maxit = maxit; }
            hipcheck(hipMemcpyAsync(x->m_sc, x->m_sc_host, (size_t)R * sizeof(Scalars), hipMemcpyHostToDevice, st),
                     "scalars");
            const Ops& o = f32 ? x->ops32 : x->ops;
            // r = b - X u0, z = W^-1 r, p = z for every right-hand side
            o.volume(st, Dv[c], u[c], x->m_q, 0, nullptr, nullptr, x->m_sc);
            o.face(st, Dv[c], 0, x->m_sc);
            o.gather(st, Dv[c], x->m_q, nullptr, x->m_sc, 0, 0);
            x->ops.update(st, Dv[c], 0, u[c], x->m_r, x->m_z, x->m_p, x->m_q, b[c], x->m_sc);
        }
        hipcheck(hipGetLastError(), "batch init");
        // one graph: `check` iterations of every context and right-hand side
        hipcheck(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking), "hipStreamCreate");
        hipcheck(hipEventCreateWithFlags(&ev, hipEventDisableTiming), "hipEventCreate");
        hipcheck(hipEventRecord(ev, st), "event");
        hipcheck(hipStreamWaitEvent(cs, ev, 0), "wait");
        hipcheck(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal), "begin capture");
        for (int k = 0; k < check; ++k)
            for (int c = 0; c < nctx; ++c) {
                sem_ctx* x = ctxs[c];
                const Ops& o = f32 ? x->ops32 : x->ops;
                o.volume(cs, Dv[c], x->m_p, x->m_q, 2, x->m_z, x->m_p, x->m_sc);
                o.face(cs, Dv[c], 0, x->m_sc);
                o.gather(cs, Dv[c], x->m_q, x->m_p, x->m_sc, 1, 0);
                x->ops.update(cs, Dv[c], 1, u[c], x->m_r, x->m_z, x->m_p, x->m_q, b[c], x->m_sc);
            }
        hipcheck(hipStreamEndCapture(cs, &graph), "end capture");
        hipcheck(hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0), "instantiate");
        for (int it = 0; it < maxit + check;) {
            hipcheck(hipGraphLaunch(exec, cs), "graph launch");
            it += check;
            for (int c = 0; c < nctx; ++c)
                hipcheck(hipMemcpyAsync(ctxs[c]->m_sc_host, ctxs[c]->m_sc, (size_t)nrhs[c] * sizeof(Scalars),
                                        hipMemcpyDeviceToHost, cs), "scalars");
            hipcheck(hipStreamSynchronize(cs), "sync");
            bool all = true;
            for (int c = 0; c < nctx && all; ++c)
                for (int k = 0; k < nrhs[c]; ++k) all = all && ctxs[c]->m_sc_host[k].done;
            if (all) break;
        }
        hipcheck(hipEventRecord(ev, cs), "event");
        hipcheck(hipStreamWaitEvent(st, ev, 0), "wait");
        hipcheck(hipStreamSynchronize(st), "sync");
    } catch (const std::bad_alloc&) {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        if (cs) (void)hipStreamDestroy(cs);
        if (ev) (void)hipEventDestroy(ev);
        return fail(SEM_ENOMEM, "PCG: device memory for the right-hand side work buffers");
    } catch (const std::exception& e) {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        if (cs) (void)hipStreamDestroy(cs);
        if (ev) (void)hipEventDestroy(ev);
        return fail(SEM_EHIP, e.what());
    }
    (void)hipGraphExecDestroy(exec);
    (void)hipGraphDestroy(graph);
    (void)hipStreamDestroy(cs);
    (void)hipEventDestroy(ev);
    sem_status worst = SEM_OK;
    int o = 0;
    for (int c = 0; c < nctx; ++c)
        for (int k = 0; k < nrhs[c]; ++k, ++o) {
            const Scalars& h = ctxs[c]->m_sc_host[k];
            int status = h.status;
            if (status == 0 && !h.done) status = SEM_ENOCONV;
            infos[o].iterations = h.iter;
            infos[o].outer = 1;
            infos[o].rel_residual = h.relres;
            infos[o].status = status;
            if (status != 0 && worst == SEM_OK) worst = (sem_status)status;
        }
    if (worst != SEM_OK) return fail(worst, "sem_pcg_solve_batch: some right-hand sides did not converge");
    return SEM_OK;
}


// Batched mixed-precision PCG: the iterations of every context run with the
// float operator in one graph; between replays the host applies, per
// context, the residual replacement rule of sem_pcg_solve_mixed to all its
// right-hand sides at once (one eager iteration whose residual is recomputed
// in FP64), and a context that stalls is switched to its FP64 operator (the
// graph is captured again).
sem_status batch_mixed(int nctx, sem_ctx* const* ctxs, const int* nrhs, const double* const* b, double* const* u,
                       double rtol, int maxit, int check, sem_pcg_info* infos, hipStream_t st) {
    struct CtxState {
        bool escalated = false, stalled = false;
        std::vector<double> last_true, last_req;  // true residual at the last replacement / last requested one
        std::vector<int> seg_start, prev_seg, floor_hits, outer;
        std::vector<char> confirmed, requested;
    };
    std::vector<CtxState> cs_(nctx);
    bool any_floor = false;
    std::vector<DevData> D64(nctx), D32(nctx), Dm64(nctx);
    hipStream_t cs = nullptr;
    hipEvent_t ev = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    auto drop_graph = [&]() {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        exec = nullptr;
        graph = nullptr;
    };
    auto cleanup = [&]() {
        drop_graph();
        if (cs) (void)hipStreamDestroy(cs);
        if (ev) (void)hipEventDestroy(ev);
    };
    try {
        for (int c = 0; c < nctx; ++c) {
            sem_ctx* x = ctxs[c];
            const int R = nrhs[c];
            x->ensure_fp32();
            x->ensure_multi(R);
            D64[c] = x->multi_view(R, false);
            D32[c] = x->multi_view(R, true);
            Dm64[c] = D64[c];                       // FP64 operator with the float blocks
            if (Dm64[c].pk == 1) Dm64[c].pk = x->mixed_pk;
            CtxState& S = cs_[c];
            S.last_true.assign(R, 1.0);
            S.last_req.assign(R, 1.0);
            S.requested.assign(R, 0);
            S.seg_start.assign(R, 0);
            S.prev_seg.assign(R, 0);
            S.floor_hits.assign(R, 0);
            S.outer.assign(R, 0);
            S.confirmed.assign(R, 0);
            std::memset(x->m_sc_host, 0, (size_t)R * sizeof(Scalars));
            for (int k = 0; k < R; ++k) { x->m_sc_host[k].tol = rtol; x->m_sc_host[k].maxit = maxit; }
            hipcheck(hipMemcpyAsync(x->m_sc, x->m_sc_host, (size_t)R * sizeof(Scalars), hipMemcpyHostToDevice, st),
                     "scalars");
            // FP64 start: r = b - X u0, z = W^-1 r, p = z
            x->ops.volume(st, D64[c], u[c], x->m_q, 0, nullptr, nullptr, x->m_sc);
            x->ops.face(st, D64[c], 0, x->m_sc);
            x->ops.gather(st, D64[c], x->m_q, nullptr, x->m_sc, 0, 0);
            x->ops.update(st, Dm64[c], 0, u[c], x->m_r, x->m_z, x->m_p, x->m_q, b[c], x->m_sc);
            hipcheck(hipMemcpyAsync(x->m_sc_host, x->m_sc, (size_t)R * sizeof(Scalars), hipMemcpyDeviceToHost, st),
                     "scalars");
        }
        hipcheck(hipStreamSynchronize(st), "sync");
        for (int c = 0; c < nctx; ++c)
            for (int k = 0; k < nrhs[c]; ++k) {
                const Scalars& h = ctxs[c]->m_sc_host[k];
                cs_[c].last_true[k] = cs_[c].last_req[k] = h.relres;
                if (h.done && h.status == 0) cs_[c].confirmed[k] = 1;
            }
        hipcheck(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking), "hipStreamCreate");
        hipcheck(hipEventCreateWithFlags(&ev, hipEventDisableTiming), "hipEventCreate");
        hipcheck(hipEventRecord(ev, st), "event");
        hipcheck(hipStreamWaitEvent(cs, ev, 0), "wait");
        auto capture = [&]() {
            drop_graph();
            hipcheck(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal), "begin capture");
            for (int it = 0; it < check; ++it)
                for (int c = 0; c < nctx; ++c) {
                    sem_ctx* x = ctxs[c];
                    const bool e64 = cs_[c].escalated;
                    const Ops& o = e64 ? x->ops : x->ops32;
                    const DevData& Dq = e64 ? D64[c] : D32[c];
                    o.volume(cs, Dq, x->m_p, x->m_q, 2, x->m_z, x->m_p, x->m_sc);
                    o.face(cs, Dq, 0, x->m_sc);
                    o.gather(cs, Dq, x->m_q, x->m_p, x->m_sc, 1, 0);
                    x->ops.update(cs, e64 ? D64[c] : Dm64[c], 1, u[c], x->m_r, x->m_z, x->m_p, x->m_q, b[c],
                                  x->m_sc);
                }
            hipcheck(hipStreamEndCapture(cs, &graph), "end capture");
            hipcheck(hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0), "instantiate");
        };
        capture();
        const double delta = 0.1;
        int guard = 0;
        while (guard++ < 4 * (maxit / check + 2) + 64) {
            hipcheck(hipGraphLaunch(exec, cs), "graph launch");
            for (int c = 0; c < nctx; ++c)
                hipcheck(hipMemcpyAsync(ctxs[c]->m_sc_host, ctxs[c]->m_sc, (size_t)nrhs[c] * sizeof(Scalars),
                                        hipMemcpyDeviceToHost, cs), "scalars");
            hipcheck(hipStreamSynchronize(cs), "sync");
            bool all_done = true, recapture = false;
            for (int c = 0; c < nctx; ++c) {
                sem_ctx* x = ctxs[c];
                CtxState& S = cs_[c];
                const int R = nrhs[c];
                bool need = false;
                for (int k = 0; k < R; ++k) {
                    const Scalars& h = x->m_sc_host[k];
                    x->m_op_host[k] = 0;
                    S.requested[k] = 0;
                    if (h.status != 0 || S.confirmed[k]) continue;
                    all_done = false;
                    if (h.done) {
                        S.requested[k] = 1;          // recursive residual met rtol: confirm in FP64
                        x->m_op_host[k] = 1;
                    } else if (!S.escalated && h.relres < delta * S.last_true[k]) {
                        S.requested[k] = 1;
                    } else if (h.iter - S.seg_start[k] > 2 * std::max(S.prev_seg[k], 50)) {
                        S.requested[k] = 1;
                        S.stalled = true;
                    }
                    need = need || S.requested[k];
                }
                if (!need) continue;
                // one iteration for all right-hand sides of the context whose
                // residual is recomputed in FP64
                hipcheck(hipMemcpyAsync(x->m_op, x->m_op_host, R * sizeof(int), hipMemcpyHostToDevice, cs), "op");
                launch_flag_ops(cs, x->m_sc, x->m_op, R);
                const bool e64 = S.escalated;
                const Ops& o = e64 ? x->ops : x->ops32;
                const DevData& Dq = e64 ? D64[c] : D32[c];
                o.volume(cs, Dq, x->m_p, x->m_q, 2, x->m_z, x->m_p, x->m_sc);
                o.face(cs, Dq, 0, x->m_sc);
                o.gather(cs, Dq, x->m_q, x->m_p, x->m_sc, 1, 0);
                launch_axpy_alpha_multi(cs, u[c], x->m_p, x->m_sc, x->D.ndof, R);
                x->ops.volume(cs, D64[c], u[c], x->m_q, 0, nullptr, nullptr, x->m_sc);
                x->ops.face(cs, D64[c], 0, x->m_sc);
                x->ops.gather(cs, D64[c], x->m_q, nullptr, x->m_sc, 0, 0);
                x->ops.update(cs, e64 ? D64[c] : Dm64[c], 3, u[c], x->m_r, x->m_z, x->m_p, x->m_q, b[c], x->m_sc);
                hipcheck(hipMemcpyAsync(x->m_sc_host, x->m_sc, (size_t)R * sizeof(Scalars), hipMemcpyDeviceToHost, cs),
                         "scalars");
                hipcheck(hipStreamSynchronize(cs), "sync");
                // the gain and stall judgments concern the right-hand sides that
                // asked for this replacement; the others only refresh their
                // true residual
                bool escalate = S.stalled, floor_stop = false;
                for (int k = 0; k < R; ++k) {
                    const Scalars& h = x->m_sc_host[k];
                    x->m_op_host[k] = 0;
                    if (h.status != 0 || S.confirmed[k]) continue;
                    S.outer[k] += 1;
                    S.last_true[k] = h.relres;
                    if (h.done) {
                        S.confirmed[k] = 1;          // converged on the true residual
                        continue;
                    }
                    if (!S.requested[k]) {
                        // refreshed by another right-hand side's replacement.
                        // Every refresh moves this one's target (delta times the
                        // refreshed residual), so with many right-hand sides it
                        // may never ask on its own: a true gain of 2x since its
                        // last request starts a new segment, and the stall test
                        // counts only iterations without such a gain.
                        if (h.relres < 0.5 * S.last_req[k]) {
                            S.seg_start[k] = h.iter;
                            S.last_req[k] = h.relres;
                        }
                        continue;
                    }
                    if (!e64 && h.relres > 0.5 * S.last_req[k]) {
                        escalate = true;
                    } else if (e64 && h.relres > 0.5 * S.last_req[k] && ++S.floor_hits[k] >= 2) {
                        x->m_op_host[k] = 2;          // attainable accuracy reached above rtol
                        floor_stop = true;
                        any_floor = true;
                    }
                    S.prev_seg[k] = h.iter - S.seg_start[k];
                    S.seg_start[k] = h.iter;
                    S.last_req[k] = h.relres;
                }
                S.stalled = false;
                if (floor_stop) {
                    hipcheck(hipMemcpyAsync(x->m_op, x->m_op_host, R * sizeof(int), hipMemcpyHostToDevice, cs), "op");
                    launch_flag_ops(cs, x->m_sc, x->m_op, R);
                }
                if (escalate && !e64) {
                    S.escalated = true;
                    recapture = true;
                }
            }
            hipcheck(hipGetLastError(), "batch launch");
            if (all_done) break;
            if (recapture) capture();
        }
        for (int c = 0; c < nctx; ++c)
            hipcheck(hipMemcpyAsync(ctxs[c]->m_sc_host, ctxs[c]->m_sc, (size_t)nrhs[c] * sizeof(Scalars),
                                    hipMemcpyDeviceToHost, cs), "scalars");
        hipcheck(hipEventRecord(ev, cs), "event");
        hipcheck(hipStreamWaitEvent(st, ev, 0), "wait");
        hipcheck(hipStreamSynchronize(st), "sync");
    } catch (const std::bad_alloc&) {
        cleanup();
        return fail(SEM_ENOMEM, "PCG: device memory for the right-hand side work buffers");
    } catch (const std::invalid_argument& e) {
        cleanup();
        return fail(SEM_EINVAL, std::string("sem_pcg_solve_batch: ") + e.what());
    } catch (const std::exception& e) {
        cleanup();
        return fail(SEM_EHIP, e.what());
    }
    cleanup();
    sem_status worst = SEM_OK;
    int o = 0;
    for (int c = 0; c < nctx; ++c)
        for (int k = 0; k < nrhs[c]; ++k, ++o) {
            const Scalars& h = ctxs[c]->m_sc_host[k];
            int status = h.status;
            if (status == 0 && !cs_[c].confirmed[k]) status = SEM_ENOCONV;
            infos[o].iterations = h.iter;
            infos[o].outer = cs_[c].outer[k];
            infos[o].rel_residual = h.relres;
            infos[o].status = status;
            if (status != 0 && worst == SEM_OK) worst = (sem_status)status;
        }
    if (worst != SEM_OK) return fail_pcg(worst, any_floor);
    return SEM_OK;
}

}  // namespace

sem_status sem_pcg_solve_batch(int nctx, sem_ctx* const* ctxs, const int* nrhs, const double* const* b,
                               double* const* u, double rtol, int maxit, int check, int precision,
                               sem_pcg_info* infos, void* stream) {
    if (nctx <= 0 || !ctxs || !nrhs || !b || !u || !infos) return fail(SEM_EINVAL, "sem_pcg_solve_batch: bad argument");
    if (maxit < 0 || !(rtol >= 0) || check < 1 || check > 1024)
        return fail(SEM_EINVAL, "sem_pcg_solve_batch: bad rtol, maxit or check");
    if (precision != SEM_FP64 && precision != SEM_MIXED_FP32) return fail(SEM_EINVAL, "sem_pcg_solve_batch: bad precision");
    for (int c = 0; c < nctx; ++c)
        if (!ctxs[c] || nrhs[c] < 1 || !b[c] || !u[c]) return fail(SEM_EINVAL, "sem_pcg_solve_batch: bad context entry");
    hipStream_t st = (hipStream_t)stream;
    if (precision == SEM_FP64) return batch_pcg(nctx, ctxs, nrhs, b, u, rtol, maxit, check, false, infos, st);
    return batch_mixed(nctx, ctxs, nrhs, b, u, rtol, maxit, check, infos, st);
}

// single solves: a batch of one context and one right-hand side (the same
// kernels and arithmetic, launched through the same graph)
sem_status sem_pcg_solve(sem_ctx* ctx, const double* b, double* u, double rtol, int maxit, sem_pcg_info* info,
                         void* stream) {
    if (!ctx || !b || !u) return fail(SEM_EINVAL, "sem_pcg_solve: NULL argument");
    if (maxit < 0 || !(rtol >= 0)) return fail(SEM_EINVAL, "sem_pcg_solve: bad rtol or maxit");
    sem_pcg_info tmp{};
    const int one = 1;
    return batch_pcg(1, &ctx, &one, &b, &u, rtol, maxit, 8, false, info ? info : &tmp, (hipStream_t)stream);
}

sem_status sem_pcg_solve_mixed(sem_ctx* ctx, const double* b, double* u, double rtol, int maxit,
                               sem_pcg_info* info, void* stream) {
    if (!ctx || !b || !u) return fail(SEM_EINVAL, "sem_pcg_solve_mixed: NULL argument");
    if (maxit < 0 || !(rtol >= 0)) return fail(SEM_EINVAL, "sem_pcg_solve_mixed: bad rtol or maxit");
    sem_pcg_info tmp{};
    const int one = 1;
    return batch_mixed(1, &ctx, &one, &b, &u, rtol, maxit, 8, info ? info : &tmp, (hipStream_t)stream);
}

sem_status sem_error(sem_ctx* ctx, const double* u, const double* uex, const double* gex, double* rel_h1,
                     void* stream) {
    if (!ctx || !u || !uex || !gex || !rel_h1) return fail(SEM_EINVAL, "sem_error: NULL argument");
    hipStream_t st = (hipStream_t)stream;
    HostSetup& S = ctx->S;
    try {
        const size_t npts = (size_t)S.Ereal * S.nq * S.nq * S.nq;
        double* d_uex = nullptr;
        double* d_gex = nullptr;
        hipcheck(hipMalloc(&d_uex, npts * sizeof(double)), "hipMalloc");
        hipcheck(hipMalloc(&d_gex, 3 * npts * sizeof(double)), "hipMalloc");
        hipcheck(hipMemcpy(d_uex, uex, npts * sizeof(double), hipMemcpyHostToDevice), "hipMemcpy");
        hipcheck(hipMemcpy(d_gex, gex, 3 * npts * sizeof(double), hipMemcpyHostToDevice), "hipMemcpy");
        ctx->ops.error(st, ctx->D, u, S.nq, ctx->d_Lg, ctx->d_Lg1, ctx->d_eji, ctx->d_ew, d_uex, d_gex, ctx->d_epart);
        hipcheck(hipGetLastError(), "sem_error launch");
        std::vector<double> part(2 * (size_t)S.Ereal);
        hipcheck(hipMemcpyAsync(part.data(), ctx->d_epart, part.size() * sizeof(double), hipMemcpyDeviceToHost, st),
                 "hipMemcpy");
        hipcheck(hipStreamSynchronize(st), "sync");
        (void)hipFree(d_uex);
        (void)hipFree(d_gex);
        double num = 0, den = 0;
        for (int r = 0; r < S.Ereal; ++r) { num += part[2 * r]; den += part[2 * r + 1]; }
        *rel_h1 = den > 0 ? std::sqrt(num / den) : 0.0;
    } catch (const std::exception& e) {
        return fail(SEM_EHIP, e.what());
    }
    return SEM_OK;
}

sem_status sem_set_coefficients(sem_ctx* ctx, const double* a, const double* beta, const double* c) {
    if (!ctx) return fail(SEM_EINVAL, "sem_set_coefficients: NULL context");
    HostSetup& S = ctx->S;
    if (!S.neu_faces.empty() && a)
        return fail(SEM_EINVAL, "sem_set_coefficients: a general a with Neumann faces (their conormal needs a on the faces)");
    try {
        const size_t npts = S.svol.size();
        if (a)
            for (size_t p = 0; p < npts; ++p) {
                const double* ap = a + 6 * p;
                // strong ellipticity at every point: a positive definite
                const double d1 = ap[0], d2 = ap[0] * ap[1] - ap[3] * ap[3];
                const double d3 = ap[0] * (ap[1] * ap[2] - ap[5] * ap[5]) - ap[3] * (ap[3] * ap[2] - ap[5] * ap[4]) +
                                  ap[4] * (ap[3] * ap[5] - ap[1] * ap[4]);
                if (!(d1 > 0 && d2 > 0 && d3 > 0))
                    return fail(SEM_EINVAL, "sem_set_coefficients: a is not positive definite at volume point " +
                                                std::to_string(p));
            }
        volume_fields(S, a, beta, c);
        DevData& D = ctx->D;
        const std::vector<double> c64 = ctx->coef_device_order<double>(S.coef);
        hipcheck(hipMemcpy(const_cast<double*>(D.d64.coef), c64.data(), c64.size() * sizeof(double),
                           hipMemcpyHostToDevice), "hipMemcpy");
        hipcheck(hipMemcpy(const_cast<unsigned*>(D.fmask), S.fmask.data(), S.fmask.size() * sizeof(unsigned),
                           hipMemcpyHostToDevice), "hipMemcpy");
        if (ctx->have32) {
            const std::vector<float> f32 = ctx->coef_device_order<float>(S.coef);
            hipcheck(hipMemcpy(const_cast<float*>(D.d32.coef), f32.data(), f32.size() * sizeof(float),
                               hipMemcpyHostToDevice), "hipMemcpy");
        }
        // element blocks of the previous operator no longer apply
        if (ctx->have_blocks) {
            ctx->have_blocks = false;
            D.pk = 0;
        }
    } catch (const std::exception& e) {
        return fail(SEM_EHIP, std::string("sem_set_coefficients: ") + e.what());
    }
    return SEM_OK;
}

int64_t sem_num_face_terms(const sem_ctx* ctx) { return ctx ? (int64_t)ctx->S.faces.size() : -1; }

sem_status sem_face_weights(const sem_ctx* ctx, double* w) {
    if (!ctx || !w) return fail(SEM_EINVAL, "sem_face_weights: NULL argument");
    std::memcpy(w, ctx->face_w_host.data(), ctx->face_w_host.size() * sizeof(double));
    return SEM_OK;
}

sem_status sem_set_face_weights(sem_ctx* ctx, const double* w) {
    if (!ctx || !w) return fail(SEM_EINVAL, "sem_set_face_weights: NULL argument");
    try {
        std::memcpy(ctx->face_w_host.data(), w, ctx->face_w_host.size() * sizeof(double));
        DevData& D = ctx->D;
        hipcheck(hipMemcpy(const_cast<double*>(D.d64.face_w), w, ctx->face_w_host.size() * sizeof(double),
                           hipMemcpyHostToDevice), "hipMemcpy");
        if (ctx->have32) {
            std::vector<float> f(ctx->face_w_host.begin(), ctx->face_w_host.end());
            hipcheck(hipMemcpy(const_cast<float*>(D.d32.face_w), f.data(), f.size() * sizeof(float),
                               hipMemcpyHostToDevice), "hipMemcpy");
        }
        if (ctx->have_blocks) {      // the element blocks belong to the previous weights
            ctx->have_blocks = false;
            D.pk = 0;
        }
    } catch (const std::exception& e) {
        return fail(SEM_EHIP, std::string("sem_set_face_weights: ") + e.what());
    }
    return SEM_OK;
}

sem_status sem_set_degrees(sem_ctx* ctx, const int* deg) {
    if (!ctx) return fail(SEM_EINVAL, "sem_set_degrees: NULL context");
    HostSetup& S = ctx->S;
    const int W = S.W;
    std::vector<int> dr((size_t)S.Ereal * 3, W);
    if (deg)
        for (int e = 0; e < S.E; ++e) {
            const int r = S.real_index[e];
            if (r < 0) continue;
            for (int d = 0; d < 3; ++d) {
                const int w = deg[3 * e + d];
                if (w < 1 || w > W)
                    return fail(SEM_EINVAL, "sem_set_degrees: degree " + std::to_string(w) + " of element " +
                                                std::to_string(e) + " outside 1.." + std::to_string(W));
                dr[3 * r + d] = w;
            }
        }
    try {
        DevData& D = ctx->D;
        S.deg = dr;
        separable_bases(S);
        D.pbasis = ctx->upload(S.pbasis);
        D.peig = ctx->upload(S.peig);
        D.pidx = ctx->upload(S.pidx);
        std::vector<int> pe, pd;
        int64_t gdof = S.ncd;
        for (int r = 0; r < S.Ereal; ++r) {
            const int w1 = dr[3 * r], w2 = dr[3 * r + 1], w3 = dr[3 * r + 2];
            gdof += (int64_t)(w1 + 1) * (w2 + 1) * (w3 + 1);
            if (w1 < W || w2 < W || w3 < W) {
                pe.push_back(r);
                pd.push_back(w1 | (w2 << 8) | (w3 << 16));
            }
        }
        ctx->graded_ndof = gdof;
        ctx->proj_elem_host = pe;
        ctx->proj_deg_host = pd;
        if (!pe.empty()) {
            std::vector<double> tab;
            for (int w = 0; w <= W; ++w) {
                const std::vector<double> Q = degree_projector(S, std::max(w, 1));
                tab.insert(tab.end(), Q.begin(), Q.end());
            }
            D.projtab = ctx->upload(tab);
            D.proj_elem = ctx->upload(pe);
            D.proj_deg = ctx->upload(pd);
        }
        D.nproj = (int)pe.size();
        // the element blocks belong to the previous space
        if (ctx->have_blocks) {
            ctx->have_blocks = false;
            D.pk = 0;
        }
    } catch (const std::exception& e) {
        return fail(SEM_EHIP, std::string("sem_set_degrees: ") + e.what());
    }
    return SEM_OK;
}

int64_t sem_graded_ndof(const sem_ctx* ctx) { return ctx ? ctx->graded_ndof : -1; }

sem_status sem_project(sem_ctx* ctx, double* u, void* stream) {
    if (!ctx || !u) return fail(SEM_EINVAL, "sem_project: NULL argument");
    try {
        ctx->ops.project((hipStream_t)stream, ctx->D, u);
        hipcheck(hipGetLastError(), "sem_project");
    } catch (const std::exception& e) {
        return fail(SEM_EHIP, e.what());
    }
    return SEM_OK;
}

sem_status sem_conforming_correction(sem_ctx* ctx, const double* u, double* uc, void* stream) {
    if (!ctx || !u || !uc) return fail(SEM_EINVAL, "sem_conforming_correction: NULL argument");
    if (u == uc) return fail(SEM_EINVAL, "sem_conforming_correction: u and uc alias");
    hipStream_t st = (hipStream_t)stream;
    HostSetup& S = ctx->S;
    try {
        if (!ctx->d_conf_tab) {
            const int n3 = S.n * S.n * S.n;
            std::vector<int> tab((size_t)S.Ereal * 30, -1);
            for (int e = 0; e < S.E; ++e) {
                const int r = S.real_index[e];
                if (r < 0) continue;
                for (int f = 0; f < 6; ++f) {
                    int* t = &tab[(size_t)r * 30 + 5 * f];
                    if (S.bc[6 * e + f] != BC_INTERIOR) continue;   // boundary faces are not corrected
                    const int e2 = S.nbr[6 * e + f];
                    t[0] = S.kind[e2] == REAL ? 0 : (S.kind[e2] == CORNER_CONST ? 1 : 2);
                    t[1] = S.kind[e2] == REAL ? S.real_index[e2] * n3 : S.cdof[e2];
                    t[2] = S.nbr_face[6 * e + f];
                    t[3] = S.orient[6 * e + f];
                    t[4] = S.cdir[e2];
                }
            }
            ctx->d_conf_tab = ctx->upload(tab);
            ctx->d_xn = ctx->upload(S.xn);
        }
        ctx->ops.conform(st, ctx->D, u, uc, ctx->d_conf_tab, ctx->d_xn);
        if (S.ncd > 0)
            hipcheck(hipMemcpyAsync(uc + S.nreal_dof, u + S.nreal_dof, (size_t)S.ncd * sizeof(double),
                                    hipMemcpyDeviceToDevice, st), "copy corner unknowns");
        hipcheck(hipGetLastError(), "sem_conforming_correction launch");
    } catch (const std::exception& e) {
        return fail(SEM_EHIP, e.what());
    }
    return SEM_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Scratch of the allocation-free entry point: the per-element partial sums of
// the H^1 error and their two totals.  One copy per device (each device that
// runs it holds it until the process ends); every call on a device reuses it,
// so calls that overlap on one device race.
constexpr size_t NOALLOC_SCRATCH_DOUBLES = (size_t)1 << 19;   // 4 MiB
static __device__ __align__(256) double scratch[NOALLOC_SCRATCH_DOUBLES];

namespace {
constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mutex;
double* g_scratch[MAX_DEVICES] = {};

// device address of this device's copy of `scratch` (looked up once per
// device, with that device current; the array's name itself is only a host
// stand-in)
double* scratch_of_current_device() {
    int dev = -1;
    hipcheck(hipGetDevice(&dev), "hipGetDevice");
    if (dev < 0 || dev >= MAX_DEVICES) throw std::invalid_argument("device index out of range");
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    if (!g_scratch[dev]) {
        void* ptr = nullptr;
        hipcheck(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)), "hipGetSymbolAddress(scratch)");
        g_scratch[dev] = static_cast<double*>(ptr);
    }
    return g_scratch[dev];
}
}  // namespace

extern "C" {

sem_status sem_error_noalloc(sem_ctx* ctx, const double* u, const double* uex, const double* gex, double* rel_h1,
                             void* stream) {
    if (!ctx || !u || !uex || !gex || !rel_h1) return fail(SEM_EINVAL, "sem_error_noalloc: NULL argument");
    const HostSetup& S = ctx->S;
    const size_t need = 2 * (size_t)S.Ereal + 2;
    if (need > NOALLOC_SCRATCH_DOUBLES)
        return fail(SEM_EINVAL, "sem_error_noalloc: " + std::to_string(S.Ereal) + " real elements exceed the " +
                                    std::to_string((NOALLOC_SCRATCH_DOUBLES - 2) / 2) + " its scratch holds");
    hipStream_t st = (hipStream_t)stream;
    try {
        int dev = -1;
        hipcheck(hipGetDevice(&dev), "hipGetDevice");
        if (dev != ctx->device) return fail(SEM_EINVAL, "sem_error_noalloc: the context's device is not current");
        double* part = scratch_of_current_device();
        // every element writes its two partials, then one kernel sums them in
        // element order into the two totals behind them: nothing to clear
        ctx->ops.error(st, ctx->D, u, S.nq, ctx->d_Lg, ctx->d_Lg1, ctx->d_eji, ctx->d_ew, uex, gex, part);
        launch_sum_rows(st, part, S.Ereal, 2, part + 2 * (size_t)S.Ereal);
        hipcheck(hipGetLastError(), "sem_error_noalloc launch");
        double tot[2] = {0.0, 0.0};
        hipcheck(hipMemcpyAsync(tot, part + 2 * (size_t)S.Ereal, sizeof(tot), hipMemcpyDeviceToHost, st), "copy");
        hipcheck(hipStreamSynchronize(st), "sync");
        *rel_h1 = tot[1] > 0 ? std::sqrt(tot[0] / tot[1]) : 0.0;
    } catch (const std::invalid_argument& e) {
        return fail(SEM_EINVAL, std::string("sem_error_noalloc: ") + e.what());
    } catch (const std::exception& e) {
        return fail(SEM_EHIP, e.what());
    }
    return SEM_OK;
}

sem_status sem_autotune(sem_ctx* ctx, int precision, int reps, int* tile_out, double* ms_out, void* stream) {
    if (!ctx || reps <= 0) return fail(SEM_EINVAL, "sem_autotune: bad argument");
    if (precision != SEM_FP64 && precision != SEM_MIXED_FP32) return fail(SEM_EINVAL, "sem_autotune: bad precision");
    hipStream_t st = (hipStream_t)stream;
    try {
        if (precision == SEM_MIXED_FP32) ctx->ensure_fp32();
        Ops& ops = (precision == SEM_MIXED_FP32) ? ctx->ops32 : ctx->ops;
        hipEvent_t e0, e1;
        hipcheck(hipEventCreate(&e0), "event");
        hipcheck(hipEventCreate(&e1), "event");
        double best = 1e300;
        int bi = 0;
        for (int t = 0; t < 3; ++t) {
            double ms = -1.0;
            if (t == 0 || ops.volume_tile[t] != ops.volume_tile[t - 1]) {
                ops.volume_tile[t](st, ctx->D, ctx->d_p, ctx->d_q, 0, nullptr, nullptr, nullptr);   // warm-up
                hipcheck(hipEventRecord(e0, st), "event");
                for (int k = 0; k < reps; ++k)
                    ops.volume_tile[t](st, ctx->D, ctx->d_p, ctx->d_q, 0, nullptr, nullptr, nullptr);
                hipcheck(hipEventRecord(e1, st), "event");
                hipcheck(hipEventSynchronize(e1), "sync");
                float f = 0;
                hipcheck(hipEventElapsedTime(&f, e0, e1), "elapsed");
                ms = f / reps;
                if (ms < best) { best = ms; bi = t; }
            }
            if (ms_out) ms_out[t] = ms;
        }
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        hipcheck(hipGetLastError(), "autotune launch");
        ops.tile = bi;
        ops.volume = ops.volume_tile[bi];
        if (tile_out) {
            tile_out[0] = bi;
            for (int t = 0; t < 3; ++t) tile_out[1 + t] = ops.tile_slab[t];
        }
    } catch (const std::exception& e) {
        return fail(SEM_EHIP, e.what());
    }
    return SEM_OK;
}

sem_status sem_set_tile(sem_ctx* ctx, int precision, int tile) {
    if (!ctx || tile < 0 || tile > 2) return fail(SEM_EINVAL, "sem_set_tile: bad argument");
    if (precision != SEM_FP64 && precision != SEM_MIXED_FP32) return fail(SEM_EINVAL, "sem_set_tile: bad precision");
    try {
        if (precision == SEM_MIXED_FP32) ctx->ensure_fp32();
    } catch (const std::exception& e) {
        return fail(SEM_EHIP, e.what());
    }
    Ops& ops = (precision == SEM_MIXED_FP32) ? ctx->ops32 : ctx->ops;
    ops.tile = tile;
    ops.volume = ops.volume_tile[tile];
    return SEM_OK;
}

sem_status sem_work_counts(const sem_ctx* ctx, int64_t* c) {
    if (!ctx || !c) return fail(SEM_EINVAL, "sem_work_counts: NULL argument");
    const HostSetup& S = ctx->S;
    int64_t fields = 0, general = 0, slots = 0, pco = 0;
    for (unsigned mk : S.fmask) {
        fields += __builtin_popcount(mk);
        general += (mk & 0x1F8u) ? 1 : 0;
    }
    for (unsigned char a : S.slot_active) slots += a;
    for (const FaceHost& F : S.faces) pco += (int64_t)F.PA.size() + (int64_t)F.PB.size();
    c[0] = S.Ereal; c[1] = S.E; c[2] = fields; c[3] = general;
    c[4] = slots; c[5] = (int64_t)S.faces.size(); c[6] = pco; c[7] = S.ndof;
    // bytes of element-block data one preconditioner apply reads (0: separable)
    c[8] = c[9] = 0;
    if (ctx->have_blocks && ctx->D.pk != 0) {
        const int64_t n3 = (int64_t)S.n * S.n * S.n;
        const int64_t U = ctx->n_stored_blocks;
        // stored inverses read once: n3 x n3 entries per distinct block (FP64 /
        // float); the float triangular-factor fallback sweeps G twice
        c[8] = U * n3 * n3 * 8;
        c[9] = (ctx->mixed_pk == 3) ? U * n3 * n3 * 4 : U * n3 * (n3 + 1) / 2 * 4 * 2;
    }
    return SEM_OK;
}

sem_status sem_kernel_times(sem_ctx* ctx, const double* u, int reps, int precision, double* ms, void* stream) {
    if (!ctx || !u || !ms || reps <= 0) return fail(SEM_EINVAL, "sem_kernel_times: bad argument");
    if (precision != SEM_FP64 && precision != SEM_MIXED_FP32) return fail(SEM_EINVAL, "sem_kernel_times: bad precision");
    hipStream_t st = (hipStream_t)stream;
    const DevData& D = ctx->D;
    try {
        if (precision == SEM_MIXED_FP32) ctx->ensure_fp32();
        const Ops& ops = (precision == SEM_MIXED_FP32) ? ctx->ops32 : ctx->ops;
        DevData Du = D;                 // the update kernel as the solver of that precision runs it
        if (precision == SEM_MIXED_FP32 && Du.pk == 1) Du.pk = ctx->mixed_pk;
        clear_done(ctx, st);
        // the four kernels of one operator apply and preconditioner solve, in
        // iteration order, reps times; events between them, so that each
        // launch sees the caches as an iteration leaves them
        std::vector<hipEvent_t> ev((size_t)5 * reps);
        for (auto& e : ev) hipcheck(hipEventCreate(&e), "hipEventCreate");
        hipcheck(hipMemcpyAsync(ctx->d_p, u, D.ndof * sizeof(double), hipMemcpyDeviceToDevice, st), "copy");
        // one untimed pass so that every buffer holds valid data
        apply_X_with(ops, ctx, st, ctx->d_p, ctx->d_q);
        ctx->ops.update(st, Du, 2, nullptr, ctx->d_q, ctx->d_z, nullptr, nullptr, nullptr, ctx->sc);
        for (int i = 0; i < reps; ++i) {
            hipEvent_t* e = &ev[(size_t)5 * i];
            hipcheck(hipEventRecord(e[0], st), "event");
            ops.volume(st, D, ctx->d_p, ctx->d_q, 0, nullptr, nullptr, nullptr);
            hipcheck(hipEventRecord(e[1], st), "event");
            ops.face(st, D, 0, nullptr);
            hipcheck(hipEventRecord(e[2], st), "event");
            ops.gather(st, D, ctx->d_q, nullptr, ctx->sc, 0, 0);
            hipcheck(hipEventRecord(e[3], st), "event");
            ctx->ops.update(st, Du, 2, nullptr, ctx->d_q, ctx->d_z, nullptr, nullptr, nullptr, ctx->sc);
            hipcheck(hipEventRecord(e[4], st), "event");
        }
        hipcheck(hipGetLastError(), "launch");
        hipcheck(hipEventSynchronize(ev.back()), "sync");
        for (int k = 0; k < 4; ++k) ms[k] = 0.0;
        for (int i = 0; i < reps; ++i)
            for (int k = 0; k < 4; ++k) {
                float t = 0;
                hipcheck(hipEventElapsedTime(&t, ev[(size_t)5 * i + k], ev[(size_t)5 * i + k + 1]), "elapsed");
                ms[k] += t / reps;
            }
        for (auto& e : ev) (void)hipEventDestroy(e);
    } catch (const std::exception& e) {
        return fail(SEM_EHIP, e.what());
    }
    return SEM_OK;
}

}  // extern "C"
