// Host-only driver of the library's setup code (sem_setup.cpp), for the
// sanitizer and thread-count tests: reads a mesh (the sem_mesh arrays,
// little-endian, in the order of the struct) from argv[1], builds the host
// setup and prints a checksum of its arrays, then rebuilds the volume fields
// with general coefficients, the separable bases with mixed degrees and
// every degree projector, and prints a few sizes.  Exit 0 on success, 2 on
// an exception.
#include <cstdio>
#include <cstdlib>
#include <exception>
#include <fstream>
#include <vector>

#include "../paper_1110_2316_amd/csrc/sem_internal.h"

namespace {
// FNV-1a over bytes
unsigned long long fnv(const void* p, size_t n, unsigned long long h = 1469598103934665603ull) {
    const unsigned char* c = static_cast<const unsigned char*>(p);
    for (size_t i = 0; i < n; ++i) { h ^= c[i]; h *= 1099511628211ull; }
    return h;
}
template <class V>
unsigned long long fnv_vec(const V& v, unsigned long long h) { return fnv(v.data(), v.size() * sizeof(v[0]), h); }

template <class T>
std::vector<T> take(std::ifstream& in, size_t n) {
    std::vector<T> v(n);
    in.read(reinterpret_cast<char*>(v.data()), (std::streamsize)(n * sizeof(T)));
    if (!in) throw std::runtime_error("mesh file too short");
    return v;
}
}  // namespace

int main(int argc, char** argv) {
    if (argc < 2) return 1;
    try {
        std::ifstream in(argv[1], std::ios::binary);
        const std::vector<int32_t> head = take<int32_t>(in, 3);
        const size_t E = (size_t)head[1];
        auto region = take<int32_t>(in, E), kind = take<int32_t>(in, E), chart = take<int32_t>(in, E);
        auto frame = take<double>(in, 9 * E), mframe = take<double>(in, 9 * E), origin = take<double>(in, 3 * E);
        auto box = take<double>(in, 6 * E), patch = take<double>(in, 12 * E);
        auto nbr = take<int32_t>(in, 6 * E), nbr_face = take<int32_t>(in, 6 * E);
        auto orient = take<int32_t>(in, 6 * E), bc = take<int32_t>(in, 6 * E);
        auto cdof = take<int32_t>(in, E), cdir = take<int32_t>(in, E);
        sem_mesh m{};
        m.W = head[0];
        m.nelem = head[1];
        m.n_corner_dof = head[2];
        m.region = region.data(); m.kind = kind.data(); m.chart = chart.data();
        m.frame = frame.data(); m.mframe = mframe.data(); m.origin = origin.data();
        m.box = box.data(); m.patch = patch.data();
        m.nbr = nbr.data(); m.nbr_face = nbr_face.data(); m.orient = orient.data(); m.bc = bc.data();
        m.cdof = cdof.data(); m.cdir = cdir.data();
        sem::HostSetup S;
        sem::build_host_setup(&m, S);
        // every array the setup fills (face terms: their used entries)
        unsigned long long h = 1469598103934665603ull;
        for (const auto* v : {&S.coef, &S.svol, &S.xvol, &S.pg, &S.pscale, &S.cinv, &S.err_x, &S.err_ji, &S.err_w,
                              &S.neu_wfac})
            h = fnv_vec(*v, h);
        h = fnv_vec(S.fmask, h);
        h = fnv_vec(S.slot_active, h);
        h = fnv_vec(S.dir_faces, h);
        h = fnv_vec(S.neu_faces, h);
        for (const sem::FaceHost& F : S.faces) {
            const int hdr[9] = {F.eA, F.fA, F.eB, F.fB, F.orient, F.region, F.nq, F.pmodeA, F.pmodeB};
            h = fnv(hdr, sizeof(hdr), h);
            h = fnv(F.wts, sizeof(F.wts[0]) * F.nq, h);
            h = fnv(F.dkind, sizeof(F.dkind[0]) * F.nq, h);
            for (const auto* v : {&F.PA, &F.PB, &F.ddir, &F.xA, &F.nuv}) h = fnv_vec(*v, h);
        }
        std::printf("setup-checksum %016llx\n", h);
        // a general operator: a = diag(1, 2, 3) + 0.1 (offdiagonal), beta, c
        const size_t np = S.svol.size();
        std::vector<double> a(6 * np), beta(3 * np), c(np);
        for (size_t p = 0; p < np; ++p) {
            const double a6[6] = {1.0, 2.0, 3.0, 0.1, 0.1, 0.1};
            for (int k = 0; k < 6; ++k) a[6 * p + k] = a6[k];
            for (int k = 0; k < 3; ++k) beta[3 * p + k] = 0.5 * (k + 1);
            c[p] = 1.5;
        }
        sem::volume_fields(S, a.data(), beta.data(), c.data());
        for (size_t i = 0; i < S.deg.size(); ++i) S.deg[i] = 1 + (int)(i % (size_t)S.W);
        sem::separable_bases(S);
        double tr = 0;
        for (int w = 1; w <= S.W; ++w) {
            const std::vector<double> Q = sem::degree_projector(S, w);
            for (int i = 0; i < S.n; ++i) tr += Q[(size_t)i * S.n + i];
        }
        std::printf("ndof %lld faces %zu bases %zu projector-trace-sum %.6f\n", (long long)S.ndof, S.faces.size(),
                    S.peig.size() / (size_t)S.n, tr);
    } catch (const std::exception& e) {
        std::fprintf(stderr, "setup failed: %s\n", e.what());
        return 2;
    }
    return 0;
}
