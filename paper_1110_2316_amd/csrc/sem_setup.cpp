// Host-side setup of the least-squares h-p spectral element operator.
//
// Builds, from a mesh description, everything the GPU kernels need:
//  * 1D GLL data on the W+1 solution nodes and the 2W+1 quadrature nodes
//    (thesis Sec. 5.3, eq 5.47), the discrete H^{1/2} double-sum matrix K;
//  * per real element the coefficient fields of the weighted operator
//    omega(x) sqrt(w |J|) L u at the (2W+1)^3 GLL points (transformed operators
//    eq 2.22, 2.28, 2.35, data transforms of eq 4.2-4.7; L = -Laplace);
//  * per face term the jump/boundary quantities and their fractional-norm
//    weights (eq 2.16-2.18, 2.25, 2.27, 2.29, 2.34, 2.38, 4.2-4.7);
//  * the separable preconditioner eigenbases (eq 5.15-5.20, 5.37-5.42) and
//    the corner blocks (U-form corner terms, eq 2.26, 2.32, 2.40);
//  * the Gauss rule for the relative H^1 error.
// Derivatives of the element maps come from second-order forward-mode dual
// numbers.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <exception>
#include <mutex>
#include <stdexcept>
#include <string>
#include <thread>
#include <vector>

#include "sem_internal.h"

namespace sem {
namespace {

// f(i) for i in [0, n) on up to 16 host threads (SEM_HOST_THREADS in the
// environment sets another limit; items handed out one at a time, so the
// results do not depend on the thread count); the first exception thrown by
// an item is rethrown here
template <class F>
void parallel_for(int n, F f) {
    unsigned cap = 16;
    if (const char* ev = std::getenv("SEM_HOST_THREADS")) {
        const long v = std::atol(ev);
        if (v > 0) cap = (unsigned)std::min(v, 256L);
    }
    const unsigned hw = std::max(1u, std::thread::hardware_concurrency());
    const unsigned nt = std::min({hw, cap, (unsigned)std::max(n, 1)});
    if (nt <= 1) {
        for (int i = 0; i < n; ++i) f(i);
        return;
    }
    std::atomic<int> next{0};
    std::exception_ptr err;
    std::mutex mu;
    auto work = [&]() {
        try {
            for (int i; (i = next.fetch_add(1)) < n;) f(i);
        } catch (...) {
            std::lock_guard<std::mutex> g(mu);
            if (!err) err = std::current_exception();
            next = n;
        }
    };
    std::vector<std::thread> pool;
    for (unsigned t = 1; t < nt; ++t) pool.emplace_back(work);
    work();
    for (auto& t : pool) t.join();
    if (err) std::rethrow_exception(err);
}

// ------------------------------------------------------------ dual numbers
// value, gradient and (symmetric) Hessian in three variables
struct J2 {
    double v = 0, g[3] = {0, 0, 0}, h[6] = {0, 0, 0, 0, 0, 0};
    J2() = default;
    J2(double c) : v(c) {}
};
inline int hidx(int c, int d) {
    if (c == d) return c;
    if (c > d) std::swap(c, d);
    return c == 0 ? (d == 1 ? 3 : 4) : 5;
}
inline J2 operator+(const J2& a, const J2& b) {
    J2 r; r.v = a.v + b.v;
    for (int i = 0; i < 3; ++i) r.g[i] = a.g[i] + b.g[i];
    for (int i = 0; i < 6; ++i) r.h[i] = a.h[i] + b.h[i];
    return r;
}
inline J2 operator-(const J2& a, const J2& b) {
    J2 r; r.v = a.v - b.v;
    for (int i = 0; i < 3; ++i) r.g[i] = a.g[i] - b.g[i];
    for (int i = 0; i < 6; ++i) r.h[i] = a.h[i] - b.h[i];
    return r;
}
inline J2 operator*(const J2& a, const J2& b) {
    J2 r; r.v = a.v * b.v;
    for (int i = 0; i < 3; ++i) r.g[i] = a.v * b.g[i] + b.v * a.g[i];
    for (int c = 0; c < 3; ++c)
        for (int d = c; d < 3; ++d) {
            int k = hidx(c, d);
            r.h[k] = a.v * b.h[k] + b.v * a.h[k] + a.g[c] * b.g[d] + a.g[d] * b.g[c];
        }
    return r;
}
inline J2 chain(const J2& a, double f, double f1, double f2) {
    J2 r; r.v = f;
    for (int i = 0; i < 3; ++i) r.g[i] = f1 * a.g[i];
    for (int c = 0; c < 3; ++c)
        for (int d = c; d < 3; ++d) {
            int k = hidx(c, d);
            r.h[k] = f1 * a.h[k] + f2 * a.g[c] * a.g[d];
        }
    return r;
}
inline J2 recip(const J2& a) { double x = a.v; return chain(a, 1 / x, -1 / (x * x), 2 / (x * x * x)); }
inline J2 operator/(const J2& a, const J2& b) { return a * recip(b); }
inline J2 jexp(const J2& a) { double e = std::exp(a.v); return chain(a, e, e, e); }
inline J2 jsin(const J2& a) { return chain(a, std::sin(a.v), std::cos(a.v), -std::sin(a.v)); }
inline J2 jcos(const J2& a) { return chain(a, std::cos(a.v), -std::sin(a.v), -std::cos(a.v)); }
inline J2 jsqrt(const J2& a) {
    double s = std::sqrt(a.v);
    return chain(a, s, 0.5 / s, -0.25 / (s * a.v));
}

// ------------------------------------------------------------ 1D rules
// Legendre P_N and P_N' at x by the three-term recurrence.
void legendre(int N, double x, double& p, double& dp) {
    double p0 = 1, p1 = x;
    if (N == 0) { p = 1; dp = 0; return; }
    for (int k = 2; k <= N; ++k) {
        double p2 = ((2 * k - 1) * x * p1 - (k - 1) * p0) / k;
        p0 = p1; p1 = p2;
    }
    p = p1;
    dp = (std::fabs(x) == 1.0) ? 0.5 * N * (N + 1) * std::pow(x, N + 1)
                               : N * (x * p1 - p0) / (x * x - 1);
}

// n-point GLL: endpoints and the roots of P'_{n-1} (Newton from
// Chebyshev-Gauss-Lobatto guesses); weights 2/(N(N+1) P_N^2).
void gll_rule(int n, std::vector<double>& x, std::vector<double>& w) {
    int N = n - 1;
    x.assign(n, 0); w.assign(n, 0);
    for (int i = 0; i < n; ++i) {
        double xi = -std::cos(M_PI * i / N);
        if (i > 0 && i < N) {
            for (int it = 0; it < 100; ++it) {
                double p, dp;
                legendre(N, xi, p, dp);
                double d2p = (2 * xi * dp - N * (N + 1) * p) / (1 - xi * xi);
                double dx = dp / d2p;
                xi -= dx;
                if (std::fabs(dx) < 1e-16) break;
            }
        }
        x[i] = xi;
        double p, dp;
        legendre(N, xi, p, dp);
        w[i] = 2.0 / (N * (N + 1) * p * p);
    }
    x[0] = -1; x[N] = 1;
}

void gauss_rule(int n, std::vector<double>& x, std::vector<double>& w) {
    x.assign(n, 0); w.assign(n, 0);
    for (int i = 0; i < n; ++i) {
        double xi = -std::cos(M_PI * (i + 0.75) / (n + 0.5));
        for (int it = 0; it < 100; ++it) {
            double p, dp;
            legendre(n, xi, p, dp);
            double dx = p / dp;
            xi -= dx;
            if (std::fabs(dx) < 1e-16) break;
        }
        double p, dp;
        legendre(n, xi, p, dp);
        x[i] = xi;
        w[i] = 2.0 / ((1 - xi * xi) * dp * dp);
    }
}

// Lagrange basis l_j on `nodes` and its first two derivatives at t, as
// products of linear factors carried in (value, d/dt, d2/dt2).
void lagrange_at(const std::vector<double>& nodes, double t, std::vector<double>& l0,
                 std::vector<double>& l1, std::vector<double>& l2) {
    int n = (int)nodes.size();
    l0.assign(n, 0); l1.assign(n, 0); l2.assign(n, 0);
    for (int j = 0; j < n; ++j) {
        double v = 1, d1 = 0, d2 = 0;
        for (int k = 0; k < n; ++k) {
            if (k == j) continue;
            double a = (t - nodes[k]) / (nodes[j] - nodes[k]);
            double b = 1.0 / (nodes[j] - nodes[k]);
            // (v, d1, d2) * (a, b, 0)
            double nv = v * a, nd1 = d1 * a + v * b, nd2 = d2 * a + 2 * d1 * b;
            v = nv; d1 = nd1; d2 = nd2;
        }
        l0[j] = v; l1[j] = d1; l2[j] = d2;
    }
}

// ------------------------------------------------------------ element maps
template <class T>
void planar(const double* p, const T& a, const T& s, bool inner_s, T& px, T& py) {
    T u = (a + T(1.0)) * T(0.5), v = (s + T(1.0)) * T(0.5);
    if ((int)p[0] == 0) {
        T th = T(p[1]) + u * T(p[2] - p[1]);
        double rin = inner_s ? p[3] : p[4];
        T ax = T(rin) * jcos(th), ay = T(rin) * jsin(th);
        T ox = T(p[5]) + u * T(p[7] - p[5]);
        T oy = T(p[6]) + u * T(p[8] - p[6]);
        px = (T(1.0) - v) * ax + v * ox;
        py = (T(1.0) - v) * ay + v * oy;
    } else {
        const double* c = p + 1;
        T w00 = (T(1.0) - u) * (T(1.0) - v), w10 = u * (T(1.0) - v), w01 = (T(1.0) - u) * v, w11 = u * v;
        px = w00 * T(c[0]) + w10 * T(c[2]) + w01 * T(c[4]) + w11 * T(c[6]);
        py = w00 * T(c[1]) + w10 * T(c[3]) + w01 * T(c[5]) + w11 * T(c[7]);
    }
}

template <class T>
void chart_local(int chart, const double* b, const double* p, const T l[3], T xl[3]) {
    T y[3];
    for (int i = 0; i < 3; ++i) y[i] = T(b[2 * i]) + (l[i] + T(1.0)) * T(0.5 * (b[2 * i + 1] - b[2 * i]));
    switch (chart) {
    case AFFINE:
        for (int i = 0; i < 3; ++i) xl[i] = y[i];
        break;
    case VTX_BOX: {
        T rho = jexp(y[2]);
        xl[0] = rho * jsin(y[0]) * jcos(y[1]);
        xl[1] = rho * jsin(y[0]) * jsin(y[1]);
        xl[2] = rho * jcos(y[0]);
    } break;
    case VE_BOX: {
        T r = jexp(y[0] + y[2]);
        xl[0] = r * jcos(y[1]); xl[1] = r * jsin(y[1]); xl[2] = jexp(y[2]);
    } break;
    case EDGE_BOX: {
        T r = jexp(y[0]);
        xl[0] = r * jcos(y[1]); xl[1] = r * jsin(y[1]); xl[2] = y[2];
    } break;
    case VTX_PATCH: {
        T px, py;
        planar(p, l[0], l[1], true, px, py);
        T nrm = jsqrt(px * px + py * py + T(1.0));
        T rho = jexp(y[2]);
        xl[0] = rho * px / nrm; xl[1] = rho * py / nrm; xl[2] = rho / nrm;
    } break;
    case COLUMN: {
        T sx, sy, tx, ty;
        planar(p, l[0], l[1], true, sx, sy);
        planar(p, l[0], l[1], false, tx, ty);
        T nrm = jsqrt(sx * sx + sy * sy + T(1.0));
        T t = y[2];
        T rs = T(p[9]);
        xl[0] = (T(1.0) - t) * rs * sx / nrm + t * tx;
        xl[1] = (T(1.0) - t) * rs * sy / nrm + t * ty;
        xl[2] = (T(1.0) - t) * rs / nrm + t;
    } break;
    default:
        throw std::runtime_error("unknown chart type");
    }
}

struct Geo {
    double x[3], J[3][3], H[3][3][3];
};

Geo element_geo(const HostSetup& S, int e, const double lam[3], bool second = true) {
    J2 l[3];
    for (int c = 0; c < 3; ++c) { l[c].v = lam[c]; l[c].g[c] = 1.0; }
    J2 xl[3];
    chart_local(S.chart[e], &S.box[6 * e], &S.patch[12 * e], l, xl);
    const double* R = &S.frame[9 * e];
    const double* o = &S.origin[3 * e];
    Geo G;
    for (int a = 0; a < 3; ++a) {
        G.x[a] = o[a];
        for (int c = 0; c < 3; ++c) { G.J[a][c] = 0; for (int d = 0; d < 3; ++d) G.H[a][c][d] = 0; }
        for (int b = 0; b < 3; ++b) {
            G.x[a] += R[3 * a + b] * xl[b].v;
            for (int c = 0; c < 3; ++c) {
                G.J[a][c] += R[3 * a + b] * xl[b].g[c];
                if (second)
                    for (int d = 0; d < 3; ++d) G.H[a][c][d] += R[3 * a + b] * xl[b].h[hidx(c, d)];
            }
        }
    }
    return G;
}

double inv3(const double A[3][3], double B[3][3]) {
    double det = A[0][0] * (A[1][1] * A[2][2] - A[1][2] * A[2][1]) -
                 A[0][1] * (A[1][0] * A[2][2] - A[1][2] * A[2][0]) +
                 A[0][2] * (A[1][0] * A[2][1] - A[1][1] * A[2][0]);
    double id = 1.0 / det;
    B[0][0] = (A[1][1] * A[2][2] - A[1][2] * A[2][1]) * id;
    B[0][1] = (A[0][2] * A[2][1] - A[0][1] * A[2][2]) * id;
    B[0][2] = (A[0][1] * A[1][2] - A[0][2] * A[1][1]) * id;
    B[1][0] = (A[1][2] * A[2][0] - A[1][0] * A[2][2]) * id;
    B[1][1] = (A[0][0] * A[2][2] - A[0][2] * A[2][0]) * id;
    B[1][2] = (A[0][2] * A[1][0] - A[0][0] * A[1][2]) * id;
    B[2][0] = (A[1][0] * A[2][1] - A[1][1] * A[2][0]) * id;
    B[2][1] = (A[0][1] * A[2][0] - A[0][0] * A[2][1]) * id;
    B[2][2] = (A[0][0] * A[1][1] - A[0][1] * A[1][0]) * id;
    return det;
}

// d x_global / d y for the modified coordinates y of a neighbourhood frame
// (eq 2.3 vertex, eq 2.8 vertex-edge, eq 2.5 edge), at global point x.
void modified_jac(int region, const double* R, const double* o, const double x[3], double Jy[3][3]) {
    double xl[3];
    for (int b = 0; b < 3; ++b) {
        xl[b] = 0;
        for (int a = 0; a < 3; ++a) xl[b] += R[3 * a + b] * (x[a] - o[a]);
    }
    double r = std::hypot(xl[0], xl[1]);
    double th = std::atan2(xl[1], xl[0]);
    J2 y[3];
    J2 f[3];
    if (region == VTX) {
        double rho = std::sqrt(r * r + xl[2] * xl[2]);
        y[0].v = std::atan2(r, xl[2]); y[1].v = th; y[2].v = std::log(rho);
        for (int c = 0; c < 3; ++c) y[c].g[c] = 1;
        J2 e = jexp(y[2]);
        f[0] = e * jsin(y[0]) * jcos(y[1]); f[1] = e * jsin(y[0]) * jsin(y[1]); f[2] = e * jcos(y[0]);
    } else if (region == VE) {
        y[0].v = std::log(r / xl[2]); y[1].v = th; y[2].v = std::log(xl[2]);
        for (int c = 0; c < 3; ++c) y[c].g[c] = 1;
        J2 rr = jexp(y[0] + y[2]);
        f[0] = rr * jcos(y[1]); f[1] = rr * jsin(y[1]); f[2] = jexp(y[2]);
    } else if (region == EDGE) {
        y[0].v = std::log(r); y[1].v = th; y[2].v = xl[2];
        for (int c = 0; c < 3; ++c) y[c].g[c] = 1;
        J2 rr = jexp(y[0]);
        f[0] = rr * jcos(y[1]); f[1] = rr * jsin(y[1]); f[2] = y[2];
    } else {
        throw std::runtime_error("modified_jac: bad region");
    }
    for (int a = 0; a < 3; ++a)
        for (int k = 0; k < 3; ++k) {
            Jy[a][k] = 0;
            for (int b = 0; b < 3; ++b) Jy[a][k] += R[3 * a + b] * f[b].g[k];
        }
}

void orient_map(int o, double a, double b, double& ra, double& rb) {
    if (o & 1) std::swap(a, b);
    if (o & 2) a = -a;
    if (o & 4) b = -b;
    ra = a; rb = b;
}

const int TANG[3][2] = {{1, 2}, {0, 2}, {0, 1}};

void face_lam(int f, double a, double b, double lam[3]) {
    int d = f / 2;
    lam[d] = (f & 1) ? 1.0 : -1.0;
    lam[TANG[d][0]] = a;
    lam[TANG[d][1]] = b;
}

// Singularity order of the regions: a face between two regions is counted
// once, in the modified coordinates of its more singular side.
int singularity(int region) {
    static const int order[4] = {/*REG*/ 0, /*VTX*/ 1, /*VE*/ 3, /*EDGE*/ 2};
    return order[region];
}

// Rank of one side of a face: an element that carries its own unknowns
// comes before a corner element, then the more singular region, then the
// lower element index.  The side of higher rank is side A.
long long side_rank(const HostSetup& S, int e) {
    return (long long)(S.kind[e] == REAL) * 4 * (1LL << 32) + (long long)singularity(S.region[e]) * (1LL << 32) +
           (long long)((1LL << 31) - 1 - e);
}

// Orientation code mapping the neighbour's face coordinates back to ours.
// Without the swap bit each negation undoes itself; with it, a negation of
// the first coordinate after the swap acts on the second before it.
int orient_inverse(int o) {
    if (!(o & 1)) return o;
    return 1 | ((o & 2) << 1) | ((o & 4) >> 1);
}

// The face norms of the functional, for one face, in the coordinates they
// are written in.  Every quantity w of a face term enters as
//   a int int w^2 + b int dq_1 (int int quotient along q_0) + c int dq_0 (...along q_1)
// over the face grid of side A, whose coordinates (q_0, q_1) are the
// tangential lambdas of side A: the master square itself for regular and
// vertex faces (eq 2.17b, 2.18, 2.25), or the rectangle of the two
// tangential modified coordinates for vertex-edge and edge faces
// (eq 2.27a-c, 2.34a-c), dy = (h / 2) dlambda, under which the quotient
// of a double integral keeps its value and only the outer integral scales.
struct NormSpec {
    double outer = 1;          // factor of |||.||| as a whole (E F, F, G or 1; R; 1)
    double quot[3] = {1, 1, 1};   // extra factor of the quotient along modified direction c
    double dscale[3] = {1, 1, 1}; // weight of the derivative jump along direction c inside |||.|||
    double l2 = 1;             // weight of ||[u]||_0^2 (and of the data term u - g)
    double half[3] = {1, 1, 1};   // h_c / 2: length element of the face coordinates
};

// Weights (alpha, beta, gamma) of one quantity: the derivative along
// direction k (k < 0: the value itself) of the face with normal direction d.
void norm_weights(const NormSpec& N, int d, int k, double w[3]) {
    const int q0 = TANG[d][0], q1 = TANG[d][1];
    if (k < 0) {
        w[0] = N.l2 * N.half[q0] * N.half[q1];
        w[1] = w[2] = 0.0;
        return;
    }
    const double s2 = N.dscale[k] * N.dscale[k];
    w[0] = s2 * N.outer * N.half[q0] * N.half[q1];
    w[1] = s2 * N.outer * N.quot[q0] * N.half[q1];
    w[2] = s2 * N.outer * N.quot[q1] * N.half[q0];
}

// The sups of the neighbourhood weights over a face (or an element), taken
// over its points: every weight is monotone along the modified
// coordinates, so its sup over a box sits at a corner, and the GLL grids
// contain the corners.  Points in the frame (R, o) of the neighbourhood.
struct Sups {
    double rho = 0;      // vertex: R = sup e^chi = sup rho
    double sinphi = 0;   // vertex-edge: E = sup sin phi
    double x3 = 0;       // vertex-edge: F = sup e^zeta = sup x3
    double r = 0;        // edge: G = sup e^tau = sup r
};
void sup_accumulate(Sups& s, const double* R, const double* o, const double x[3]) {
    double xl[3];
    for (int b = 0; b < 3; ++b) {
        xl[b] = 0;
        for (int a = 0; a < 3; ++a) xl[b] += R[3 * a + b] * (x[a] - o[a]);
    }
    const double r = std::hypot(xl[0], xl[1]);
    const double rho = std::sqrt(r * r + xl[2] * xl[2]);
    s.rho = std::max(s.rho, rho);
    s.sinphi = std::max(s.sinphi, r / rho);
    s.x3 = std::max(s.x3, xl[2]);
    s.r = std::max(s.r, r);
}

// eq 2.16-2.18 (regular), 2.25 (vertex: R), 2.27 / 2.29 (vertex-edge: E, F,
// G = E on zeta-faces), 2.34 / 2.38 (edge: G, H = G on x3-faces), for a face
// with normal direction d whose side A has modified extents h.
NormSpec norm_spec(int region, int d, const Sups& sp, const double h[3]) {
    NormSpec N;
    if (region == REG) return N;
    if (region == VTX) {
        N.outer = N.l2 = sp.rho;
        return N;
    }
    for (int c = 0; c < 3; ++c) N.half[c] = 0.5 * h[c];
    // the weight that eq 2.27 / 2.34 attach to the third modified direction
    // (zeta or x3): it multiplies its quotient, its derivative jump, and on
    // faces normal to it the whole norm and the L2 weight of [u]
    const double w3 = (region == VE) ? sp.sinphi : sp.r;
    const double base = (region == VE) ? sp.x3 : 1.0;
    N.outer = base * (d == 2 ? w3 : 1.0);
    N.l2 = N.outer;
    N.quot[2] = w3;
    N.dscale[2] = w3;
    return N;
}

// symmetric Jacobi eigensolver for a small dense matrix (row-major n x n)
void jacobi_eig(int n, std::vector<double> A, std::vector<double>& V, std::vector<double>& lam) {
    V.assign(n * n, 0);
    for (int i = 0; i < n; ++i) V[i * n + i] = 1;
    for (int sweep = 0; sweep < 100; ++sweep) {
        double off = 0, tot = 0;
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j) {
                tot += A[i * n + j] * A[i * n + j];
                if (i != j) off += A[i * n + j] * A[i * n + j];
            }
        if (off <= 1e-32 * tot) break;
        for (int p = 0; p < n; ++p)
            for (int q = p + 1; q < n; ++q) {
                double apq = A[p * n + q];
                if (std::fabs(apq) < 1e-300) continue;
                double app = A[p * n + p], aqq = A[q * n + q];
                double theta = (aqq - app) / (2 * apq);
                double t = (theta >= 0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1));
                double c = 1 / std::sqrt(t * t + 1), s = t * c;
                for (int k = 0; k < n; ++k) {
                    double akp = A[k * n + p], akq = A[k * n + q];
                    A[k * n + p] = c * akp - s * akq;
                    A[k * n + q] = s * akp + c * akq;
                }
                for (int k = 0; k < n; ++k) {
                    double apk = A[p * n + k], aqk = A[q * n + k];
                    A[p * n + k] = c * apk - s * aqk;
                    A[q * n + k] = s * apk + c * aqk;
                }
                for (int k = 0; k < n; ++k) {
                    double vkp = V[k * n + p], vkq = V[k * n + q];
                    V[k * n + p] = c * vkp - s * vkq;
                    V[k * n + q] = s * vkp + c * vkq;
                }
            }
    }
    lam.resize(n);
    for (int i = 0; i < n; ++i) lam[i] = A[i * n + i];
}

}  // namespace

// ===========================================================================
// Graded degrees (Sec. 2.3): the polynomials of degree <= w < W in one
// direction, as values at the n = W+1 GLL nodes, are spanned by the columns
// of Lv[i][c] = P_c(x_i), c = 0..w (Legendre).
namespace {
std::vector<double> legendre_columns(const HostSetup& S, int w) {
    const int n = S.n, k = w + 1;
    std::vector<double> Lv((size_t)n * k);
    for (int i = 0; i < n; ++i)
        for (int c = 0; c < k; ++c) {
            double p, dp;
            legendre(c, S.xn[i], p, dp);
            Lv[(size_t)i * k + c] = p;
        }
    return Lv;
}

// in-place Cholesky G = L L^T of a small SPD matrix (row-major; lower part)
void cholesky(int k, std::vector<double>& G) {
    for (int j = 0; j < k; ++j) {
        double d = G[j * k + j];
        for (int l = 0; l < j; ++l) d -= G[j * k + l] * G[j * k + l];
        if (!(d > 0)) throw std::runtime_error("degree basis: Gram matrix not positive definite");
        G[j * k + j] = std::sqrt(d);
        for (int i = j + 1; i < k; ++i) {
            double v = G[i * k + j];
            for (int l = 0; l < j; ++l) v -= G[i * k + l] * G[j * k + l];
            G[i * k + j] = v / G[j * k + j];
        }
    }
}

// X <- L^-1 X (X: k x c row-major) for the lower factor L in G
void lower_solve(int k, const std::vector<double>& L, std::vector<double>& X, int c) {
    for (int i = 0; i < k; ++i)
        for (int col = 0; col < c; ++col) {
            double v = X[(size_t)i * c + col];
            for (int l = 0; l < i; ++l) v -= L[i * k + l] * X[(size_t)l * c + col];
            X[(size_t)i * c + col] = v / L[i * k + i];
        }
}
}  // namespace

std::vector<double> degree_projector(const HostSetup& S, int w) {
    const int n = S.n;
    std::vector<double> Q((size_t)n * n, 0.0);
    if (w >= S.W) {
        for (int i = 0; i < n; ++i) Q[(size_t)i * n + i] = 1.0;
        return Q;
    }
    const int k = w + 1;
    const std::vector<double> Lv = legendre_columns(S, w);
    // Q = Lv (Lv^T Lv)^-1 Lv^T = Y^T Y with Y = L^-1 Lv^T, L L^T = Lv^T Lv
    std::vector<double> G((size_t)k * k, 0.0), Y((size_t)k * n);
    for (int a = 0; a < k; ++a)
        for (int b = 0; b < k; ++b)
            for (int i = 0; i < n; ++i) G[a * k + b] += Lv[(size_t)i * k + a] * Lv[(size_t)i * k + b];
    cholesky(k, G);
    for (int a = 0; a < k; ++a)
        for (int i = 0; i < n; ++i) Y[(size_t)a * n + i] = Lv[(size_t)i * k + a];
    lower_solve(k, G, Y, n);
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) {
            double v = 0;
            for (int a = 0; a < k; ++a) v += Y[(size_t)a * n + i] * Y[(size_t)a * n + j];
            Q[(size_t)i * n + j] = v;
        }
    return Q;
}

// Separable forms of Sec. 5.2 per element direction: the pencil
// (a S2 + b S1, F) with F = diag(w), S1 = D^T F D, S2 = (DD)^T F (DD) on the
// (W+1)-point GLL rule, a = g^4, b = g^2.  On the degree-w polynomials
// (Lv) the pencil is (Lv^T A Lv, Lv^T F Lv); with its Cholesky factor L and
// the eigenpairs (Y, lam) of L^-1 Lv^T A Lv L^-T the basis is
// Phi = Lv L^-T Y (Phi^T F Phi = I on the graded space), padded with zero
// columns (eigenvalue 0: those modes carry nothing).  For w = W the basis is
// F^-1/2 times the eigenvectors of F^-1/2 A F^-1/2.
void separable_bases(HostSetup& S) {
    const int n = S.n, W = S.W, Er = S.Ereal;
    std::vector<double> S1(n * n, 0), S2(n * n, 0), DD(n * n, 0);
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j)
            for (int k = 0; k < n; ++k) DD[i * n + j] += S.Dn[i * n + k] * S.Dn[k * n + j];
    for (int a = 0; a < n; ++a)
        for (int b = 0; b < n; ++b)
            for (int i = 0; i < n; ++i) {
                S1[a * n + b] += S.wn[i] * S.Dn[i * n + a] * S.Dn[i * n + b];
                S2[a * n + b] += S.wn[i] * DD[i * n + a] * DD[i * n + b];
            }
    S.pbasis.clear();
    S.peig.clear();
    S.pidx.assign((size_t)Er * 3, 0);
    struct Key { double a, b; int w; };
    std::vector<Key> keys;
    auto basis_of = [&](double a, double b, int w) -> int {
        for (size_t i = 0; i < keys.size(); ++i)
            if (keys[i].a == a && keys[i].b == b && keys[i].w == w) return (int)i;
        keys.push_back({a, b, w});
        std::vector<double> V, lam;
        if (w >= W) {
            std::vector<double> A(n * n);
            for (int i = 0; i < n; ++i)
                for (int j = 0; j < n; ++j)
                    A[i * n + j] = (a * S2[i * n + j] + b * S1[i * n + j]) / std::sqrt(S.wn[i] * S.wn[j]);
            jacobi_eig(n, A, V, lam);
            for (int i = 0; i < n; ++i)
                for (int j = 0; j < n; ++j) S.pbasis.push_back(V[i * n + j] / std::sqrt(S.wn[i]));
            for (int j = 0; j < n; ++j) S.peig.push_back(lam[j]);
            return (int)keys.size() - 1;
        }
        const int k = w + 1;
        const std::vector<double> Lv = legendre_columns(S, w);
        std::vector<double> Ar((size_t)k * k, 0.0), Fr((size_t)k * k, 0.0), ALv((size_t)n * k, 0.0);
        for (int i = 0; i < n; ++i)
            for (int c = 0; c < k; ++c)
                for (int j = 0; j < n; ++j) ALv[(size_t)i * k + c] += (a * S2[i * n + j] + b * S1[i * n + j]) * Lv[(size_t)j * k + c];
        for (int c = 0; c < k; ++c)
            for (int d = 0; d < k; ++d)
                for (int i = 0; i < n; ++i) {
                    Ar[c * k + d] += Lv[(size_t)i * k + c] * ALv[(size_t)i * k + d];
                    Fr[c * k + d] += Lv[(size_t)i * k + c] * S.wn[i] * Lv[(size_t)i * k + d];
                }
        cholesky(k, Fr);
        // B = L^-1 Ar L^-T: solve on the columns, transpose, solve again
        lower_solve(k, Fr, Ar, k);
        std::vector<double> At((size_t)k * k);
        for (int c = 0; c < k; ++c)
            for (int d = 0; d < k; ++d) At[c * k + d] = Ar[d * k + c];
        lower_solve(k, Fr, At, k);
        for (int c = 0; c < k; ++c)
            for (int d = c + 1; d < k; ++d) At[c * k + d] = At[d * k + c] = 0.5 * (At[c * k + d] + At[d * k + c]);
        jacobi_eig(k, At, V, lam);
        // Psi = L^-T Y: back substitution with L^T
        std::vector<double> Psi = V;
        for (int i = k - 1; i >= 0; --i)
            for (int col = 0; col < k; ++col) {
                double v = Psi[(size_t)i * k + col];
                for (int l = i + 1; l < k; ++l) v -= Fr[l * k + i] * Psi[(size_t)l * k + col];
                Psi[(size_t)i * k + col] = v / Fr[i * k + i];
            }
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j) {
                double v = 0;
                if (j < k)
                    for (int c = 0; c < k; ++c) v += Lv[(size_t)i * k + c] * Psi[(size_t)c * k + j];
                S.pbasis.push_back(v);
            }
        for (int j = 0; j < n; ++j) S.peig.push_back(j < k ? lam[j] : 0.0);
        return (int)keys.size() - 1;
    };
    for (int r = 0; r < Er; ++r)
        for (int d = 0; d < 3; ++d) {
            const double g = S.pg[3 * r + d];
            S.pidx[3 * r + d] = basis_of(g * g * g * g, g * g, S.deg[3 * r + d]);
        }
}

// ===========================================================================
// Coefficient fields of the weighted operator at the (2W+1)^3 GLL points of
// every real element, for L u = -sum_ij a_ij u_{x_i x_j} + sum_j beta_j u_{x_j}
// + c u (eq 2.2 with beta_j = b_j - sum_i d a_ij / d x_i; a, beta, c host
// arrays over the volume points, NULL: a = I, beta = 0, c = 0).  With
// Ji = J^-1 and the map's second derivatives H^b (x_b's Hessian in lambda),
//   -tr(a Hess_x u) = -sum_cd (Ji a Ji^T)_cd u_cd + sum_b (grad_x u)_b tr(Ji a Ji^T H^b),
// (grad_x u)_b = sum_c Ji_cb u_c, so the lambda-fields carry the coefficients
// -(Ji a Ji^T)_cd (x2 off the diagonal), sum_b Ji_cb (tr(Ji a Ji^T H^b) +
// beta_b) and c, each times s = sqrt(w |J|) omega (eq 2.22, 2.28, 2.35).
void volume_fields(HostSetup& S, const double* acoef, const double* beta, const double* ccoef) {
    const int m = S.m, m3 = m * m * m, Er = S.Ereal;
    S.coef.assign((size_t)Er * NFIELD * m3, 0.0);
    S.fmask.assign(Er, 0);
    S.svol.assign((size_t)Er * m3, 0.0);
    S.xvol.assign((size_t)Er * m3 * 3, 0.0);
    static const int SYM[6][2] = {{0, 0}, {1, 1}, {2, 2}, {0, 1}, {0, 2}, {1, 2}};
    // elements in parallel: each writes its own slices of coef, svol, xvol, fmask
    parallel_for(S.E, [&](int e) {
        const int r = S.real_index[e];
        if (r < 0) return;
        const double* R = &S.frame[9 * e];
        const double* o = &S.origin[3 * e];
        double* C = &S.coef[(size_t)r * NFIELD * m3];
        double maxc = 0;
        for (int c3 = 0; c3 < m; ++c3)
            for (int b = 0; b < m; ++b)
                for (int a = 0; a < m; ++a) {
                    const int q = a + m * (b + m * c3);
                    const size_t pt = (size_t)r * m3 + q;
                    double lam[3] = {S.xm[a], S.xm[b], S.xm[c3]};
                    Geo g = element_geo(S, e, lam, true);
                    double Ji[3][3];
                    const double det = std::fabs(inv3(g.J, Ji));
                    double A[3][3] = {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}};
                    if (acoef)
                        for (int k = 0; k < 6; ++k) A[SYM[k][0]][SYM[k][1]] = A[SYM[k][1]][SYM[k][0]] = acoef[pt * 6 + k];
                    double JA[3][3], G[3][3];
                    for (int c = 0; c < 3; ++c)
                        for (int j = 0; j < 3; ++j) {
                            JA[c][j] = 0;
                            for (int i = 0; i < 3; ++i) JA[c][j] += Ji[c][i] * A[i][j];
                        }
                    for (int c = 0; c < 3; ++c)
                        for (int d = 0; d < 3; ++d) {
                            G[c][d] = 0;
                            for (int j = 0; j < 3; ++j) G[c][d] += JA[c][j] * Ji[d][j];
                        }
                    double tb[3];
                    for (int bb = 0; bb < 3; ++bb) {
                        tb[bb] = beta ? beta[pt * 3 + bb] : 0.0;
                        for (int c = 0; c < 3; ++c)
                            for (int d = 0; d < 3; ++d) tb[bb] += g.H[bb][c][d] * G[c][d];
                    }
                    double a1[3];
                    for (int aa = 0; aa < 3; ++aa) {
                        a1[aa] = 0;
                        for (int bb = 0; bb < 3; ++bb) a1[aa] += Ji[aa][bb] * tb[bb];
                    }
                    double xl[3];
                    for (int bb = 0; bb < 3; ++bb) {
                        xl[bb] = 0;
                        for (int aa = 0; aa < 3; ++aa) xl[bb] += R[3 * aa + bb] * (g.x[aa] - o[aa]);
                    }
                    double om = 1.0;
                    if (S.region[e] == VTX) om = std::sqrt(xl[0] * xl[0] + xl[1] * xl[1] + xl[2] * xl[2]);
                    else if (S.region[e] == VE || S.region[e] == EDGE) om = std::hypot(xl[0], xl[1]);
                    const double s = std::sqrt(S.wm[a] * S.wm[b] * S.wm[c3] * det) * om;
                    const double vals[NFIELD] = {-G[0][0], -G[1][1], -G[2][2], -2 * G[0][1], -2 * G[0][2],
                                                 -2 * G[1][2], a1[0], a1[1], a1[2], ccoef ? ccoef[pt] : 0.0};
                    for (int k = 0; k < NFIELD; ++k) {
                        C[(size_t)k * m3 + q] = s * vals[k];
                        maxc = std::max(maxc, std::fabs(s * vals[k]));
                    }
                    S.svol[pt] = s;
                    for (int aa = 0; aa < 3; ++aa) S.xvol[pt * 3 + aa] = g.x[aa];
                }
        // fields that vanish on the element are skipped by the kernels
        uint32_t mask = 0;
        for (int k = 0; k < NFIELD; ++k) {
            double mk = 0;
            for (int q = 0; q < m3; ++q) mk = std::max(mk, std::fabs(C[(size_t)k * m3 + q]));
            if (mk > 1e-15 * maxc) mask |= 1u << k;
            else for (int q = 0; q < m3; ++q) C[(size_t)k * m3 + q] = 0.0;
        }
        S.fmask[r] = mask;
    });
}

void build_host_setup(const sem_mesh* mesh, HostSetup& S) {
    if (!mesh) throw std::runtime_error("null mesh");
    const int W = mesh->W;
    if (W < 1 || W > 12) throw std::runtime_error("W must be in 1..12");
    const int E = mesh->nelem;
    if (E <= 0) throw std::runtime_error("empty mesh");
    S.W = W; S.n = W + 1; S.m = 2 * W + 1; S.E = E; S.ncd = mesh->n_corner_dof;
    const int n = S.n, m = S.m;
    auto cp_i = [&](const int32_t* p, int cnt) { return std::vector<int>(p, p + cnt); };
    auto cp_d = [&](const double* p, int cnt) { return std::vector<double>(p, p + cnt); };
    S.region = cp_i(mesh->region, E); S.kind = cp_i(mesh->kind, E); S.chart = cp_i(mesh->chart, E);
    S.cdof = cp_i(mesh->cdof, E); S.cdir = cp_i(mesh->cdir, E);
    S.box = cp_d(mesh->box, 6 * E); S.frame = cp_d(mesh->frame, 9 * E);
    S.mframe = cp_d(mesh->mframe, 9 * E);
    S.origin = cp_d(mesh->origin, 3 * E); S.patch = cp_d(mesh->patch, 12 * E);
    S.nbr = cp_i(mesh->nbr, 6 * E); S.nbr_face = cp_i(mesh->nbr_face, 6 * E);
    S.orient = cp_i(mesh->orient, 6 * E); S.bc = cp_i(mesh->bc, 6 * E);

    // real elements and validation
    S.real_index.assign(E, -1);
    int Er = 0;
    for (int e = 0; e < E; ++e) {
        if (S.kind[e] == REAL) S.real_index[e] = Er++;
        else {
            if (S.kind[e] != CORNER_CONST && S.kind[e] != CORNER_POLY) throw std::runtime_error("bad element kind");
            int width = S.kind[e] == CORNER_CONST ? 1 : n;
            if (S.cdof[e] < 0 || S.cdof[e] + width > S.ncd) throw std::runtime_error("corner offset out of range");
            if (S.kind[e] == CORNER_POLY && (S.cdir[e] < 0 || S.cdir[e] > 2)) throw std::runtime_error("bad cdir");
        }
        if (S.region[e] < 0 || S.region[e] > 3) throw std::runtime_error("bad region");
        for (int f = 0; f < 6; ++f) {
            int bc = S.bc[6 * e + f];
            if (bc == BC_INTERIOR) {
                int e2 = S.nbr[6 * e + f], f2 = S.nbr_face[6 * e + f];
                if (e2 < 0 || e2 >= E || f2 < 0 || f2 > 5) throw std::runtime_error("bad neighbour");
                if (S.nbr[6 * e2 + f2] != e || S.nbr_face[6 * e2 + f2] != f)
                    throw std::runtime_error("neighbour table not symmetric");
                if (S.orient[6 * e + f] < 0 || S.orient[6 * e + f] > 7) throw std::runtime_error("bad orientation");
            } else if (bc != BC_DIRICHLET && bc != BC_SKIP && bc != BC_NEUMANN) {
                throw std::runtime_error("bad boundary code");
            } else if ((bc == BC_DIRICHLET || bc == BC_NEUMANN) && S.kind[e] != REAL) {
                throw std::runtime_error("boundary data face on a corner element");
            }
        }
    }
    S.Ereal = Er;
    S.nreal_dof = (int64_t)Er * n * n * n;
    S.ndof = S.nreal_dof + S.ncd;

    // 1D data
    gll_rule(n, S.xn, S.wn);
    gll_rule(m, S.xm, S.wm);
    S.Im.assign(m * n, 0); S.D1m.assign(m * n, 0); S.D2m.assign(m * n, 0);
    std::vector<double> l0, l1, l2;
    for (int a = 0; a < m; ++a) {
        lagrange_at(S.xn, S.xm[a], l0, l1, l2);
        for (int j = 0; j < n; ++j) { S.Im[a * n + j] = l0[j]; S.D1m[a * n + j] = l1[j]; S.D2m[a * n + j] = l2[j]; }
    }
    S.Dn.assign(n * n, 0);
    for (int i = 0; i < n; ++i) {
        lagrange_at(S.xn, S.xn[i], l0, l1, l2);
        for (int j = 0; j < n; ++j) S.Dn[i * n + j] = l1[j];
    }
    {
        // K: sum_{i != i'} w_i w_i' ((l_i - l_i')/(x_i - x_i'))^2 + sum_i w_i^2 (D l)_i^2
        std::vector<double> Dm(m * m);
        for (int i = 0; i < m; ++i) {
            lagrange_at(S.xm, S.xm[i], l0, l1, l2);
            for (int j = 0; j < m; ++j) Dm[i * m + j] = l1[j];
        }
        S.K.assign(m * m, 0);
        for (int i = 0; i < m; ++i)
            for (int ip = 0; ip < m; ++ip) {
                if (i == ip) continue;
                double c = S.wm[i] * S.wm[ip] / ((S.xm[i] - S.xm[ip]) * (S.xm[i] - S.xm[ip]));
                S.K[i * m + i] += c; S.K[ip * m + ip] += c;
                S.K[i * m + ip] -= c; S.K[ip * m + i] -= c;
            }
        for (int a = 0; a < m; ++a)
            for (int b = 0; b < m; ++b) {
                double s = 0;
                for (int i = 0; i < m; ++i) s += S.wm[i] * S.wm[i] * Dm[i * m + a] * Dm[i * m + b];
                S.K[a * m + b] += s;
            }
    }

    // ---------------------------------------------------------------- volume
    volume_fields(S, nullptr, nullptr, nullptr);

    // ---------------------------------------------------------------- faces
    S.slot_active.assign(6 * E, 0);
    const int P = m * m;
    // one face term (no side effects on S: the terms are computed in
    // parallel and recorded in order below); wfo: the Neumann datum factors
    auto make_face = [&](int e, int f, int e2, int f2, int o, bool neumann, FaceHost& F, std::vector<double>& wfo) {
        if (e2 >= 0 && side_rank(S, e2) > side_rank(S, e)) {
            std::swap(e, e2);
            std::swap(f, f2);
            o = orient_inverse(o);
        }
        F.eA = e; F.fA = f; F.eB = e2; F.fB = f2; F.orient = (e2 >= 0) ? o : 0;
        const int reg = S.region[e];
        F.region = reg;
        const bool dir = e2 < 0;
        const int d = f / 2, t0 = TANG[d][0], t1 = TANG[d][1];
        const double* bx = &S.box[6 * e];
        double h[3] = {bx[1] - bx[0], bx[3] - bx[2], bx[5] - bx[4]};
        // per-point geometry
        std::vector<double> JiA(P * 9), JiB(P * 9), JA(P * 9), Jyv(P * 9);
        F.xA.assign(P * 3, 0);
        for (int j = 0; j < m; ++j)
            for (int i = 0; i < m; ++i) {
                int p = i + m * j;
                double lam[3];
                face_lam(f, S.xm[i], S.xm[j], lam);
                Geo gA = element_geo(S, e, lam, false);
                double Ji[3][3];
                inv3(gA.J, Ji);
                for (int a = 0; a < 3; ++a) {
                    F.xA[3 * p + a] = gA.x[a];
                    for (int c = 0; c < 3; ++c) { JiA[9 * p + 3 * a + c] = Ji[a][c]; JA[9 * p + 3 * a + c] = gA.J[a][c]; }
                }
                if (!dir) {
                    double ba, bb, lamB[3];
                    orient_map(o, S.xm[i], S.xm[j], ba, bb);
                    face_lam(f2, ba, bb, lamB);
                    Geo gB = element_geo(S, e2, lamB, false);
                    double err = 0, sc = 1;
                    for (int a = 0; a < 3; ++a) { err = std::max(err, std::fabs(gB.x[a] - gA.x[a])); sc = std::max(sc, std::fabs(gA.x[a])); }
                    if (err > 1e-9 * sc)
                        throw std::runtime_error("non-conforming face between elements " + std::to_string(e) +
                                                 " and " + std::to_string(e2));
                    double JiBl[3][3];
                    inv3(gB.J, JiBl);
                    for (int a = 0; a < 3; ++a)
                        for (int c = 0; c < 3; ++c) JiB[9 * p + 3 * a + c] = JiBl[a][c];
                }
                double Jy[3][3];
                if (reg == REG) {
                    for (int a = 0; a < 3; ++a) for (int c = 0; c < 3; ++c) Jy[a][c] = (a == c);
                } else {
                    modified_jac(reg, &S.mframe[9 * e], &S.origin[3 * e], gA.x, Jy);
                }
                for (int a = 0; a < 3; ++a) for (int c = 0; c < 3; ++c) Jyv[9 * p + 3 * a + c] = Jy[a][c];
            }
        // quantities: coefficients over (value, d/dlam1, d/dlam2, d/dlam3)
        std::vector<double> PA, PB;
        int nq = 0;
        auto addq = [&](int kind, int idx, const double w[3], bool interior, int dkind) {
            // kind 0: value; 1: d/dy_idx (y = x for REG); 2: d/dlam_idx
            PA.resize((nq + 1) * 4 * P, 0.0);
            PB.resize((nq + 1) * 4 * P, 0.0);
            for (int p = 0; p < P; ++p) {
                for (int c = 0; c < 4; ++c) {
                    double va = 0, vb = 0;
                    if (kind == 0) { va = vb = (c == 0); }
                    else if (kind == 2) { va = (c == idx + 1); }
                    else if (c > 0) {
                        for (int l = 0; l < 3; ++l) {
                            va += JiA[9 * p + 3 * (c - 1) + l] * Jyv[9 * p + 3 * l + idx];
                            if (interior) vb += JiB[9 * p + 3 * (c - 1) + l] * Jyv[9 * p + 3 * l + idx];
                        }
                    }
                    PA[(nq * 4 + c) * P + p] = va;
                    PB[(nq * 4 + c) * P + p] = interior ? vb : 0.0;
                }
            }
            for (int k = 0; k < 3; ++k) F.wts[nq][k] = w[k];
            F.dkind[nq] = dkind;
            if (!interior) {
                F.ddir.resize((nq + 1) * P * 3, 0.0);
                for (int p = 0; p < P; ++p)
                    for (int a = 0; a < 3; ++a) {
                        double v = 0;
                        if (kind == 2) v = JA[9 * p + 3 * a + idx];
                        else if (kind == 1) v = Jyv[9 * p + 3 * a + idx];
                        F.ddir[(nq * P + p) * 3 + a] = v;
                    }
            }
            ++nq;
        };
        // the norms of this face (sups over side A's face points; the extents
        // of a box chart are its box, dy = (h / 2) dlambda)
        Sups sp;
        {
            const double* Rn = &S.mframe[9 * e];
            for (int p = 0; p < P; ++p) sup_accumulate(sp, Rn, &S.origin[3 * e], &F.xA[3 * p]);
        }
        const NormSpec NS = norm_spec(reg, d, sp, h);
        double wv[3];
        if (neumann) {
            // Neumann face (eq 2.16 / 4.2; 4.3, 4.5, 4.7): one quantity, the
            // normal derivative du/dnu = nu . grad_x u (the Laplacian's conormal)
            // times the factor the thesis applies to the datum in the
            // neighbourhoods (e^chi / sin phi = rho^2 / r; e^zeta e^psi = r;
            // e^tau = r), normed like the face's derivative jumps
            std::vector<double> wf(P, 1.0);
            PA.assign(4 * P, 0.0);
            for (int p = 0; p < P; ++p) {
                // outward unit normal: the gradient of lambda_d, row d of J^-1
                double nu[3], nn = 0;
                for (int a = 0; a < 3; ++a) { nu[a] = ((f & 1) ? 1.0 : -1.0) * JiA[9 * p + 3 * d + a]; nn += nu[a] * nu[a]; }
                nn = std::sqrt(nn);
                if (reg != REG) {
                    const double* Rn = &S.mframe[9 * e];
                    double xl[3];
                    for (int b = 0; b < 3; ++b) {
                        xl[b] = 0;
                        for (int a = 0; a < 3; ++a) xl[b] += Rn[3 * a + b] * (F.xA[3 * p + a] - S.origin[3 * e + a]);
                    }
                    const double r = std::hypot(xl[0], xl[1]);
                    const double rho2 = r * r + xl[2] * xl[2];
                    wf[p] = (reg == VTX) ? rho2 / r : r;
                }
                for (int c = 0; c < 3; ++c) {
                    double v = 0;
                    for (int a = 0; a < 3; ++a) v += JiA[9 * p + 3 * c + a] * nu[a] / nn;
                    PA[(1 + c) * P + p] = wf[p] * v;
                }
                for (int a = 0; a < 3; ++a) F.nuv.push_back(nu[a] / nn);
            }
            wfo = wf;
            norm_weights(NS, d, t0, wv);
            for (int k = 0; k < 3; ++k) F.wts[0][k] = wv[k];
            F.dkind[0] = 2;
            F.ddir.assign(P * 3, 0.0);
            nq = 1;
        } else {
            norm_weights(NS, d, -1, wv);
            addq(0, 0, wv, !dir, 0);
            if (!dir) {
                // the jumps of the three derivatives in the region's coordinates
                for (int k = 0; k < 3; ++k) {
                    double wk[3];
                    norm_weights(NS, d, k, wk);
                    addq(1, k, wk, true, 1);
                }
            } else {
                // data faces: the two tangential derivatives, along the master
                // square's lambdas for regular and vertex faces (eq 2.18), along
                // the modified coordinates for vertex-edge and edge faces (eq 4.5, 4.7)
                const int kind = (reg == REG || reg == VTX) ? 2 : 1;
                for (int k : {t0, t1}) {
                    double wk[3];
                    norm_weights(NS, d, k, wk);
                    addq(kind, k, wk, false, 1);
                }
            }
        }
        F.nq = nq;
        // compress constant coefficient blocks
        auto compress = [&](std::vector<double>& Pv, int& mode) {
            bool cst = true;
            for (int k = 0; k < nq * 4 && cst; ++k) {
                double v0 = Pv[k * P], sc = std::fabs(v0);
                for (int p = 1; p < P; ++p) sc = std::max(sc, std::fabs(Pv[k * P + p]));
                for (int p = 1; p < P; ++p)
                    if (std::fabs(Pv[k * P + p] - v0) > 1e-14 * std::max(sc, 1e-300)) { cst = false; break; }
            }
            if (cst) {
                std::vector<double> c(nq * 4);
                for (int k = 0; k < nq * 4; ++k) c[k] = Pv[k * P];
                Pv = c;
                mode = 0;
            } else mode = 1;
        };
        compress(PA, F.pmodeA);
        if (!dir) compress(PB, F.pmodeB);
        else { PB.clear(); F.pmodeB = 0; }
        F.PA = PA; F.PB = PB;
    };
    struct FaceJob { int e, f, e2, f2, o, bc; };
    std::vector<FaceJob> jobs;
    for (int e = 0; e < E; ++e)
        for (int f = 0; f < 6; ++f) {
            int bc = S.bc[6 * e + f];
            if (bc == BC_INTERIOR) {
                int e2 = S.nbr[6 * e + f], f2 = S.nbr_face[6 * e + f];
                if (e2 < e || (e2 == e && f2 < f)) continue;
                jobs.push_back({e, f, e2, f2, S.orient[6 * e + f], bc});
            } else if (bc == BC_DIRICHLET || bc == BC_NEUMANN) {
                jobs.push_back({e, f, -1, -1, 0, bc});
            }
        }
    std::vector<FaceHost> fterms(jobs.size());
    std::vector<std::vector<double>> fwf(jobs.size());
    parallel_for((int)jobs.size(), [&](int j) {
        const FaceJob& J = jobs[j];
        make_face(J.e, J.f, J.e2, J.f2, J.o, J.bc == BC_NEUMANN, fterms[j], fwf[j]);
    });
    for (size_t j = 0; j < jobs.size(); ++j) {
        FaceHost& F = fterms[j];
        if (jobs[j].bc == BC_DIRICHLET) S.dir_faces.push_back((int)S.faces.size());
        if (jobs[j].bc == BC_NEUMANN) {
            S.neu_faces.push_back((int)S.faces.size());
            S.neu_wfac.insert(S.neu_wfac.end(), fwf[j].begin(), fwf[j].end());
        }
        S.slot_active[6 * F.eA + F.fA] = 1;
        if (F.eB >= 0) S.slot_active[6 * F.eB + F.fB] = 1;
        S.faces.push_back(std::move(F));
    }

    // ---------------------------------------------------------------- preconditioner
    {
        S.pg.assign(Er * 3, 1.0);
        S.deg.assign(Er * 3, W);
        S.pscale.assign(Er, 1.0);
        // d y / d lambda (y: modified coordinates of the element's region)
        // at lambda, from the element map and the neighbourhood chart
        auto dy_dlam = [&](int e, const double lam[3], double out[3][3]) {
            Geo g = element_geo(S, e, lam, false);
            double Jy[3][3], Jyi[3][3];
            modified_jac(S.region[e], &S.mframe[9 * e], &S.origin[3 * e], g.x, Jy);
            inv3(Jy, Jyi);
            for (int a = 0; a < 3; ++a)
                for (int c = 0; c < 3; ++c) {
                    out[a][c] = 0;
                    for (int l = 0; l < 3; ++l) out[a][c] += Jyi[a][l] * g.J[l][c];
                }
        };
        // sups of the region weights over an element, on its solution grid
        // (which holds the corners, where the monotone weights peak)
        auto element_sups = [&](int e) {
            Sups sp;
            for (int k = 0; k < n; ++k)
                for (int j = 0; j < n; ++j)
                    for (int i = 0; i < n; ++i) {
                        double lam[3] = {S.xn[i], S.xn[j], S.xn[k]};
                        Geo g = element_geo(S, e, lam, false);
                        sup_accumulate(sp, &S.mframe[9 * e], &S.origin[3 * e], g.x);
                    }
            return sp;
        };
        // elements in parallel: each writes its own pg and pscale entries
        parallel_for(E, [&](int e) {
            const int r = S.real_index[e];
            if (r < 0) return;
            const int reg = S.region[e];
            // The U-forms (eq 2.19 on the master cube; eq 2.26, 2.32, 2.40 in
            // the modified coordinates, with their weights): per direction the
            // 1D pair (int v''^2 + v'^2, int v^2) scaled to the extent h_d of
            // the element along that coordinate, h_d = 2 |d y / d lambda_d| at
            // the centre (the box for box charts); the weight e^chi / e^zeta
            // as its sup s, the factor of the third direction's second
            // derivative (sin phi / e^tau) as its sup eta.
            double h[3] = {2.0, 2.0, 2.0}, s = 1.0, eta = 1.0;
            if (reg != REG) {
                const double centre[3] = {0.0, 0.0, 0.0};
                double dy[3][3];
                dy_dlam(e, centre, dy);
                for (int c = 0; c < 3; ++c) h[c] = 2.0 * std::sqrt(dy[0][c] * dy[0][c] + dy[1][c] * dy[1][c] + dy[2][c] * dy[2][c]);
                const Sups sp = element_sups(e);
                if (reg == VTX) s = sp.rho;
                if (reg == VE) { s = sp.x3; eta = sp.sinphi; }
                if (reg == EDGE) eta = sp.r;
            }
            for (int d = 0; d < 3; ++d) S.pg[3 * r + d] = (2.0 / h[d]) * (d == 2 ? eta : 1.0);
            S.pscale[r] = s * h[0] * h[1] * h[2] / 8.0;
        });
        separable_bases(S);
        // corner blocks, all diagonal: the U-form corner terms with the
        // (W+1)-point rule.  A constant corner contributes its weight's sup
        // times the area of its finite face (lambda_3 = 1) in modified
        // coordinates (the infinite direction integrates the normalised
        // weight w of eq 2.32 to 1); a corner polynomial along lambda_c
        // contributes at each node the theta-extent times its 1D mass, the
        // vertex-edge one weighted by e^zeta = x3 at the node.
        std::vector<double> cd(S.ncd, 0.0);
        for (int e = 0; e < E; ++e) {
            if (S.kind[e] == REAL) continue;
            const int o = S.cdof[e];
            const int reg = S.region[e];
            if (S.kind[e] == CORNER_CONST) {
                if (reg != VTX && reg != VE) throw std::runtime_error("constant corner outside vertex / vertex-edge region");
                double area = 0;
                for (int j = 0; j < m; ++j)
                    for (int i = 0; i < m; ++i) {
                        const double lam[3] = {S.xm[i], S.xm[j], 1.0};
                        double dy[3][3];
                        dy_dlam(e, lam, dy);
                        area += S.wm[i] * S.wm[j] * std::fabs(dy[0][0] * dy[1][1] - dy[0][1] * dy[1][0]);
                    }
                const Sups sp = element_sups(e);
                cd[o] += (reg == VTX ? sp.rho : sp.x3) * area;
            } else {
                const int dd = S.cdir[e];
                const double* b = &S.box[6 * e];
                const double hth = b[3] - b[2], hp = b[2 * dd + 1] - b[2 * dd];
                for (int i = 0; i < n; ++i) {
                    double v = hth * 0.5 * hp * S.wn[i];
                    if (reg == VE) {
                        double lam[3] = {0.0, 0.0, 0.0};
                        lam[dd] = S.xn[i];
                        const Geo g = element_geo(S, e, lam, false);
                        const double* R = &S.frame[9 * e];
                        double x3 = 0;
                        for (int a = 0; a < 3; ++a) x3 += R[3 * a + 2] * (g.x[a] - S.origin[3 * e + a]);
                        v *= x3;
                    }
                    cd[o + i] += v;
                }
            }
        }
        S.cinv.assign(S.ncd, 0.0);
        for (int i = 0; i < S.ncd; ++i) {
            if (!(cd[i] > 0)) throw std::runtime_error("corner DOF without a preconditioner block");
            S.cinv[i] = 1.0 / cd[i];
        }
    }

    // ---------------------------------------------------------------- corner reduction lists
    {
        std::vector<std::vector<int>> lists(S.ncd);
        for (int e = 0; e < E; ++e) {
            if (S.kind[e] == REAL) continue;
            int v = (int)S.virt_elems.size();
            S.virt_elems.push_back(e);
            if (S.kind[e] == CORNER_CONST) lists[S.cdof[e]].push_back(v * n);
            else for (int k = 0; k < n; ++k) lists[S.cdof[e] + k].push_back(v * n + k);
        }
        S.cptr.assign(S.ncd + 1, 0);
        for (int c = 0; c < S.ncd; ++c) {
            S.cptr[c + 1] = S.cptr[c] + (int)lists[c].size();
            for (int x : lists[c]) S.cidx.push_back(x);
        }
    }

    // ---------------------------------------------------------------- error quadrature
    S.nq = W + 6;
    gauss_rule(S.nq, S.xg, S.wg);
    const int nq = S.nq, nq3 = nq * nq * nq;
    S.Lg.assign(nq * n, 0); S.Lg1.assign(nq * n, 0);
    for (int a = 0; a < nq; ++a) {
        lagrange_at(S.xn, S.xg[a], l0, l1, l2);
        for (int j = 0; j < n; ++j) { S.Lg[a * n + j] = l0[j]; S.Lg1[a * n + j] = l1[j]; }
    }
    S.err_x.assign((size_t)Er * nq3 * 3, 0);
    S.err_ji.assign((size_t)Er * nq3 * 9, 0);
    S.err_w.assign((size_t)Er * nq3, 0);
    // elements in parallel: each writes its own points
    parallel_for(E, [&](int e) {
        int r = S.real_index[e];
        if (r < 0) return;
        for (int c3 = 0; c3 < nq; ++c3)
            for (int b = 0; b < nq; ++b)
                for (int a = 0; a < nq; ++a) {
                    int q = a + nq * (b + nq * c3);
                    double lam[3] = {S.xg[a], S.xg[b], S.xg[c3]};
                    Geo g = element_geo(S, e, lam, false);
                    double Ji[3][3];
                    double det = std::fabs(inv3(g.J, Ji));
                    size_t base = (size_t)r * nq3 + q;
                    for (int aa = 0; aa < 3; ++aa) S.err_x[base * 3 + aa] = g.x[aa];
                    for (int aa = 0; aa < 3; ++aa)
                        for (int cc = 0; cc < 3; ++cc) S.err_ji[base * 9 + 3 * aa + cc] = Ji[aa][cc];
                    S.err_w[base] = S.wg[a] * S.wg[b] * S.wg[c3] * det;
                }
    });
}

}  // namespace sem
