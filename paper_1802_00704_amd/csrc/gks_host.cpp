// Host side of libgks: per-mesh setup (geometry, faces, CLS normal
// equations, renumbering, BILU(0)), the GMRES drivers and the C ABI.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <memory>
#include <mutex>
#include <new>
#include <numeric>
#include <string>
#include <type_traits>
#include <vector>

#include "gks_internal.h"

using namespace gks;

// Sweeps of the mixed form's first outer step, adapted after each successful
// step from the Arnoldi steps its solve took (the rule is stated with
// gks_params.adapt_sweeps).  Fewer sweeps cost less per outer step, but a
// first direction too weak to meet the tolerance costs a whole outer step
// more; the count that suffices changes as the flow and the extrapolated
// start change, so the handle probes one sweep lower now and then and backs
// off at once when that costs an outer step.  The hold after a failed trial
// doubles with each failure in a row (64 steps up to 1024), so a handle whose
// count is already the lowest that works probes rarely.
void gks::sweep_rule(SweepAdapt& s, int outer, int top) {
    ++s.step;
    if (s.trial) {
        s.trial = false;
        if (outer > 1) {   // the lower count cost an outer step: back, and hold
            s.q1 = s.prev;
            s.fails = std::min(s.fails + 1, 5);
            s.hold_until = s.step + (64 << (s.fails - 1));
            s.ones = s.hard = 0;
            return;
        }
        s.fails = 0;
    }
    if (outer <= 1) {
        s.hard = 0;
        if (++s.ones >= 8 && s.q1 > 2 && s.step >= s.hold_until) {
            s.prev = s.q1;
            s.q1 -= 1;
            s.trial = true;
            s.ones = 0;
        }
    } else {
        s.ones = 0;
        if (++s.hard >= 4 && s.q1 < top) {
            s.q1 += 1;
            s.hard = 0;
        }
    }
}

// Points of the extrapolated start (gks_params.extrap_points = 0).  Each
// point added cuts the extrapolation error of a smooth flow about ten-fold,
// but the weights grow (their absolute sum is 2^P - 1 at uniform steps), and
// they amplify what the earlier solves left: residuals up to tol each, in
// the directions the solver resolves slowest.  Once the starting residual
// r0 comes within 50 (2^P - 1) tol of that floor, a point fewer may do
// better; while it stays above 1000 (2^P - 1) tol, a point more may (up to
// 6).  Such a step tries it once, after at least 8 steps at the current
// count (2 when r0 is within 5 (2^P - 1) tol), and keeps it if its start is
// below 0.8 times the median of the last four at the current count or its
// solve took fewer Arnoldi steps than their median; else the count goes
// back and no trial follows for 48 steps, doubling with each failure in a
// row up to 384.  Steps whose start took fewer points (a short history) or
// met the tolerance outright leave the rule alone.
void gks::points_rule(PointsAdapt& s, double r0, int used, int outer, double tol) {
    ++s.step;
    if (used != s.P || !(r0 > 0.0)) return;
    if (s.trial) {
        s.trial = false;
        double v[4];
        int o[4];
        std::copy(s.r0, s.r0 + s.nr, v);
        std::copy(s.outer, s.outer + s.nr, o);
        std::sort(v, v + s.nr);
        std::sort(o, o + s.nr);
        const int h = s.nr / 2;
        const double med = s.nr % 2 ? v[h] : 0.5 * (v[h - 1] + v[h]);
        const double omed = s.nr % 2 ? o[h] : 0.5 * (o[h - 1] + o[h]);
        if (r0 < 0.8 * med || outer < omed) {   // the trial count does better: keep it
            s.nr = 0;
            s.since = 0;
            s.fails = 0;
            return;
        }
        s.P = s.prev;
        s.fails = std::min(s.fails + 1, 4);
        s.hold_until = s.step + (24 << s.fails);
        s.since = 0;
        return;
    }
    for (int i = 3; i > 0; --i) {
        s.r0[i] = s.r0[i - 1];
        s.outer[i] = s.outer[i - 1];
    }
    s.r0[0] = r0;
    s.outer[0] = outer;
    s.nr = std::min(s.nr + 1, 4);
    ++s.since;
    const double floor = ((1 << s.P) - 1) * tol;
    const int wait = r0 < 5.0 * floor ? 2 : 8;
    if (s.nr < 2 || s.since < wait || s.step < s.hold_until) return;
    int np = 0;
    if (s.P > 2 && r0 < 50.0 * floor) np = s.P - 1;
    else if (s.P < MAXH + 1 && r0 > 1000.0 * floor) np = s.P + 1;
    if (np) {
        s.prev = s.P;
        s.P = np;
        s.trial = true;
        s.since = 0;
    }
}

void gks::adapt_points(gks_mesh* m, double r0, int used, int outer) {
    if (m->prm.extrap_points == 0) points_rule(m->pts, r0, used, outer, m->prm.tol);
}

static bool adapts(const gks_mesh* m) {
    return m->prm.adapt_sweeps && m->prm.precision == GKS_MIXED && m->prm.inner_solver == GKS_INNER_RICHARDSON;
}

static int top_sweeps(const gks_params& p) { return p.inner_iters_first > 0 ? p.inner_iters_first : p.inner_iters; }

int gks::next_first_sweeps(const gks_mesh* m, int outer) {
    if (!adapts(m)) return m->sw.q1;
    SweepAdapt s = m->sw;
    sweep_rule(s, outer, top_sweeps(m->prm));
    return s.q1;
}

void gks::adapt_first_sweeps(gks_mesh* m, int outer) {
    if (adapts(m)) sweep_rule(m->sw, outer, top_sweeps(m->prm));
}

namespace {

thread_local std::string g_create_err;

// GKS_VERBOSE=1 prints the duration of each setup phase to stderr.
struct PhaseTimer {
    bool on;
    std::chrono::steady_clock::time_point t0;
    PhaseTimer() : on(std::getenv("GKS_VERBOSE") != nullptr), t0(std::chrono::steady_clock::now()) {}
    void mark(const char* what) {
        if (!on) return;
        const auto t1 = std::chrono::steady_clock::now();
        std::fprintf(stderr, "[gks] %-22s %8.1f ms\n", what,
                     std::chrono::duration<double, std::milli>(t1 - t0).count());
        t0 = t1;
    }
};

struct Fail {
    int code;
    std::string msg;
};

#define HIPCHK(expr)                                                                      \
    do {                                                                                  \
        hipError_t e_ = (expr);                                                           \
        if (e_ != hipSuccess)                                                             \
            throw Fail{GKS_EHIP, std::string(#expr) + ": " + hipGetErrorString(e_)};      \
    } while (0)

// ------------------------------------------------------------------ set-up arrays
// The large host arrays of the set-up (matrix, factors and their device
// layouts: several KB per cell) are allocated without initialisation and
// first written by OpenMP loops, so that their page faults spread over the
// threads instead of one serial zero fill each.
template <class T>
struct NoInitAlloc : std::allocator<T> {
    template <class U>
    struct rebind {
        using other = NoInitAlloc<U>;
    };
    NoInitAlloc() = default;
    template <class U>
    NoInitAlloc(const NoInitAlloc<U>&) noexcept {}
    template <class U>
    void construct(U* p) noexcept {
        ::new ((void*)p) U;
    }
    template <class U, class... A>
    void construct(U* p, A&&... a) {
        ::new ((void*)p) U(std::forward<A>(a)...);
    }
};
template <class T>
using hvec = std::vector<T, NoInitAlloc<T>>;

// v = n copies of x, written in parallel
template <class T>
void par_fill(hvec<T>& v, size_t n, const T& x) {
    v.clear();
    v.resize(n);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < (int64_t)n; ++i) v[i] = x;
}

// ------------------------------------------------------------------ 5x5 blocks
using Blk = std::array<double, 25>;

Blk bzero() {
    Blk b;
    b.fill(0.0);
    return b;
}

Blk bmul(const Blk& a, const Blk& b) {
    Blk c = bzero();
    for (int i = 0; i < 5; ++i)
        for (int k = 0; k < 5; ++k) {
            const double aik = a[i * 5 + k];
            for (int j = 0; j < 5; ++j) c[i * 5 + j] += aik * b[k * 5 + j];
        }
    return c;
}

// Gauss-Jordan inverse with partial pivoting; throws on a singular block
Blk binv(const Blk& a) {
    double m[5][10];
    for (int i = 0; i < 5; ++i)
        for (int j = 0; j < 10; ++j) m[i][j] = j < 5 ? a[i * 5 + j] : (j - 5 == i ? 1.0 : 0.0);
    for (int c = 0; c < 5; ++c) {
        int p = c;
        for (int r = c + 1; r < 5; ++r)
            if (std::fabs(m[r][c]) > std::fabs(m[p][c])) p = r;
        if (!(std::fabs(m[p][c]) > 0.0)) throw Fail{GKS_EINVAL, "singular pivot block in the CLS matrix"};
        if (p != c)
            for (int j = 0; j < 10; ++j) std::swap(m[p][j], m[c][j]);
        const double ip = 1.0 / m[c][c];
        for (int j = 0; j < 10; ++j) m[c][j] *= ip;
        for (int r = 0; r < 5; ++r)
            if (r != c) {
                const double f = m[r][c];
                if (f != 0.0)
                    for (int j = 0; j < 10; ++j) m[r][j] -= f * m[c][j];
            }
    }
    Blk o;
    for (int i = 0; i < 5; ++i)
        for (int j = 0; j < 5; ++j) o[i * 5 + j] = m[i][j + 5];
    return o;
}

// ------------------------------------------------------------------ geometry
struct HostMesh {
    int nt = 0, nf = 0;
    std::vector<double> vx, vy;            // [nt][3] unwrapped vertex coordinates
    std::vector<double> area, cx, cy, Ixx, Ixy, Iyy, h;
    std::vector<int> own, nbr, loc, tag;   // faces
    std::vector<double> nx, ny, S, gx, gy; // gx/gy [nf][2]
    std::vector<int> kord;                 // reconstruction order k_i
    std::vector<std::array<int, 3>> nb;    // interior neighbours per cell (face order), -1 padded
    std::vector<std::array<int, 3>> cf;    // faces per cell (code f or ~f)
    bool periodic[2] = {false, false};
    double L[2] = {0, 0};

    double mimg(double d, int ax) const {
        if (periodic[ax]) d -= L[ax] * std::nearbyint(d / L[ax]);
        return d;
    }
};

void build_host_mesh(const gks_mesh_desc* de, const gks_params* prm, HostMesh& hm) {
    const int nt = de->nt, nv = de->nv;
    hm.nt = nt;
    hm.periodic[0] = de->periodic_x != 0;
    hm.periodic[1] = de->periodic_y != 0;
    hm.L[0] = de->Lx;
    hm.L[1] = de->Ly;
    if ((hm.periodic[0] && !(de->Lx > 0)) || (hm.periodic[1] && !(de->Ly > 0)))
        throw Fail{GKS_EINVAL, "periodic axis needs a positive period"};
    hm.vx.resize(3 * (size_t)nt);
    hm.vy.resize(3 * (size_t)nt);
    hm.area.resize(nt);
    hm.cx.resize(nt);
    hm.cy.resize(nt);
    hm.Ixx.resize(nt);
    hm.Ixy.resize(nt);
    hm.Iyy.resize(nt);
    hm.h.resize(nt);
    int bad_tri = -1, bad_kind = 0;
#pragma omp parallel for schedule(static)
    for (int t = 0; t < nt; ++t) {
        int v[3];
        bool ok = true;
        for (int k = 0; k < 3; ++k) {
            v[k] = de->tri[3 * (size_t)t + k];
            if (v[k] < 0 || v[k] >= nv) ok = false;
        }
        if (!ok || v[0] == v[1] || v[1] == v[2] || v[0] == v[2]) {
#pragma omp critical
            if (bad_tri < 0 || t < bad_tri) {
                bad_tri = t;
                bad_kind = 1;
            }
            continue;
        }
        const double x0 = de->xy[2 * (size_t)v[0]], y0 = de->xy[2 * (size_t)v[0] + 1];
        double xs[3], ys[3];
        for (int k = 0; k < 3; ++k) {
            xs[k] = x0 + hm.mimg(de->xy[2 * (size_t)v[k]] - x0, 0);
            ys[k] = y0 + hm.mimg(de->xy[2 * (size_t)v[k] + 1] - y0, 1);
            hm.vx[3 * (size_t)t + k] = xs[k];
            hm.vy[3 * (size_t)t + k] = ys[k];
        }
        const double a = 0.5 * ((xs[1] - xs[0]) * (ys[2] - ys[0]) - (xs[2] - xs[0]) * (ys[1] - ys[0]));
        if (!(a > 0.0)) {
#pragma omp critical
            if (bad_tri < 0 || t < bad_tri) {
                bad_tri = t;
                bad_kind = 2;
            }
            continue;
        }
        const double cx = (xs[0] + xs[1] + xs[2]) / 3.0, cy = (ys[0] + ys[1] + ys[2]) / 3.0;
        double ixx = 0, ixy = 0, iyy = 0;
        for (int k = 0; k < 3; ++k) {
            ixx += (xs[k] - cx) * (xs[k] - cx);
            ixy += (xs[k] - cx) * (ys[k] - cy);
            iyy += (ys[k] - cy) * (ys[k] - cy);
        }
        const double la = std::hypot(xs[1] - xs[0], ys[1] - ys[0]);
        const double lb = std::hypot(xs[2] - xs[1], ys[2] - ys[1]);
        const double lc = std::hypot(xs[0] - xs[2], ys[0] - ys[2]);
        const double rad = la * lb * lc / (4.0 * a);
        hm.area[t] = a;
        hm.cx[t] = cx;
        hm.cy[t] = cy;
        hm.Ixx[t] = ixx / 12.0;
        hm.Ixy[t] = ixy / 12.0;
        hm.Iyy[t] = iyy / 12.0;
        hm.h[t] = std::max(rad, std::sqrt(a));
    }
    if (bad_tri >= 0) {
        if (bad_kind == 1) throw Fail{GKS_EINVAL, "triangle " + std::to_string(bad_tri) + " has an invalid or repeated vertex"};
        throw Fail{GKS_EINVAL, "triangle " + std::to_string(bad_tri) + " is clockwise or degenerate"};
    }

    // edges -> neighbours
    struct E {
        int64_t key;
        int t, e;
    };
    std::vector<E> edges(3 * (size_t)nt);
    for (int t = 0; t < nt; ++t)
        for (int e = 0; e < 3; ++e) {
            int a = de->tri[3 * (size_t)t + e], b = de->tri[3 * (size_t)t + (e + 1) % 3];
            if (a > b) std::swap(a, b);
            edges[3 * (size_t)t + e] = {(int64_t)a * nv + b, t, e};
        }
    std::sort(edges.begin(), edges.end(), [](const E& p, const E& q) {
        return p.key < q.key || (p.key == q.key && (p.t < q.t || (p.t == q.t && p.e < q.e)));
    });
    std::vector<int> across(3 * (size_t)nt, -1);
    for (size_t i = 0; i < edges.size();) {
        size_t j = i;
        while (j < edges.size() && edges[j].key == edges[i].key) ++j;
        if (j - i > 2) throw Fail{GKS_EINVAL, "non-manifold edge"};
        if (j - i == 2) {
            if (edges[i].t == edges[i + 1].t) throw Fail{GKS_EINVAL, "triangle shares an edge with itself"};
            across[3 * (size_t)edges[i].t + edges[i].e] = edges[i + 1].t;
            across[3 * (size_t)edges[i + 1].t + edges[i + 1].e] = edges[i].t;
        }
        i = j;
    }
    hm.nb.assign(nt, {-1, -1, -1});
    hm.cf.assign(nt, {0, 0, 0});
    std::vector<int> ncf(nt, 0), nnb(nt, 0);
    for (int t = 0; t < nt; ++t)
        for (int e = 0; e < 3; ++e) {
            const int o = across[3 * (size_t)t + e];
            if (o >= 0 && o < t) continue;
            int tg = 0;
            if (o < 0) {
                tg = de->edge_tag ? de->edge_tag[3 * (size_t)t + e] : 0;
                if (tg <= 0 || tg > de->n_bc) throw Fail{GKS_EINVAL, "open edge without a valid boundary tag"};
            }
            const int f = (int)hm.own.size();
            hm.own.push_back(t);
            hm.nbr.push_back(o);
            hm.loc.push_back(e);
            hm.tag.push_back(tg);
            hm.cf[t][ncf[t]++] = f;
            if (o >= 0) {
                hm.cf[o][ncf[o]++] = ~f;
                hm.nb[t][nnb[t]++] = o;
                hm.nb[o][nnb[o]++] = t;
            }
        }
    hm.nf = (int)hm.own.size();
    for (int t = 0; t < nt; ++t)
        if (ncf[t] != 3) throw Fail{GKS_EINVAL, "cell without three faces"};
    const int nf = hm.nf;
    hm.nx.resize(nf);
    hm.ny.resize(nf);
    hm.S.resize(nf);
    hm.gx.resize(2 * (size_t)nf);
    hm.gy.resize(2 * (size_t)nf);
    const double r3 = 1.0 / (2.0 * std::sqrt(3.0));
    for (int f = 0; f < nf; ++f) {
        const int t = hm.own[f], e = hm.loc[f];
        const double ax = hm.vx[3 * (size_t)t + e], ay = hm.vy[3 * (size_t)t + e];
        const double bx = hm.vx[3 * (size_t)t + (e + 1) % 3], by = hm.vy[3 * (size_t)t + (e + 1) % 3];
        const double dx = bx - ax, dy = by - ay;
        const double s = std::hypot(dx, dy);
        hm.S[f] = s;
        hm.nx[f] = dy / s;
        hm.ny[f] = -dx / s;
        const double mx = 0.5 * (ax + bx), my = 0.5 * (ay + by);
        hm.gx[2 * (size_t)f] = mx - dx * r3;
        hm.gy[2 * (size_t)f] = my - dy * r3;
        hm.gx[2 * (size_t)f + 1] = mx + dx * r3;
        hm.gy[2 * (size_t)f + 1] = my + dy * r3;
    }
    hm.kord.assign(nt, 2);
    if (!prm->all_quadratic)
        for (int f = 0; f < nf; ++f)
            if (hm.nbr[f] < 0) hm.kord[hm.own[f]] = 1;
}

// ------------------------------------------------------------------ CLS normal equations
// Per ordered neighbour pair (i, j): the weighted rows of Eqs. A:B:b:2-3.
void pair_blocks(const HostMesh& hm, int i, int j, double w, double A[6][5], double B[6][5]) {
    const double hi = hm.h[i], hj = hm.h[j];
    const double dx = hm.mimg(hm.cx[j] - hm.cx[i], 0) / hi;
    const double dy = hm.mimg(hm.cy[j] - hm.cy[i], 1) / hi;
    const double r = hi / hj, ih2 = 1.0 / (hi * hi);
    for (int a = 0; a < 6; ++a)
        for (int b = 0; b < 5; ++b) A[a][b] = B[a][b] = 0.0;
    // p = 0: cell-j means of the zero-mean basis of cell i
    A[0][0] = dx;
    A[0][1] = dy;
    A[0][2] = 0.5 * (dx * dx + (hm.Ixx[j] - hm.Ixx[i]) * ih2);
    A[0][3] = dx * dy + (hm.Ixy[j] - hm.Ixy[i]) * ih2;
    A[0][4] = 0.5 * (dy * dy + (hm.Iyy[j] - hm.Iyy[i]) * ih2);
    // p = 1, weight w h_i
    A[1][0] = w;
    A[1][2] = w * dx;
    A[1][3] = w * dy;
    A[2][1] = w;
    A[2][3] = w * dx;
    A[2][4] = w * dy;
    B[1][0] = w * r;
    B[2][1] = w * r;
    // p = 2, weight (w h_i)^2
    for (int q = 0; q < 3; ++q) {
        A[3 + q][2 + q] = w * w;
        B[3 + q][2 + q] = w * w * r * r;
    }
    if (hm.kord[i] == 1) {
        for (int a = 3; a < 6; ++a)
            for (int b = 0; b < 5; ++b) A[a][b] = B[a][b] = 0.0;
        for (int a = 0; a < 6; ++a)
            for (int b = 2; b < 5; ++b) A[a][b] = 0.0;
    }
    if (hm.kord[j] == 1)
        for (int a = 0; a < 6; ++a)
            for (int b = 2; b < 5; ++b) B[a][b] = 0.0;
}

Blk atb(const double A[6][5], const double B[6][5], double s) {
    Blk o = bzero();
    for (int k = 0; k < 5; ++k)
        for (int l = 0; l < 5; ++l) {
            double v = 0.0;
            for (int r = 0; r < 6; ++r) v += A[r][k] * B[r][l];
            o[k * 5 + l] = s * v;
        }
    return o;
}

struct Assembly {
    hvec<Blk> diag;                           // [nt]
    hvec<std::array<Blk, 3>> off;             // [nt][slot] block K_{i, nb[i][slot]}
    hvec<std::array<std::array<double, 5>, 3>> a0;  // [nt][slot]
};

// Row i of the normal equations gathers the rows of the pairs (i, j) (cell i
// reconstructed, blocks A_ij, B_ij) and (j, i) (cell i as the neighbour,
// blocks A_ji, B_ji) over its face neighbours j:
//   K_ii = sum_j A_ij^T A_ij + B_ji^T B_ji,   K_ij = -A_ij^T B_ij - B_ji^T A_ji.
void assemble(const HostMesh& hm, double w, Assembly& as) {
    const int nt = hm.nt;
    as.diag.resize(nt);
    as.off.resize(nt);
    as.a0.resize(nt);
#pragma omp parallel for schedule(static)
    for (int i = 0; i < nt; ++i) {
        Blk d = bzero();
        for (int s = 0; s < 3; ++s) {
            as.off[i][s] = bzero();
            as.a0[i][s].fill(0.0);
            const int j = hm.nb[i][s];
            if (j < 0) continue;
            double A[6][5], B[6][5], Aj[6][5], Bj[6][5];
            pair_blocks(hm, i, j, w, A, B);
            pair_blocks(hm, j, i, w, Aj, Bj);
            const Blk AtA = atb(A, A, 1.0), AtB = atb(A, B, 1.0), BjtBj = atb(Bj, Bj, 1.0), AjtBj = atb(Aj, Bj, 1.0);
            for (int e = 0; e < 25; ++e) d[e] += AtA[e] + BjtBj[e];
            for (int k = 0; k < 5; ++k)
                for (int l = 0; l < 5; ++l) as.off[i][s][k * 5 + l] = -AtB[k * 5 + l] - AjtBj[l * 5 + k];
            for (int l = 0; l < 5; ++l) as.a0[i][s][l] = A[0][l];
        }
        if (hm.kord[i] == 1)
            for (int l = 2; l < 5; ++l) d[l * 5 + l] += 1.0;
        as.diag[i] = d;
    }
}

// ------------------------------------------------------------------ orderings
std::vector<int> rcm_order(const HostMesh& hm) {
    const int nt = hm.nt;
    std::vector<int> deg(nt);
    for (int i = 0; i < nt; ++i) {
        int d = 0;
        for (int s = 0; s < 3; ++s) d += hm.nb[i][s] >= 0;
        deg[i] = d;
    }
    auto less = [&](int a, int b) { return deg[a] < deg[b] || (deg[a] == deg[b] && a < b); };
    std::vector<int> dist(nt, -1), q;
    q.reserve(nt);
    // breadth-first level structure of the component of root (left in q/dist);
    // returns the eccentricity of root
    auto bfs = [&](int root) {
        q.clear();
        q.push_back(root);
        dist[root] = 0;
        int ecc = 0;
        for (size_t p = 0; p < q.size(); ++p) {
            const int u = q[p];
            for (int s = 0; s < 3; ++s) {
                const int v = hm.nb[u][s];
                if (v >= 0 && dist[v] < 0) {
                    dist[v] = dist[u] + 1;
                    ecc = std::max(ecc, dist[v]);
                    q.push_back(v);
                }
            }
        }
        return ecc;
    };
    auto reset = [&]() {
        for (int u : q) dist[u] = -1;
    };
    std::vector<char> seen(nt, 0);
    std::vector<int> order;
    order.reserve(nt);
    for (int start = 0; start < nt; ++start) {
        if (seen[start]) continue;
        // George-Liu pseudo-peripheral node: start from a minimum-degree node
        // and move to the minimum-degree node of the last level while the
        // eccentricity grows
        bfs(start);
        int root = start;
        for (int u : q)
            if (less(u, root)) root = u;
        reset();
        int ecc = bfs(root);
        for (int it = 0; it < 32; ++it) {
            int cand = -1;
            for (int u : q)
                if (dist[u] == ecc && (cand < 0 || less(u, cand))) cand = u;
            reset();
            const int e2 = bfs(cand);
            if (e2 > ecc) {
                root = cand;
                ecc = e2;
            } else {
                break;
            }
        }
        reset();
        // Cuthill-McKee: breadth first, unvisited neighbours by (degree, index)
        const size_t base = order.size();
        order.push_back(root);
        seen[root] = 1;
        for (size_t p = base; p < order.size(); ++p) {
            const int u = order[p];
            int cand[3], nc = 0;
            for (int s = 0; s < 3; ++s) {
                const int v = hm.nb[u][s];
                if (v >= 0 && !seen[v]) cand[nc++] = v;
            }
            std::sort(cand, cand + nc, less);
            for (int k = 0; k < nc; ++k) {
                seen[cand[k]] = 1;
                order.push_back(cand[k]);
            }
        }
    }
    std::reverse(order.begin(), order.end());
    return order;
}

// ------------------------------------------------------------------ device helpers
// Handles may live on several host threads (one per stream).  Allocation,
// release and stream capture are serialised process-wide, and no library
// call synchronises the whole device or uses the legacy stream, so one
// handle's set-up or tear-down cannot disturb another handle's capture.
std::mutex g_dev_mu;

// Device memory of a handle.  Allocation is serialised; the copy or clear
// that follows runs on the handle's own stream outside the lock.
void* dev_malloc(gks_mesh* m, size_t bytes) {
    void* p = nullptr;
    std::lock_guard<std::mutex> lk(g_dev_mu);
    hipError_t e = hipMalloc(&p, bytes);
    if (e != hipSuccess) throw Fail{GKS_ENOMEM, "hipMalloc of " + std::to_string(bytes) + " bytes failed"};
    m->allocs.push_back(p);
    m->dev_bytes += (int64_t)bytes;
    return p;
}

template <typename T>
T* dev_alloc(gks_mesh* m, size_t count) {
    const size_t bytes = std::max<size_t>(1, count) * sizeof(T);
    T* p = (T*)dev_malloc(m, bytes);
    HIPCHK(hipMemsetAsync(p, 0, bytes, m->stream));   // set-up only, never captured
    return p;
}

// Host arrays bound for the device, sent in one transfer into one
// allocation; each array starts on a 256-byte boundary.  The device pointers
// are written by send(), which returns once the copy is complete.
struct Staging {
    struct Item {
        const void* src;
        size_t bytes;
        std::function<void(char*)> bind;
    };
    std::vector<Item> items;
    std::vector<std::shared_ptr<void>> held;   // arrays built only to be sent

    template <class Vec, class P>
    void add(const Vec& v, P* dst) {
        using T = typename Vec::value_type;
        static_assert(std::is_same<std::remove_cv_t<std::remove_pointer_t<P>>, T>::value, "element type");
        items.push_back({v.data(), v.size() * sizeof(T), [dst](char* a) { *dst = reinterpret_cast<P>(a); }});
    }
    template <class Vec, class P>
    void add_owned(Vec&& v, P* dst) {
        auto h = std::make_shared<std::decay_t<Vec>>(std::move(v));
        held.push_back(h);
        add(*h, dst);
    }
    void send(gks_mesh* m) {
        std::vector<size_t> off(items.size());
        size_t tot = 0;
        for (size_t k = 0; k < items.size(); ++k) {
            off[k] = tot;
            tot += (items[k].bytes + 255) / 256 * 256;
        }
        tot = std::max<size_t>(tot, 256);
        char* dev = (char*)dev_malloc(m, tot);
        hvec<char> host(tot);
        // copy in 4 MiB pieces spread over the threads
        constexpr size_t PIECE = (size_t)4 << 20;
        std::vector<std::pair<size_t, size_t>> pieces;   // (item, offset in it)
        for (size_t k = 0; k < items.size(); ++k)
            for (size_t o = 0; o < items[k].bytes; o += PIECE) pieces.push_back({k, o});
#pragma omp parallel for schedule(dynamic)
        for (int64_t q = 0; q < (int64_t)pieces.size(); ++q) {
            const Item& it = items[pieces[q].first];
            const size_t o = pieces[q].second;
            std::memcpy(host.data() + off[pieces[q].first] + o, (const char*)it.src + o, std::min(PIECE, it.bytes - o));
        }
        held.clear();   // everything is in the staging buffer now
        for (size_t k = 0; k < items.size(); ++k) {   // alignment gaps as zeros
            const size_t end = k + 1 < items.size() ? off[k + 1] : tot;
            std::memset(host.data() + off[k] + items[k].bytes, 0, end - off[k] - items[k].bytes);
        }
        HIPCHK(hipMemcpyAsync(dev, host.data(), tot, hipMemcpyHostToDevice, m->stream));
        HIPCHK(hipStreamSynchronize(m->stream));
        for (size_t k = 0; k < items.size(); ++k) items[k].bind(dev + off[k]);
    }
};

// Work arrays of a handle carved from one allocation (256-byte aligned
// pieces), cleared to zero on the handle's stream by commit().
struct Arena {
    std::vector<std::pair<size_t, std::function<void(char*)>>> items;   // offset, binder
    size_t tot = 0;
    template <class T>
    void add(T** dst, size_t count) {
        items.push_back({tot, [dst](char* a) { *dst = reinterpret_cast<T*>(a); }});
        tot += (std::max<size_t>(1, count) * sizeof(T) + 255) / 256 * 256;
    }
    void commit(gks_mesh* m) {
        char* dev = (char*)dev_malloc(m, std::max<size_t>(tot, 256));
        HIPCHK(hipMemsetAsync(dev, 0, std::max<size_t>(tot, 256), m->stream));   // set-up only, never captured
        for (auto& it : items) it.second(dev + it.first);
    }
};

// List of limited cells and their coefficients: at set-up when gks_step
// limits, else on the first gks_limit call.
void ensure_limit_buffers(gks_mesh* m) {
    if (m->w.lim_list) return;
    m->w.lim_list = dev_alloc<int32_t>(m, (size_t)m->d.nt);
    m->w.lim_buf = dev_alloc<double>(m, (size_t)20 * m->d.nt);
}

// Everything the device needs, built on the host (no HIP calls).
struct HostSystem {
    HostMesh hm;
    std::vector<int> perm;                        // solver order -> cell
    std::vector<int32_t> lev_ptr;
    int n_levels = 0, n_colors = 0, rcm_bw = 0, nfb = 0;
    hvec<double> Kval, a0c, Lval, Uval, Dv;
    // When the cell graph has no 3-cycles BILU(0) has no off-diagonal fill:
    // U = K_U and L = K_L D^-1 exactly, and the mixed-form inner sweeps use
    // the split form (K_L blocks in L's slots, E = D - K_D per row).
    bool tri_free = false;
    hvec<double> KLval, Ev;
    // split form, rows scaled by their pivot inverse: Dinv_i K_ik (k < i),
    // Dinv_i K_ij (j > i), Dinv_i E_i
    hvec<double> KLs, KUs, Gs;
    std::vector<int32_t> Kcol, nbc, iperm, Lcol, Ucol;
    std::vector<int32_t> worder;                  // SpMV order of the 64-row groups (multicolour only)
    std::vector<int32_t> own, nbr, cface, bck;
    std::vector<double> fgeo, gpd, cgeo, bcs;
};

// Entry-major [slots*25][n] -> vector-packed device layout (gks_internal.h).
template <typename T>
hvec<T> pack_blocks(const hvec<double>& src, int slots, int n, int np) {
    constexpr int V = 16 / sizeof(T);
    hvec<T> dst;
    par_fill(dst, (size_t)slots * 25 * np, T(0));
#pragma omp parallel for schedule(static)
    for (int i = 0; i < n; ++i)
        for (int s = 0; s < slots; ++s) {
            const size_t base = (size_t)s * 25 * np;
            for (int e = 0; e < 25; ++e) {
                const size_t at = e < 24 ? base + ((size_t)(e / V) * np + i) * V + e % V : base + (size_t)24 * np + i;
                dst[at] = (T)src[((size_t)s * 25 + e) * n + i];
            }
        }
    return dst;
}

// Slice tables of a factor stored as ELL [slots][n] with its real entries in
// the leading slots (padding = column n): slices of 64 rows inside each level,
// each as wide as its widest row.
struct SliceLayout {
    std::vector<int32_t> sbase;        // [levels + 1] first slice of each level
    std::vector<int32_t> off, w;       // [slices] first chunk, slots
    std::vector<double> lev_blocks;    // [levels] stored blocks (chunks * 64, rows that exist)
    int32_t chunks = 0;
};

SliceLayout slice_layout(const std::vector<int32_t>& col, int slots, int n, const std::vector<int32_t>& lev_ptr) {
    SliceLayout L;
    const int nl = (int)lev_ptr.size() - 1;
    L.sbase.assign(nl + 1, 0);
    L.lev_blocks.assign(nl, 0.0);
    for (int l = 0; l < nl; ++l) {
        L.sbase[l] = (int32_t)L.w.size();
        const int r1 = lev_ptr[l + 1];
        for (int r = lev_ptr[l]; r < r1; r += 64) {
            int w = 0;
            for (int i = r; i < std::min(r + 64, r1); ++i) {
                int c = 0;
                while (c < slots && col[(size_t)c * n + i] != n) ++c;
                w = std::max(w, c);
            }
            L.off.push_back(L.chunks);
            L.w.push_back(w);
            L.chunks += w;
            L.lev_blocks[l] += (double)w * (std::min(r + 64, r1) - r);
        }
    }
    L.sbase[nl] = (int32_t)L.w.size();
    return L;
}

// Blocks of an ELL factor in the sliced layout (element type T) and, when
// col_out is given, the column indices per chunk.
template <typename T>
hvec<T> pack_sliced(const hvec<double>& val, const std::vector<int32_t>& col, int n,
                           const std::vector<int32_t>& lev_ptr, const SliceLayout& L, std::vector<int32_t>* col_out) {
    constexpr int V = 16 / sizeof(T);
    const size_t nch = std::max<int32_t>(1, L.chunks);
    hvec<T> dst;
    par_fill(dst, nch * 25 * 64, T(0));
    if (col_out) col_out->assign(nch * 64, n);
    const int nl = (int)lev_ptr.size() - 1;
    for (int l = 0; l < nl; ++l) {
        const int r0 = lev_ptr[l], r1 = lev_ptr[l + 1];
        const int ns = L.sbase[l + 1] - L.sbase[l];
#pragma omp parallel for schedule(static)
        for (int k = 0; k < ns; ++k) {
            const int sl = L.sbase[l] + k;
            for (int s = 0; s < L.w[sl]; ++s) {
                const size_t ch = (size_t)L.off[sl] + s;
                for (int ln = 0; ln < 64; ++ln) {
                    const int i = r0 + 64 * k + ln;
                    if (i >= r1) break;
                    if (col_out) (*col_out)[ch * 64 + ln] = col[(size_t)s * n + i];
                    for (int e = 0; e < 25; ++e) {
                        const size_t at = e < 24 ? ch * 25 * 64 + ((size_t)(e / V) * 64 + ln) * V + e % V
                                                 : ch * 25 * 64 + 24 * 64 + ln;
                        dst[at] = (T)val[((size_t)s * 25 + e) * n + i];
                    }
                }
            }
        }
    }
    return dst;
}

void build_system(const gks_mesh_desc* de, const gks_params& prm, HostSystem& S) {
    PhaseTimer pt;
    HostMesh& hm = S.hm;
    build_host_mesh(de, &prm, hm);
    pt.mark("geometry + faces");
    const int nt = hm.nt, nf = hm.nf;
    Assembly as;
    assemble(hm, prm.cls_w, as);
    pt.mark("CLS assembly");

    // renumbering
    const std::vector<int> rcm = rcm_order(hm);
    std::vector<int> pos(nt);
    for (int p = 0; p < nt; ++p) pos[rcm[p]] = p;
    int bw = 0;
    for (int i = 0; i < nt; ++i)
        for (int s = 0; s < 3; ++s)
            if (hm.nb[i][s] >= 0) bw = std::max(bw, std::abs(pos[i] - pos[hm.nb[i][s]]));
    S.rcm_bw = bw;
    std::vector<int> key(nt, 0);
    int nkeys = 0;
    if (prm.ordering == GKS_ORDER_RCM) {
        // dependency level of each row of the lower factor in RCM order
        for (int p = 0; p < nt; ++p) {
            const int i = rcm[p];
            int lv = 0;
            for (int s = 0; s < 3; ++s) {
                const int j = hm.nb[i][s];
                if (j >= 0 && pos[j] < p) lv = std::max(lv, key[j] + 1);
            }
            key[i] = lv;
            nkeys = std::max(nkeys, lv + 1);
        }
        S.n_colors = 0;
    } else {
        std::vector<int> col(nt, -1);
        for (int p = 0; p < nt; ++p) {
            const int i = rcm[p];
            bool used[4] = {false, false, false, false};
            for (int s = 0; s < 3; ++s) {
                const int j = hm.nb[i][s];
                if (j >= 0 && col[j] >= 0) used[col[j]] = true;
            }
            int c = 0;
            while (used[c]) ++c;
            col[i] = c;
            nkeys = std::max(nkeys, c + 1);
        }
        // Order of the colour classes.  After the first sweep, level 0 has a
        // backward pass only and the last level a forward pass only, while
        // middle levels take both: the largest class goes first, the second
        // largest last, the smaller ones in between.
        if (nkeys >= 3) {
            std::vector<int> cnt(nkeys, 0), byc(nkeys), newc(nkeys);
            for (int i = 0; i < nt; ++i) ++cnt[col[i]];
            std::iota(byc.begin(), byc.end(), 0);
            std::stable_sort(byc.begin(), byc.end(), [&](int a, int b) { return cnt[a] > cnt[b]; });
            newc[byc[0]] = 0;
            newc[byc[1]] = nkeys - 1;
            for (int k = 2; k < nkeys; ++k) newc[byc[k]] = k - 1;
            for (int i = 0; i < nt; ++i) col[i] = newc[col[i]];
        }
        key = col;
        S.n_colors = nkeys;
    }
    // Rows of one level are independent.  Inside each window of 4096 rows of
    // a level (RCM order) they are sorted by their number of neighbours in
    // earlier levels, most first, so that 64-row slices of the factors have
    // uniform widths (see the sliced factor storage of the sweep kernels)
    // while a window keeps the spatial locality of its neighbour gathers.
    std::vector<int> nlow(nt, 0);
    for (int i = 0; i < nt; ++i)
        for (int s = 0; s < 3; ++s) {
            const int j = hm.nb[i][s];
            if (j >= 0 && key[j] < key[i]) ++nlow[i];
        }
    std::vector<int>& perm = S.perm;
    perm = rcm;  // new -> old
    std::stable_sort(perm.begin(), perm.end(), [&](int a, int b) { return key[a] < key[b]; });
    {
        constexpr int SORT_WINDOW = 4096;   // a multiple of the 64-row slice
        std::vector<int> lp(nkeys + 1, 0);
        for (int i = 0; i < nt; ++i) lp[key[i] + 1]++;
        for (int l = 0; l < nkeys; ++l) lp[l + 1] += lp[l];
        for (int l = 0; l < nkeys; ++l)
            for (int w0 = lp[l]; w0 < lp[l + 1]; w0 += SORT_WINDOW)
                std::stable_sort(perm.begin() + w0, perm.begin() + std::min(w0 + SORT_WINDOW, lp[l + 1]),
                                 [&](int a, int b) { return nlow[a] > nlow[b]; });
    }
    std::vector<int> iperm(nt);
    for (int p = 0; p < nt; ++p) iperm[perm[p]] = p;
    S.lev_ptr.assign(nkeys + 1, 0);
    for (int i = 0; i < nt; ++i) S.lev_ptr[key[i] + 1]++;
    for (int l = 0; l < nkeys; ++l) S.lev_ptr[l + 1] += S.lev_ptr[l];
    S.n_levels = nkeys;

    if (S.n_colors > 0) {
        // SpMV wave order: chunk k of every colour in turn (rows of a colour
        // are in RCM order, so chunk k covers about the same part of the mesh
        // in each colour); chunks of about 4096 rows of the largest colour
        const int nw = (nt + 63) / 64;
        const int nl = nkeys;
        std::vector<int> wa(nl + 1);
        for (int l = 0; l <= nl; ++l) wa[l] = (S.lev_ptr[l] + 63) / 64;   // waves whose first row is in level l
        int wmax = 1;
        for (int l = 0; l < nl; ++l) wmax = std::max(wmax, wa[l + 1] - wa[l]);
        const int K = std::max(1, (wmax + 63) / 64);
        S.worder.reserve(nw);
        for (int k = 0; k < K; ++k)
            for (int l = 0; l < nl; ++l) {
                const int64_t cnt = wa[l + 1] - wa[l];
                for (int64_t g = wa[l] + cnt * k / K; g < wa[l] + cnt * (k + 1) / K; ++g) S.worder.push_back((int32_t)g);
            }
        if ((int)S.worder.size() != nw) throw Fail{GKS_EINVAL, "internal: SpMV wave order does not cover the rows"};
    }
    pt.mark("ordering");
    // matrix in solver order: slot 0 diagonal, then neighbours, padded with the dummy row
    const int n = nt;
    hvec<double>& Kval = S.Kval;
    par_fill(Kval, (size_t)KW * 25 * n, 0.0);
    std::vector<int32_t>& Kcol = S.Kcol;
    Kcol.assign((size_t)KW * n, n);
    S.iperm.assign(iperm.begin(), iperm.end());
    S.nbc.assign((size_t)3 * n, 0);
    par_fill(S.a0c, (size_t)3 * 5 * n, 0.0);
    for (int o = 0; o < n; ++o)
        for (int s2 = 0; s2 < 3; ++s2) {
            const int j = hm.nb[o][s2];
            S.nbc[(size_t)s2 * n + o] = j >= 0 ? j : o;
            if (j >= 0)
                for (int l = 0; l < 5; ++l) S.a0c[((size_t)s2 * 5 + l) * n + o] = as.a0[o][s2][l];
        }
#pragma omp parallel for schedule(static)
    for (int i = 0; i < n; ++i) {
        const int o = perm[i];
        Kcol[i] = i;
        for (int e = 0; e < 25; ++e) Kval[(size_t)e * n + i] = as.diag[o][e];
        for (int s = 0; s < 3; ++s) {
            const int j = hm.nb[o][s];
            if (j < 0) continue;
            Kcol[(size_t)(s + 1) * n + i] = iperm[j];
            for (int e = 0; e < 25; ++e) Kval[((size_t)(s + 1) * 25 + e) * n + i] = as.off[o][s][e];
        }
    }

    pt.mark("ELL matrix");
    // BILU(0) in solver order: row-wise IKJ elimination restricted to the
    // pattern.  Rows of one level only read rows of earlier levels, so each
    // level is factored in parallel.
    hvec<Blk> rv((size_t)KW * n);   // entries [0, rnz[i]) of each row are written below
    std::vector<int> rc((size_t)KW * n), rnz(n);
#pragma omp parallel for schedule(static)
    for (int i = 0; i < n; ++i) {
        int nz = 0;
        for (int s2 = 0; s2 < KW; ++s2) {
            const int c = Kcol[(size_t)s2 * n + i];
            if (c == n) continue;
            rc[(size_t)KW * i + nz] = c;
            Blk& dst = rv[(size_t)KW * i + nz];
            for (int e = 0; e < 25; ++e) dst[e] = Kval[((size_t)s2 * 25 + e) * n + i];
            ++nz;
        }
        for (int a = 1; a < nz; ++a)
            for (int b = a; b > 0 && rc[(size_t)KW * i + b - 1] > rc[(size_t)KW * i + b]; --b) {
                std::swap(rc[(size_t)KW * i + b - 1], rc[(size_t)KW * i + b]);
                std::swap(rv[(size_t)KW * i + b - 1], rv[(size_t)KW * i + b]);
            }
        rnz[i] = nz;
    }
    pt.mark("BILU rows");
    hvec<Blk> dinv(n);
    int singular = -1;
    for (size_t l = 0; l + 1 < S.lev_ptr.size(); ++l) {
#pragma omp parallel for schedule(static)
        for (int i = S.lev_ptr[l]; i < S.lev_ptr[l + 1]; ++i) {
            const int* ci = &rc[(size_t)KW * i];
            Blk* vi = &rv[(size_t)KW * i];
            const int nz = rnz[i];
            for (int a = 0; a < nz && ci[a] < i; ++a) {
                const int k = ci[a];
                vi[a] = bmul(vi[a], dinv[k]);  // L_ik = A_ik U_kk^{-1}
                const int* ck = &rc[(size_t)KW * k];
                const Blk* vk = &rv[(size_t)KW * k];
                for (int b2 = 0; b2 < nz; ++b2) {
                    const int j = ci[b2];
                    if (j <= k) continue;
                    for (int q = 0; q < rnz[k]; ++q)
                        if (ck[q] == j) {
                            const Blk t = bmul(vi[a], vk[q]);
                            for (int e = 0; e < 25; ++e) vi[b2][e] -= t[e];
                        }
                }
            }
            int dpos = -1;
            for (int a = 0; a < nz; ++a)
                if (ci[a] == i) dpos = a;
            try {
                dinv[i] = binv(vi[dpos]);
            } catch (const Fail&) {
#pragma omp critical
                singular = i;
            }
        }
        if (singular >= 0) throw Fail{GKS_EINVAL, "singular pivot block in the CLS matrix"};
    }
    pt.mark("BILU elimination");
    hvec<double>& Lval = S.Lval;
    hvec<double>& Uval = S.Uval;
    hvec<double>& Dv = S.Dv;
    std::vector<int32_t>& Lcol = S.Lcol;
    std::vector<int32_t>& Ucol = S.Ucol;
    // the split form's blocks serve the mixed form only
    const bool want_split = prm.precision == GKS_MIXED;
    par_fill(Lval, (size_t)LW * 25 * n, 0.0);
    par_fill(Uval, (size_t)LW * 25 * n, 0.0);
    par_fill(Dv, (size_t)25 * n, 0.0);
    Lcol.assign((size_t)LW * n, n);
    Ucol.assign((size_t)LW * n, n);
    if (want_split) {
        par_fill(S.KLval, (size_t)LW * 25 * n, 0.0);
        par_fill(S.Ev, (size_t)25 * n, 0.0);
    }
#pragma omp parallel for schedule(static)
    for (int i = 0; i < n; ++i) {
        const int* ci = &rc[(size_t)KW * i];
        const Blk* vi = &rv[(size_t)KW * i];
        int nl = 0, nu = 0;
        for (int a = 0; a < rnz[i]; ++a) {
            const int c = ci[a];
            if (c < i) {
                Lcol[(size_t)nl * n + i] = c;
                for (int e = 0; e < 25; ++e) Lval[((size_t)nl * 25 + e) * n + i] = vi[a][e];
                for (int s2 = 0; s2 < KW && want_split; ++s2)
                    if (Kcol[(size_t)s2 * n + i] == c)
                        for (int e = 0; e < 25; ++e)
                            S.KLval[((size_t)nl * 25 + e) * n + i] = Kval[((size_t)s2 * 25 + e) * n + i];
                ++nl;
            } else if (c > i) {
                Ucol[(size_t)nu * n + i] = c;
                for (int e = 0; e < 25; ++e) Uval[((size_t)nu * 25 + e) * n + i] = vi[a][e];
                ++nu;
            } else {
                // E = D - K_D: the pivot block after elimination minus the diagonal of K
                if (want_split)
                    for (int e = 0; e < 25; ++e) S.Ev[(size_t)e * n + i] = vi[a][e] - Kval[(size_t)e * n + i];
            }
        }
        for (int e = 0; e < 25; ++e) Dv[(size_t)e * n + i] = dinv[i][e];
    }
    pt.mark("factor arrays");
    {
        // 3-cycles of the cell graph (three mutually adjacent cells)
        bool tri = false;
#pragma omp parallel for schedule(static) reduction(|| : tri)
        for (int i = 0; i < nt; ++i)
            for (int a = 0; a < 3; ++a)
                for (int b = a + 1; b < 3; ++b) {
                    const int j = hm.nb[i][a], k = hm.nb[i][b];
                    if (j < 0 || k < 0 || j == k) continue;
                    for (int c = 0; c < 3; ++c)
                        if (hm.nb[j][c] == k) tri = true;
                }
        S.tri_free = !tri;
    }
    if (S.tri_free && want_split) {
        // without fill U = K_U, so the split form's blocks are K_L, K_U, E
        // scaled from the left by the row's pivot inverse (every entry is
        // written below)
        S.KLs.resize((size_t)LW * 25 * n);
        S.KUs.resize((size_t)LW * 25 * n);
        S.Gs.resize((size_t)25 * n);
        auto scale = [&](const hvec<double>& src, hvec<double>& dst, int slots, int i) {
            for (int s2 = 0; s2 < slots; ++s2)
                for (int r = 0; r < 5; ++r)
                    for (int c = 0; c < 5; ++c) {
                        double t = 0.0;
                        for (int q = 0; q < 5; ++q)
                            t += Dv[(size_t)(5 * r + q) * n + i] * src[((size_t)s2 * 25 + 5 * q + c) * n + i];
                        dst[((size_t)s2 * 25 + 5 * r + c) * n + i] = t;
                    }
        };
#pragma omp parallel for schedule(static)
        for (int i = 0; i < n; ++i) {
            scale(S.KLval, S.KLs, LW, i);
            scale(Uval, S.KUs, LW, i);
            scale(S.Ev, S.Gs, 1, i);
        }
    }
    pt.mark("split-form blocks");
    // ---- face / cell arrays in device layout
    std::vector<int32_t>& own = S.own;
    std::vector<int32_t>& nbr = S.nbr;
    std::vector<double>& fgeo = S.fgeo;
    std::vector<double>& gpd = S.gpd;
    own.assign(nf, 0);
    nbr.assign(nf, 0);
    fgeo.assign(3 * (size_t)nf, 0.0);
    gpd.assign(8 * (size_t)nf, 0.0);
    int nfb = 0;
    for (int f = 0; f < nf; ++f) {
        own[f] = hm.own[f];
        nbr[f] = hm.nbr[f] >= 0 ? hm.nbr[f] : -hm.tag[f];
        nfb += hm.nbr[f] < 0;
        fgeo[f] = hm.nx[f];
        fgeo[(size_t)nf + f] = hm.ny[f];
        fgeo[2 * (size_t)nf + f] = hm.S[f];
        for (int g = 0; g < 2; ++g) {
            const double px = hm.gx[2 * (size_t)f + g], py = hm.gy[2 * (size_t)f + g];
            const int o = hm.own[f];
            gpd[(size_t)(4 * g + 0) * nf + f] = hm.mimg(px - hm.cx[o], 0) / hm.h[o];
            gpd[(size_t)(4 * g + 1) * nf + f] = hm.mimg(py - hm.cy[o], 1) / hm.h[o];
            const int b = hm.nbr[f];
            if (b >= 0) {
                gpd[(size_t)(4 * g + 2) * nf + f] = hm.mimg(px - hm.cx[b], 0) / hm.h[b];
                gpd[(size_t)(4 * g + 3) * nf + f] = hm.mimg(py - hm.cy[b], 1) / hm.h[b];
            }
        }
    }
    S.nfb = nfb;
    std::vector<double>& cgeo = S.cgeo;
    std::vector<int32_t>& cface = S.cface;
    cgeo.assign(4 * (size_t)nt, 0.0);
    cface.assign(3 * (size_t)nt, 0);
    for (int t = 0; t < nt; ++t) {
        const double h = hm.h[t];
        cgeo[t] = 1.0 / h;
        cgeo[(size_t)nt + t] = hm.Ixx[t] / (h * h);
        cgeo[2 * (size_t)nt + t] = hm.Ixy[t] / (h * h);
        cgeo[3 * (size_t)nt + t] = hm.Iyy[t] / (h * h);
        for (int k = 0; k < 3; ++k) cface[(size_t)k * nt + t] = hm.cf[t][k];
    }
    std::vector<int32_t>& bck = S.bck;
    std::vector<double>& bcs = S.bcs;
    bck.assign(de->n_bc + 1, 0);
    bcs.assign(4 * (size_t)(de->n_bc + 1), 0.0);
    for (int r = 0; r < de->n_bc; ++r) {
        const int k = de->bc_kind[r];
        if (k < GKS_BC_SLIP || k > GKS_BC_OUTFLOW) throw Fail{GKS_EINVAL, "unknown boundary kind"};
        bck[r + 1] = k;
        for (int q = 0; q < 4; ++q) bcs[4 * (size_t)(r + 1) + q] = de->bc_state ? de->bc_state[4 * (size_t)r + q] : 0.0;
        if (k == GKS_BC_INFLOW && !(bcs[4 * (size_t)(r + 1)] > 0 && bcs[4 * (size_t)(r + 1) + 3] > 0))
            throw Fail{GKS_EINVAL, "inflow state must have positive density and pressure"};
    }
    pt.mark("face and cell arrays");
}

void setup(gks_mesh* m, const gks_mesh_desc* de) {
    const gks_params& prm = m->prm;
    HostSystem S;
    build_system(de, prm, S);
    PhaseTimer pt;
    const HostMesh& hm = S.hm;
    const int nt = hm.nt, nf = hm.nf, n = nt;
    m->rcm_bw = S.rcm_bw;
    m->n_colors = S.n_colors;
    m->n_levels = S.n_levels;
    m->h_own = S.own;
    m->h_nbr = S.nbr;
    DevMesh& d = m->d;
    d.nt = nt;
    d.nf = nf;
    d.n = n;
    d.nfb = S.nfb;
    d.lev_ptr = S.lev_ptr;
    d.n_bc = de->n_bc;
    // Every array the device reads is gathered into one host buffer and
    // sent in one transfer: the handle's stream shares a hardware queue with
    // other handles' streams, so each separate transfer would wait behind
    // their queued kernels.
    Staging up;
    up.add(S.own, &d.own);
    up.add(S.nbr, &d.nbr);
    up.add(S.fgeo, &d.fgeo);
    up.add(S.gpd, &d.gpd);
    up.add(hm.area, &d.area);
    up.add(S.cgeo, &d.cgeo);
    up.add(S.cface, &d.cface);
    up.add(S.bck, &d.bc_kind);
    up.add(S.bcs, &d.bc_state);
    up.add(S.iperm, &d.iperm);
    up.add(S.nbc, &d.nbc);
    up.add(S.a0c, &d.a0c);
    d.np = (n + 3) / 4 * 4;
    const int np = d.np;
    up.add_owned(pack_blocks<double>(S.Kval, KW, n, np), &d.Kval);
    up.add(S.Kcol, &d.Kcol);
    if (!S.worder.empty()) up.add(S.worder, &d.worder);
    const SliceLayout Ls = slice_layout(S.Lcol, LW, n, S.lev_ptr);
    const SliceLayout Us = slice_layout(S.Ucol, LW, n, S.lev_ptr);
    {
        std::vector<int32_t> lcol, ucol;
        up.add_owned(pack_sliced<double>(S.Lval, S.Lcol, n, S.lev_ptr, Ls, &lcol), &d.Lval);
        up.add_owned(pack_sliced<double>(S.Uval, S.Ucol, n, S.lev_ptr, Us, &ucol), &d.Uval);
        up.add_owned(std::move(lcol), &d.Li.col);
        up.add_owned(std::move(ucol), &d.Ui.col);
    }
    up.add(Ls.off, &d.Li.off);
    up.add(Ls.w, &d.Li.w);
    up.add(Us.off, &d.Ui.off);
    up.add(Us.w, &d.Ui.w);
    d.Lsbase = Ls.sbase;
    d.Usbase = Us.sbase;
    d.lev_Lb = Ls.lev_blocks;
    d.lev_Ub = Us.lev_blocks;
    {
        const int nl = (int)S.lev_ptr.size() - 1;
        d.lev_Kb.assign(nl, 0.0);
        for (int l = 0; l < nl; ++l)
            for (int i = S.lev_ptr[l]; i < S.lev_ptr[l + 1]; ++i)
                for (int s2 = 0; s2 < KW; ++s2) d.lev_Kb[l] += S.Kcol[(size_t)s2 * n + i] != n ? 1.0 : 0.0;
    }
    if (prm.precision == GKS_MIXED) {
        d.split = S.tri_free;
        // split form: Dinv K_L and Dinv K_U in L's and U's slots; general
        // form: the factors L and U themselves
        up.add_owned(pack_sliced<float>(d.split ? S.KLs : S.Lval, S.Lcol, n, S.lev_ptr, Ls, nullptr), &d.Lval32);
        up.add_owned(pack_sliced<float>(d.split ? S.KUs : S.Uval, S.Ucol, n, S.lev_ptr, Us, nullptr), &d.Uval32);
    }
    up.add_owned(pack_blocks<double>(S.Dv, 1, n, np), &d.Dinv);
    if (prm.precision == GKS_MIXED) {
        if (d.split)
            up.add_owned(pack_blocks<float>(S.Gs, 1, n, np), &d.E32);   // Dinv E
        else
            up.add_owned(pack_blocks<float>(S.Kval, KW, n, np), &d.Kval32);
        up.add_owned(pack_blocks<float>(S.Dv, 1, n, np), &d.Dinv32);
    }
    up.add_owned(std::vector<double>((size_t)(MAXM + 1) * NC, 1.0), &m->w.ones);
    pt.mark("pack device layouts");
    up.send(m);
    pt.mark("upload");
    // ---- work space: one zeroed allocation
    Work& w = m->w;
    const size_t vec = (size_t)(n + 1) * CB;
    const int mres = prm.restart;
    Arena ws;
    ws.add(&w.X, vec);
    ws.add(&w.R, vec);
    ws.add(&w.V, vec * (mres + 1));
    if (prm.precision == GKS_MIXED) {
        ws.add(&w.Z, vec * mres);
        ws.add(&w.yf, vec);
        ws.add(&w.df, vec);
        ws.add(&w.bf, vec);
        if (prm.inner_solver == GKS_INNER_GMRES) {
            ws.add(&w.U, vec * (prm.inner_iters + 1));
            ws.add(&w.T, vec * prm.inner_iters);
            ws.add(&w.ks_in, 1);
        }
    }
    for (int i = 0; i < ring_slots(prm); ++i) ws.add(&w.H[i], vec);
    ws.add(&w.w, vec);
    ws.add(&w.t1, vec);
    ws.add(&w.t2, vec);
    ws.add(&w.t3, vec);
    w.nblk_red = std::max(1, std::min(1024, (n + 255) / 256));
    ws.add(&w.partial, (size_t)w.nblk_red * (MAXM + 1) * NC);
    ws.add(&w.npart, (size_t)NC * (((size_t)n * 10 + 255) / 256 + 5));   // blocks of k_axpy/k_axpy_dots
    ws.add(&w.dpart, (size_t)FUSED_DOTS_MAX * NC * (std::max<size_t>((n + 255) / 256, 2048) + 1));
    ws.add(&w.ks, 1);
    ws.add(&w.Xcell, (size_t)20 * nt);
    ws.add(&w.F, (size_t)4 * nf);
    ws.add(&w.Wn, (size_t)4 * nt);
    ws.add(&w.Wint, (size_t)4 * nt);
    ws.add(&w.dt_dev, 1);
    ws.add(&w.dtpart, 1024);
    ws.add(&w.counters, 4);
    ws.commit(m);
    if (prm.limiter) ensure_limit_buffers(m);
    {
        // pinned status words, read back by the host: one allocation
        constexpr size_t o_cnt = (sizeof(Status) + 63) / 64 * 64, o_scal = o_cnt + 64;
        char* hp = nullptr;
        std::lock_guard<std::mutex> lk(g_dev_mu);
        HIPCHK(hipHostMalloc((void**)&hp, o_scal + 4 * sizeof(double), hipHostMallocDefault));
        w.st_host = (Status*)hp;
        w.counters_host = (int32_t*)(hp + o_cnt);
        w.scal_host = (double*)(hp + o_scal);
    }
    launch_set_scalar(m, &w.ks->tol, prm.tol);
    launch_set_scalar(m, &w.ks->reorth_tol, prm.reorth_tol);
    if (w.ks_in) launch_set_scalar(m, &w.ks_in->reorth_tol, prm.reorth_tol);   // inner tolerance stays 0
    // device address of the static limiter scratch (gks_limit_noalloc), looked
    // up once per device with this handle's device current
    m->scratch = scratch_device_ptr(&m->scratch_err);
    pt.mark("work space");
}

// ------------------------------------------------------------------ GMRES driver (FP64)
void read_status(gks_mesh* m) {
    HIPCHK(hipMemcpyAsync(m->w.st_host, &m->w.ks->st, sizeof(Status), hipMemcpyDeviceToHost, m->stream));
    HIPCHK(hipStreamSynchronize(m->stream));
}

bool all_conv(const Status* s) {
    for (int c = 0; c < NC; ++c)
        if (!s->conv[c]) return false;
    return true;
}

// Restarted GMRES on the four columns in lockstep, right-preconditioned
// (FP64: BILU(0) in FP64) or flexible (mixed: the preconditioner is q =
// inner_iters sweeps of BILU(0)-preconditioned Richardson iteration on the
// FP32 copies of K and of the factors, z = M^-1 v; z += M^-1 (v - K z)).
// Arnoldi with classical Gram-Schmidt applied twice, Givens rotations and
// all convergence bookkeeping stay on the device (k_gmres_ctl); the host
// reads the status once per step.  The same launch sequence is issued
// eagerly or captured into a graph; in a graph the kernels are gated on the
// device flags st.run (Arnoldi steps) and st.fin (end of cycle), so the
// arithmetic is the same either way.

// norms of the right-hand side (ks->sq, written by the RHS launch), zero
// columns of X masked
void solve_begin(gks_mesh* m) {
    launch_ctl(m, 0);
    launch_mask_cols(m, m->w.X);
}

// r = R - K X, its norms, v_0 = r / |r|   (gate: st.fin in graphs)
void cycle_start(gks_mesh* m, const int32_t* gate) {
    Work& w = m->w;
    launch_resid(m, w.X, w.R, w.V, gate, w.ks->sq);
    launch_ctl(m, 1, gate != nullptr);
}

// Arnoldi step k: w = K M^-1 v_k, two Gram-Schmidt passes, |w|, Givens
void arnoldi_step(gks_mesh* m, int k, const int32_t* gate) {
    Work& w = m->w;
    KrylovState* ks = w.ks;
    const int64_t vs = (int64_t)(m->d.n + 1) * CB;
    double* vk = w.V + (int64_t)k * vs;
    double* vk1 = w.V + (int64_t)(k + 1) * vs;
    const double* sk = &ks->scale[k][0];
    const bool fused = k + 1 <= FUSED_DOTS_MAX;
    if (m->prm.precision == GKS_MIXED) {
        float* zk = w.Z + (int64_t)k * vs;
        launch_mx_precond(m, vk, sk, zk, gate, outer_step_sweeps(m, k));
        if (fused)
            launch_spmv64_f32x_dots(m, zk, w.w, w.V, vs, k + 1, &ks->scale[0][0], &ks->h1[0][0], gate);
        else
            launch_spmv64_f32x(m, zk, w.w, gate);
    } else {
        launch_ilu(m, vk, sk, w.t1, w.t2, gate);
        if (fused)
            launch_spmv64_dots(m, w.t2, w.w, w.V, vs, k + 1, &ks->scale[0][0], &ks->h1[0][0], gate);
        else
            launch_spmv64(m, w.t2, nullptr, w.w, gate);
    }
    // Classical Gram-Schmidt with a selective second pass (CGS2 where the
    // first pass leaves the new vector measurably non-orthogonal, see the
    // control kernel's mode 4): w1 = w - V h1 goes straight to slot k + 1
    // with h2 = V^T w1 and |w1|^2 (one fused pass while the basis is short,
    // separate ones beyond); the second pass v_{k+1} = w1 - V h2 (in place,
    // with its norm) runs only where the control kernel asks for it.
    if (fused) {
        launch_axpy_dots(m, w.V, vs, k + 1, &ks->h1[0][0], &ks->scale[0][0], w.w, vk1, &ks->h2[0][0], gate, ks->sq);
    } else {
        launch_dots_reduce(m, KC_DOTS, w.V, vs, k + 1, w.w, &ks->scale[0][0], &ks->h1[0][0], gate);
        launch_axpy(m, w.V, vs, k + 1, &ks->h1[0][0], &ks->scale[0][0], w.w, vk1, gate, ks->sq);
        launch_dots_reduce(m, KC_DOTS, w.V, vs, k + 1, vk1, &ks->scale[0][0], &ks->h2[0][0], gate);
    }
    launch_ctl(m, 4);
    launch_axpy(m, w.V, vs, k + 1, &ks->h2[0][0], &ks->scale[0][0], vk1, vk1, &ks->reorth, ks->sq, true);
    launch_ctl(m, 2);
}

// End of a cycle of nvec steps: y from the triangular system, then
// X += M^-1 (V y) (FP64) or X += Z y (mixed).  In graphs the device count
// st.k bounds nvec and st.fin gates the work.
void end_cycle(gks_mesh* m, int nvec, bool graph) {
    Work& w = m->w;
    KrylovState* ks = w.ks;
    const int64_t vs = (int64_t)(m->d.n + 1) * CB;
    const int32_t* gate = graph ? &ks->st.fin : nullptr;
    const int32_t* nvec_dev = graph ? &ks->st.k : nullptr;
    launch_ctl(m, 3, graph);
    if (m->prm.precision == GKS_MIXED) {
        launch_combine_f32(m, w.Z, vs, nvec, &ks->y[0][0], w.ones, w.X, nvec_dev, gate, true);   // X += Z y
    } else {
        launch_combine(m, w.V, vs, nvec, &ks->y[0][0], &ks->scale[0][0], w.t1, nvec_dev, gate);
        launch_ilu(m, w.t1, nullptr, w.t2, w.t3, gate);
        launch_acc(m, w.X, w.t3, gate);
    }
}

void fill_info(gks_mesh* m, gks_solve_info* info) {
    if (!info) return;
    const Status* st = m->w.st_host;
    for (int c = 0; c < NC; ++c) {
        info->iters[c] = st->its[c];
        info->restarts[c] = st->cycles;
        info->rel_resid[c] = st->bnorm[c] > 0.0 ? st->beta[c] / st->bnorm[c] : 0.0;
    }
    info->reorth = st->reorths;
    info->start_resid = start_resid(*st);
    info->start_points = m->last_npts;
    info->first_sweeps = m->prm.precision == GKS_MIXED && m->prm.inner_solver == GKS_INNER_RICHARDSON
                             ? outer_step_sweeps(m, 0) : 0;
}

enum { RESUME_NONE = 0, RESUME_CYCLE_START = 1, RESUME_IN_CYCLE = 2 };

// Host-driven cycles from the state the device holds.  RESUME_NONE: the
// solve starts (R is in place); RESUME_CYCLE_START: the status of a cycle
// start has been read; RESUME_IN_CYCLE: k0 steps of the current cycle are
// done.  Returns GKS_OK or GKS_ENOCONV; fills info.
int solve_loop(gks_mesh* m, gks_solve_info* info, int resume, int k0) {
    const Status* st = m->w.st_host;
    const int mres = m->prm.restart;
    if (resume == RESUME_NONE) solve_begin(m);
    int status = GKS_ENOCONV;
    for (;; resume = RESUME_NONE) {
        int k = 0;
        if (resume == RESUME_IN_CYCLE) {
            k = k0;
        } else {
            if (resume == RESUME_NONE) {
                cycle_start(m, nullptr);
                read_status(m);
            }
            if (all_conv(st)) {
                status = GKS_OK;
                break;
            }
            if (st->total >= m->prm.max_iter) break;
        }
        while (k < mres && st->total < m->prm.max_iter) {
            arnoldi_step(m, k, nullptr);
            ++k;
            read_status(m);
            if (all_conv(st)) break;
        }
        end_cycle(m, k, false);
    }
    fill_info(m, info);
    return status;
}

// ------------------------------------------------------------------ captured step graphs
// Graph A: RHS, solve set-up, the first cycle unrolled to `budget` gated
// Arnoldi steps, the gated end of cycle and the next cycle start.  Graph B:
// copy-out of X, fluxes and update.  Both read the handle's own buffers only
// (W is copied into Wint first), so they stay valid for any caller W.
void issue_solve_graph(gks_mesh* m, int budget) {
    KrylovState* ks = m->w.ks;
    launch_rhs(m, m->w.Wint, ks->sq);
    solve_begin(m);
    cycle_start(m, nullptr);
    for (int k = 0; k < budget; ++k) arnoldi_step(m, k, &ks->st.run);
    end_cycle(m, budget, true);
    cycle_start(m, &ks->st.fin);
}

// Continuation of a first cycle still running after graph A: Arnoldi step
// k, then the same gated end of cycle and next cycle start as graph A.
void issue_continue_graph(gks_mesh* m, int k) {
    KrylovState* ks = m->w.ks;
    arnoldi_step(m, k, &ks->st.run);
    end_cycle(m, k + 1, true);
    cycle_start(m, &ks->st.fin);
}

void issue_update_graph(gks_mesh* m) {
    Work& w = m->w;
    launch_copyout(m, w.X, w.Xcell);
    launch_zero_i32(m, w.counters, 4);
    // the limiter changes the flagged cells of Xcell in place
    if (m->prm.limiter) launch_limit(m, w.Wint, w.Xcell, nullptr, w.Xcell, 1.0, m->prm.limiter, w.counters + 2);
    launch_flux(m, w.Wint, w.Xcell, w.dt_dev, w.F);
    launch_update(m, w.Wint, w.F, w.Wn);
}

// A capture that did not produce an executable graph (nothing of it ran).
struct CaptureFailed {
    std::string msg;
};

template <typename F>
hipGraphExec_t capture(gks_mesh* m, F&& issue) {
    const auto t0 = std::chrono::steady_clock::now();
    struct Count {
        gks_mesh* m;
        std::chrono::steady_clock::time_point t0;
        ~Count() {
            ++m->captures;
            m->capture_ms += std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
        }
    } count{m, t0};
    std::lock_guard<std::mutex> lk(g_dev_mu);
    hipError_t e = hipStreamBeginCapture(m->stream, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) throw CaptureFailed{std::string("hipStreamBeginCapture: ") + hipGetErrorString(e)};
    m->capturing = true;
    std::string why;
    try {
        issue();
    } catch (const LaunchError& le) {
        why = std::string("launch of ") + le.kernel + ": " + hipGetErrorString(le.err);
    } catch (const Fail& f) {
        why = f.msg;
    }
    m->capturing = false;
    hipGraph_t g = nullptr;
    e = hipStreamEndCapture(m->stream, &g);
    if (why.empty() && e != hipSuccess) why = std::string("hipStreamEndCapture: ") + hipGetErrorString(e);
    hipGraphExec_t ex = nullptr;
    if (why.empty()) {
        e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
        if (e != hipSuccess) why = std::string("hipGraphInstantiate: ") + hipGetErrorString(e);
    }
    if (g) (void)hipGraphDestroy(g);
    if (!why.empty()) {
        (void)hipGetLastError();
        throw CaptureFailed{why};
    }
    return ex;
}

// The solve graph for (budget, first-step sweeps q1), from the handle's
// cache or captured into it; the cache is bounded, the least recently used
// graph going first (never the current gA).
hipGraphExec_t solve_graph_for(gks_mesh* m, int budget, int q1) {
    auto& c = m->gA_cache;
    auto hit = std::find_if(c.begin(), c.end(),
                            [&](const gks_mesh::GraphA& e) { return e.budget == budget && e.q1 == q1; });
    gks_mesh::GraphA e;
    if (hit != c.end()) {
        e = *hit;
        c.erase(hit);
    } else {
        if (c.size() >= (size_t)GRAPH_A_CACHE) {
            auto old = c.begin();
            if (old->ex == m->gA) ++old;
            (void)hipGraphExecDestroy(old->ex);
            c.erase(old);
        }
        const int keep = m->sw.q1;
        m->sw.q1 = q1;   // the count issue_solve_graph reads
        try {
            e = {budget, q1, capture(m, [&] { issue_solve_graph(m, budget); })};
        } catch (...) {
            m->sw.q1 = keep;
            throw;
        }
        m->sw.q1 = keep;
    }
    c.push_back(e);   // most recently used last
    return e.ex;
}

// Both step graphs, captured as needed before either is launched.
void ensure_graphs(gks_mesh* m) {
    const int cap = std::min(m->prm.restart, m->prm.max_iter);
    if (m->prm.graph_budget > 0) m->budget = std::min(cap, m->prm.graph_budget);
    if (m->budget <= 0) m->budget = cap;
    if (!m->gB) m->gB = capture(m, [&] { issue_update_graph(m); });
    const int q1 = outer_step_sweeps(m, 0);
    if (m->gA && m->gA_budget == m->budget && m->gA_q1 == q1) return;
    m->gA = solve_graph_for(m, m->budget, q1);
    m->gA_budget = m->budget;
    m->gA_q1 = q1;
}

// The solve graph the next step will want, captured while this step's graph
// B runs on the device (the capture is host work), so that a new budget or
// sweep count costs the next step no capture.  A failure here only leaves
// the capture to the next step.
void prepare_next_graph(gks_mesh* m, int outer) {
    const int q1 = next_first_sweeps(m, outer);
    if (m->budget <= 0 || (m->budget == m->gA_budget && q1 == m->gA_q1)) return;
    try {
        (void)solve_graph_for(m, m->budget, q1);
    } catch (const CaptureFailed&) {
    }
}

// The solve of a step through graph A.  A first cycle still running after
// it goes on one Arnoldi step per continuation graph C[k] (a status read
// after each, as the eager loop does); anything else (a restart, a capture
// that fails) continues on the host with the same arithmetic.  The adaptive
// budget is the shortest first cycle of the last 8 steps: every step pays
// for the steps graph A holds even when they are gated off (about 0.3 ms
// each at 10^6 cells, as the device overtakes the host's enqueueing of
// near-empty kernels), while a continuation costs one status read.
int solve_graph(gks_mesh* m, gks_solve_info* info) {
    const int cap = std::min(m->prm.restart, m->prm.max_iter);
    HIPCHK(hipGraphLaunch(m->gA, m->stream));
    read_status(m);
    const Status* st = m->w.st_host;
    bool graphs_ok = true;
    while (graphs_ok && !all_conv(st) && st->run && st->k > 0 && st->k < cap && st->total < m->prm.max_iter) {
        const int k = st->k;
        if ((int)m->gC.size() <= k) m->gC.resize(k + 1, nullptr);
        if (!m->gC[k]) {
            try {
                m->gC[k] = capture(m, [&] { issue_continue_graph(m, k); });
            } catch (const CaptureFailed& cf) {
                ++m->capture_failures;
                m->capture_err = cf.msg;
                graphs_ok = false;
                break;
            }
        }
        HIPCHK(hipGraphLaunch(m->gC[k], m->stream));
        read_status(m);
    }
    int r;
    if (all_conv(st)) {
        fill_info(m, info);
        r = GKS_OK;
    } else if (st->run && st->k > 0) {
        r = solve_loop(m, info, RESUME_IN_CYCLE, st->k);
    } else {
        r = solve_loop(m, info, RESUME_CYCLE_START, 0);
    }
    const int need = std::min(cap, std::max(1, (int)m->w.st_host->total));
    m->need_hist[m->need_n % 8] = need;
    ++m->need_n;
    if (m->prm.graph_budget <= 0) {
        int b = cap;
        for (int q = 0; q < std::min(m->need_n, 8); ++q) b = std::min(b, m->need_hist[q]);
        m->budget = b;
    }
    return r;
}

double ms_since(std::chrono::steady_clock::time_point t0) {
    return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
}

// RHS + solve; the solve's wall time (it synchronises on every convergence
// check, so host time measures the device work) goes to info->solve_ms.
int run_solve(gks_mesh* m, const double* W, gks_solve_info* info) {
    const auto t0 = std::chrono::steady_clock::now();
    launch_rhs(m, W, m->w.ks->sq);
    const int st = solve_loop(m, info, RESUME_NONE, 0);
    if (info) info->solve_ms = ms_since(t0);
    return st;
}

void prof_collect(gks_mesh* m) {
    if (m->prof.pending.empty()) return;
    HIPCHK(hipStreamSynchronize(m->stream));
    for (auto& p : m->prof.pending) {
        float ms = 0.0f;
        if (hipEventElapsedTime(&ms, p.second.first, p.second.second) == hipSuccess) {
            m->prof.ms[p.first] += ms;
            m->prof.launches[p.first] += 1;
        }
        m->prof.pool.push_back(p.second.first);
        m->prof.pool.push_back(p.second.second);
    }
    m->prof.pending.clear();
}

bool params_ok(const gks_params& p) {
    return p.gamma > 1.0 && p.cfl > 0.0 && p.tol > 0.0 && p.restart >= 1 && p.restart <= MAXM &&
           p.max_iter >= 1 && p.mu >= 0.0 && p.tau_eps >= 0.0 && p.cls_w > 0.0 &&
           (p.precision == GKS_FP64 || p.precision == GKS_MIXED) &&
           (p.ordering == GKS_ORDER_MULTICOLOR || p.ordering == GKS_ORDER_RCM) && p.inner_iters >= 1 &&
           (p.graphs == 0 || p.graphs == 1) && p.graph_budget >= 0 && (p.limiter == 0 || p.limiter == GKS_LIMIT_CONSERVATIVE || p.limiter == GKS_LIMIT_CHARACTERISTIC) &&
           p.reorth_tol >= 0.0 && p.reorth_tol < 1.0 &&
           p.inner_iters_first >= 0 && (p.adapt_sweeps == 0 || p.adapt_sweeps == 1) &&
           p.extrap_points >= 0 && p.extrap_points <= MAXH + 1 &&
           (p.inner_solver == GKS_INNER_RICHARDSON ||
            (p.inner_solver == GKS_INNER_GMRES && p.inner_iters <= FUSED_DOTS_MAX));
}

int fail(gks_mesh* m, const Fail& f) {
    if (m) m->err = f.msg;
    return f.code;
}

}  // namespace

// ================================================================== C ABI

extern "C" {

void gks_params_default(gks_params* p) {
    if (!p) return;
    std::memset(p, 0, sizeof(*p));
    p->gamma = 1.4;
    p->mu = 0.0;
    p->tau_eps = 0.01;
    p->cls_w = 0.3;
    p->cfl = 0.5;
    p->tol = 1e-10;
    p->restart = 30;
    p->max_iter = 500;
    p->precision = GKS_FP64;
    p->ordering = GKS_ORDER_MULTICOLOR;
    p->inner_iters = 4;
    p->inner_iters_first = 7;
    p->adapt_sweeps = 1;
    p->extrap_points = 0;
    p->exact_time = 0;
    p->nonphys_fallback = 0;
    p->all_quadratic = 0;
    p->graphs = 1;
    p->graph_budget = 0;
    p->limiter = 0;
    p->reorth_tol = REORTH_TOL_DEFAULT;
    p->inner_solver = GKS_INNER_RICHARDSON;
}

int gks_mesh_create(const gks_mesh_desc* desc, const gks_params* prm, void* hip_stream, gks_mesh** out) {
    if (out) *out = nullptr;
    g_create_err.clear();
    if (!desc || !out) {
        g_create_err = "null descriptor or output pointer";
        return GKS_EINVAL;
    }
    if (desc->nt <= 0 || desc->nv < 3 || !desc->xy || !desc->tri) {
        g_create_err = "mesh needs nt > 0, nv >= 3 and vertex/triangle arrays";
        return GKS_EINVAL;
    }
    if (desc->n_bc < 0 || (desc->n_bc > 0 && !desc->bc_kind)) {
        g_create_err = "boundary table is inconsistent";
        return GKS_EINVAL;
    }
    gks_params p;
    if (prm)
        p = *prm;
    else
        gks_params_default(&p);
    if (!params_ok(p)) {
        g_create_err = "invalid parameters";
        return GKS_EINVAL;
    }
    gks_mesh* m = new (std::nothrow) gks_mesh();
    if (!m) {
        g_create_err = "out of host memory";
        return GKS_ENOMEM;
    }
    m->prm = p;
    m->sw.q1 = top_sweeps(p);
    m->pts.P = start_points(p);
    m->stream = (hipStream_t)hip_stream;
    try {
        HIPCHK(hipGetDevice(&m->device));
        if (!m->stream) {
            std::lock_guard<std::mutex> lk(g_dev_mu);
            HIPCHK(hipStreamCreate(&m->stream));
            m->own_stream = true;
        }
        setup(m, desc);
    } catch (const Fail& f) {
        g_create_err = f.msg;
        const int code = f.code;
        gks_destroy(m);
        return code;
    } catch (const std::bad_alloc&) {
        g_create_err = "out of host memory";
        gks_destroy(m);
        return GKS_ENOMEM;
    }
    *out = m;
    return GKS_OK;
}

int gks_cls_reconstruct(gks_mesh* m, const double* W, double* X, gks_solve_info* info) {
    if (!m) return GKS_EINVAL;
    const auto t_call = std::chrono::steady_clock::now();
    if (!W || !X || (const void*)W == (const void*)X) {
        m->err = "null or aliased W / X";
        return GKS_EINVAL;
    }
    try {
        m->last_npts = 1;   // warm start from the handle's last solution
        const int st = run_solve(m, W, info);
        m->hist = st == GKS_OK ? 1 : 0;   // X is a solution, but not of the step sequence
        std::fill(m->dth, m->dth + MAXH + 1, 0.0);
        launch_copyout(m, m->w.X, X);
        HIPCHK(hipStreamSynchronize(m->stream));
        prof_collect(m);
        if (info) {
            info->nonphys = 0;
            info->call_ms = ms_since(t_call);
        }
        if (st != GKS_OK) m->err = "GMRES did not converge within max_iter";
        return st;
    } catch (const Fail& f) {
        return fail(m, f);
    } catch (const LaunchError& e) {
        return fail(m, Fail{GKS_EHIP, std::string("launch of ") + e.kernel + " failed: " + hipGetErrorString(e.err)});
    }
}

int gks_limit(gks_mesh* m, const double* W, const double* X, double* Xout, double threshold, int32_t variables,
              int32_t* n_limited) {
    if (!m) return GKS_EINVAL;
    if (!W || !X || !Xout || (const void*)X == (const void*)Xout || !(threshold == threshold)) {
        m->err = "gks_limit needs W, X, Xout (not aliasing X) and a threshold";
        return GKS_EINVAL;
    }
    if (variables != GKS_LIMIT_CONSERVATIVE && variables != GKS_LIMIT_CHARACTERISTIC) {
        m->err = "gks_limit: variables must be GKS_LIMIT_CONSERVATIVE or GKS_LIMIT_CHARACTERISTIC";
        return GKS_EINVAL;
    }
    try {
        ensure_limit_buffers(m);
        launch_zero_i32(m, m->w.counters, 4);
        launch_limit(m, W, X, Xout, Xout, threshold, variables, m->w.counters + 2);
        HIPCHK(hipMemcpyAsync(m->w.counters_host, m->w.counters, 4 * sizeof(int32_t), hipMemcpyDeviceToHost,
                              m->stream));
        HIPCHK(hipStreamSynchronize(m->stream));
        prof_collect(m);
        if (n_limited) *n_limited = m->w.counters_host[2];
        return GKS_OK;
    } catch (const Fail& f) {
        return fail(m, f);
    } catch (const LaunchError& e) {
        return fail(m, Fail{GKS_EHIP, std::string("launch of ") + e.kernel + " failed: " + hipGetErrorString(e.err)});
    }
}

int gks_limit_noalloc(gks_mesh* m, const double* W, const double* X, double* Xout, double threshold,
                      int32_t variables, int32_t* n_limited) {
    if (!m) return GKS_EINVAL;
    if (!W || !X || !Xout || (const void*)X == (const void*)Xout || !(threshold == threshold)) {
        m->err = "gks_limit_noalloc needs W, X, Xout (not aliasing X) and a threshold";
        return GKS_EINVAL;
    }
    if (variables != GKS_LIMIT_CONSERVATIVE && variables != GKS_LIMIT_CHARACTERISTIC) {
        m->err = "gks_limit_noalloc: variables must be GKS_LIMIT_CONSERVATIVE or GKS_LIMIT_CHARACTERISTIC";
        return GKS_EINVAL;
    }
    if (!m->scratch) {
        m->err = "gks_limit_noalloc: no static scratch on this device (" + m->scratch_err + ")";
        return GKS_EHIP;
    }
    try {
        launch_limit_noalloc(m, m->scratch, 1, W, X, Xout, threshold, variables);
        HIPCHK(hipMemcpyAsync(m->w.counters_host + 3, scratch_count(m->scratch), sizeof(int32_t),
                              hipMemcpyDeviceToHost, m->stream));
        HIPCHK(hipStreamSynchronize(m->stream));
        const int32_t cnt = m->w.counters_host[3];
        if (n_limited) *n_limited = cnt;
        if (cnt > GKS_LIMIT_NOALLOC_MAX_CELLS) {
            m->err = "gks_limit_noalloc: " + std::to_string(cnt) + " cells to limit exceed the static scratch (" +
                     std::to_string(GKS_LIMIT_NOALLOC_MAX_CELLS) + " cells); Xout holds X unlimited";
            return GKS_EINVAL;
        }
        if (cnt > 0) launch_limit_noalloc(m, m->scratch, 2, W, X, Xout, threshold, variables);
        HIPCHK(hipStreamSynchronize(m->stream));
        return GKS_OK;
    } catch (const Fail& f) {
        return fail(m, f);
    } catch (const LaunchError& e) {
        return fail(m, Fail{GKS_EHIP, std::string("launch of ") + e.kernel + " failed: " + hipGetErrorString(e.err)});
    }
}

int gks_apply_precond(gks_mesh* m, const double* V, double* Z, int form) {
    if (!m) return GKS_EINVAL;
    if (!V || !Z || (const void*)V == (const void*)Z) {
        m->err = "null or aliased V / Z";
        return GKS_EINVAL;
    }
    if (form != GKS_FP64 && !(form == GKS_MIXED && m->prm.precision == GKS_MIXED)) {
        m->err = "form must be GKS_FP64, or GKS_MIXED on a handle created with precision GKS_MIXED";
        return GKS_EINVAL;
    }
    try {
        Work& w = m->w;
        launch_copyin(m, V, w.t1);
        if (form == GKS_FP64) {
            launch_ilu(m, w.t1, nullptr, w.t2, w.t3);
            launch_copyout(m, w.t3, Z);
        } else {
            launch_mx_precond(m, w.t1, w.ones, w.Z);
            launch_copyout_f32(m, w.Z, Z);
        }
        HIPCHK(hipStreamSynchronize(m->stream));
        prof_collect(m);
        return GKS_OK;
    } catch (const Fail& f) {
        return fail(m, f);
    } catch (const LaunchError& e) {
        return fail(m, Fail{GKS_EHIP, std::string("launch of ") + e.kernel + " failed: " + hipGetErrorString(e.err)});
    }
}

int gks_flux(gks_mesh* m, const double* W, const double* X, double dt, double* F) {
    if (!m) return GKS_EINVAL;
    if (!W || !X || !F || !(dt > 0.0)) {
        m->err = "gks_flux needs W, X, F and dt > 0";
        return GKS_EINVAL;
    }
    try {
        launch_set_scalar(m, m->w.dt_dev, dt);
        launch_zero_i32(m, m->w.counters, 4);
        launch_flux(m, W, X, m->w.dt_dev, F);
        HIPCHK(hipMemcpyAsync(m->w.counters_host, m->w.counters, 4 * sizeof(int32_t), hipMemcpyDeviceToHost,
                              m->stream));
        HIPCHK(hipStreamSynchronize(m->stream));
        prof_collect(m);
        if (m->w.counters_host[0] > 0 && !m->prm.nonphys_fallback) {
            m->err = "non-physical reconstructed state at " + std::to_string(m->w.counters_host[0]) + " Gauss points";
            return GKS_ENONPHYS;
        }
        return GKS_OK;
    } catch (const Fail& f) {
        return fail(m, f);
    } catch (const LaunchError& e) {
        return fail(m, Fail{GKS_EHIP, std::string("launch of ") + e.kernel + " failed: " + hipGetErrorString(e.err)});
    }
}

int gks_step(gks_mesh* m, double* W, double dt, double* dt_used, gks_solve_info* info) {
    if (!m) return GKS_EINVAL;
    const auto t_call = std::chrono::steady_clock::now();
    if (!W) {
        m->err = "null W";
        return GKS_EINVAL;
    }
    const int hist = m->hist;
    m->hist = 0;   // until this step has succeeded
    try {
        Work& w = m->w;
        // initial guess of the solve: extrapolation of the last solutions
        int outer = 0;     // Arnoldi steps of this step's solve
        double r0s = 0.0;  // relative residual of its starting guess
        bool speculate = false;
        bool graphs = m->prm.graphs && !m->prof.on && m->capture_failures < 3;
        if (graphs) {
            try {
                ensure_graphs(m);
            } catch (const CaptureFailed& cf) {
                // eager launches for this step (same kernels, same result)
                ++m->capture_failures;
                m->capture_err = cf.msg;
                graphs = false;
            }
        }
        if (graphs) {
            // graph path: the step works on the handle's copy of W
            ++m->graph_steps;
            launch_copy(m, w.Wint, W, (int64_t)4 * m->d.nt);
            launch_extrap(m, hist);
            if (dt > 0.0)
                launch_set_scalar(m, w.dt_dev, dt);
            else
                launch_cfl(m, w.Wint, w.dt_dev);
            const auto t0 = std::chrono::steady_clock::now();
            const int st = solve_graph(m, info);
            if (info) info->solve_ms = ms_since(t0);
            if (st != GKS_OK) {
                HIPCHK(hipStreamSynchronize(m->stream));
                m->err = "GMRES did not converge within max_iter";
                return st;
            }
            outer = m->w.st_host->total;
            r0s = start_resid(*m->w.st_host);
            HIPCHK(hipGraphLaunch(m->gB, m->stream));
            speculate = true;
        } else {
            if (dt > 0.0)
                launch_set_scalar(m, w.dt_dev, dt);
            else
                launch_cfl(m, W, w.dt_dev);
            launch_zero_i32(m, w.counters, 4);
            launch_extrap(m, hist);
            const int st = run_solve(m, W, info);
            if (st != GKS_OK) {
                HIPCHK(hipStreamSynchronize(m->stream));
                prof_collect(m);
                m->err = "GMRES did not converge within max_iter";
                return st;
            }
            outer = m->w.st_host->total;
            r0s = start_resid(*m->w.st_host);
            launch_copyout(m, w.X, w.Xcell);
            if (m->prm.limiter) launch_limit(m, W, w.Xcell, nullptr, w.Xcell, 1.0, m->prm.limiter, w.counters + 2);
            launch_flux(m, W, w.Xcell, w.dt_dev, w.F);
            launch_update(m, W, w.F, w.Wn);
        }
        HIPCHK(hipMemcpyAsync(w.counters_host, w.counters, 4 * sizeof(int32_t), hipMemcpyDeviceToHost, m->stream));
        HIPCHK(hipMemcpyAsync(w.scal_host, w.dt_dev, sizeof(double), hipMemcpyDeviceToHost, m->stream));
        if (speculate) prepare_next_graph(m, outer);
        HIPCHK(hipStreamSynchronize(m->stream));
        if (info) {
            info->nonphys = w.counters_host[0];
            info->limited = w.counters_host[2];
        }
        if (dt_used) *dt_used = w.scal_host[0];
        if ((w.counters_host[0] > 0 && !m->prm.nonphys_fallback) || w.counters_host[1] > 0) {
            prof_collect(m);
            m->err = "non-physical state (" + std::to_string(w.counters_host[0]) + " Gauss points, " +
                     std::to_string(w.counters_host[1]) + " updated cells)";
            return GKS_ENONPHYS;
        }
        launch_copy(m, W, w.Wn, (int64_t)4 * m->d.nt);
        HIPCHK(hipStreamSynchronize(m->stream));
        prof_collect(m);
        if (info) info->call_ms = ms_since(t_call);
        m->hist = std::min(hist, ring_slots(m->prm)) + 1;
        push_step(m, w.scal_host[0]);
        adapt_first_sweeps(m, outer);
        adapt_points(m, r0s, m->last_npts, outer);
        return GKS_OK;
    } catch (const Fail& f) {
        return fail(m, f);
    } catch (const LaunchError& e) {
        return fail(m, Fail{GKS_EHIP, std::string("launch of ") + e.kernel + " failed: " + hipGetErrorString(e.err)});
    }
}

int gks_faces(const gks_mesh* m, int32_t* own, int32_t* nbr) {
    if (!m) return GKS_EINVAL;
    const size_t nf = m->h_own.size();
    if (own) std::memcpy(own, m->h_own.data(), nf * sizeof(int32_t));
    if (nbr) std::memcpy(nbr, m->h_nbr.data(), nf * sizeof(int32_t));
    return GKS_OK;
}

int gks_mesh_get_stats(const gks_mesh* m, gks_mesh_stats* st) {
    if (!m || !st) return GKS_EINVAL;
    st->nt = m->d.nt;
    st->nf = m->d.nf;
    st->nf_boundary = m->d.nfb;
    st->n_levels = m->n_levels;
    st->n_colors = m->n_colors;
    st->rcm_bandwidth = m->rcm_bw;
    st->device_bytes = m->dev_bytes;
    st->graph_steps = m->graph_steps;
    st->capture_failures = m->capture_failures;
    st->split_form = m->d.split ? 1 : 0;
    st->graph_captures = m->captures;
    st->capture_ms = m->capture_ms;
    return GKS_OK;
}

int gks_profile_enable(gks_mesh* m, int enable) {
    if (!m) return GKS_EINVAL;
    try {
        prof_collect(m);
    } catch (const Fail& f) {
        return fail(m, f);
    } catch (const LaunchError& e) {
        return fail(m, Fail{GKS_EHIP, std::string("launch of ") + e.kernel + " failed: " + hipGetErrorString(e.err)});
    }
    if (enable) {
        for (int i = 0; i < NPROF; ++i) {
            m->prof.launches[i] = 0;
            m->prof.ms[i] = 0.0;
            m->prof.bytes[i] = 0.0;
            m->prof.flops[i] = 0.0;
        }
    }
    m->prof.on = enable != 0;
    return GKS_OK;
}

int gks_profile_get(gks_mesh* m, int n, const char** names, int64_t* launches, double* total_ms,
                    double* total_bytes) {
    if (!m) return GKS_EINVAL;
    try {
        prof_collect(m);
    } catch (const Fail& f) {
        return fail(m, f);
    } catch (const LaunchError& e) {
        return fail(m, Fail{GKS_EHIP, std::string("launch of ") + e.kernel + " failed: " + hipGetErrorString(e.err)});
    }
    const int k = std::min(n, (int)KC_COUNT);
    for (int i = 0; i < k; ++i) {
        if (names) names[i] = kc_names[i];
        if (launches) launches[i] = m->prof.launches[i];
        if (total_ms) total_ms[i] = m->prof.ms[i];
        if (total_bytes) total_bytes[i] = m->prof.bytes[i];
    }
    return k;
}

int gks_host_inspect(const gks_mesh_desc* desc, const gks_params* prm, gks_host_system* out) {
    g_create_err.clear();
    if (!desc || !out || desc->nt <= 0 || desc->nv < 3 || !desc->xy || !desc->tri) {
        g_create_err = "invalid descriptor";
        return GKS_EINVAL;
    }
    std::memset(out, 0, sizeof(*out));
    gks_params p;
    if (prm)
        p = *prm;
    else
        gks_params_default(&p);
    if (!params_ok(p)) {
        g_create_err = "invalid parameters";
        return GKS_EINVAL;
    }
    try {
        HostSystem S;
        build_system(desc, p, S);
        const int nt = S.hm.nt, nf = S.hm.nf;
        out->nt = nt;
        out->nf = nf;
        out->n_levels = S.n_levels;
        out->n_colors = S.n_colors;
        out->rcm_bandwidth = S.rcm_bw;
        auto dup = [](const auto& v) {
            using T = typename std::decay_t<decltype(v)>::value_type;
            T* q = (T*)std::malloc(std::max<size_t>(1, v.size()) * sizeof(T));
            if (!q) throw std::bad_alloc();
            std::copy(v.begin(), v.end(), q);
            return q;
        };
        std::vector<int32_t> perm(S.perm.begin(), S.perm.end());
        out->own = dup(S.own);
        out->nbr = dup(S.nbr);
        out->area = dup(S.hm.area);
        out->h = dup(S.hm.h);
        out->perm = dup(perm);
        out->lev_ptr = dup(S.lev_ptr);
        out->kcol = dup(S.Kcol);
        out->kval = dup(S.Kval);
        out->lcol = dup(S.Lcol);
        out->lval = dup(S.Lval);
        out->ucol = dup(S.Ucol);
        out->uval = dup(S.Uval);
        out->dinv = dup(S.Dv);
        out->n_spmv_waves = (int32_t)S.worder.size();
        out->spmv_order = S.worder.empty() ? nullptr : dup(S.worder);
        (void)nf;
    } catch (const Fail& f) {
        g_create_err = f.msg;
        gks_host_free(out);
        return f.code;
    } catch (const std::bad_alloc&) {
        g_create_err = "out of host memory";
        gks_host_free(out);
        return GKS_ENOMEM;
    }
    return GKS_OK;
}

void gks_host_free(gks_host_system* s) {
    if (!s) return;
    void* ptrs[] = {s->own, s->nbr, s->area, s->h, s->perm, s->lev_ptr, s->kcol, s->kval,
                    s->lcol, s->lval, s->ucol, s->uval, s->dinv, s->spmv_order};
    for (void* q : ptrs) std::free(q);
    std::memset(s, 0, sizeof(*s));
}

const char* gks_last_error(const gks_mesh* m) {
    if (!m) return g_create_err.c_str();
    return m->err.c_str();
}

void gks_destroy(gks_mesh* m) {
    if (!m) return;
    if (m->stream) (void)hipStreamSynchronize(m->stream);
    std::lock_guard<std::mutex> lk(g_dev_mu);
    for (auto& p : m->prof.pending) {
        (void)hipEventDestroy(p.second.first);
        (void)hipEventDestroy(p.second.second);
    }
    for (auto e : m->prof.pool) (void)hipEventDestroy(e);
    for (auto& e : m->gA_cache) (void)hipGraphExecDestroy(e.ex);   // gA among them
    if (m->gB) (void)hipGraphExecDestroy(m->gB);
    for (hipGraphExec_t c : m->gC)
        if (c) (void)hipGraphExecDestroy(c);
    for (void* p : m->allocs) (void)hipFree(p);
    if (m->own_stream && m->stream) (void)hipStreamDestroy(m->stream);
    if (m->w.st_host) (void)hipHostFree(m->w.st_host);   // the status words share this allocation
    delete m;
}

}  // extern "C"
