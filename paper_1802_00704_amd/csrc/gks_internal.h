// Internal layout of a gks_mesh handle and the kernel launchers.
//
// Orders: "cell order" is the caller's triangle order; "solver order" is the
// renumbering used by the reconstruction solve (colour-major or RCM-level
// major, RCM inside).  perm[new] = old, iperm[old] = new.
//
// Solver vectors are cell-major: v[(i * NC + col) * NB + l] for cell i,
// conserved variable col (NC = 4) and coefficient l (NB = 5), so one cell's
// 4 x 5 block is 160 contiguous bytes.  Every vector has n + 1 cells; cell n
// is a zero dummy that padded matrix slots point at.
//
// Block-ELL matrices are uploaded "vector-packed": for slot s of row i the
// entries e < 24 of the 5 x 5 block (e = 5 r + c) lie at
// s*25*np + ((e / V) * np + i) * V + e % V (V = 4 floats or 2 doubles, 16
// bytes) and entry 24 at s*25*np + 24*np + i, np = n rounded up to 4, so each
// thread reads a block with 16-byte loads and a wave reads contiguous runs.
// (Host-side arrays, e.g. those of gks_host_inspect, are entry-major
// val[(slot * 25 + e) * n + i].)
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/gks.h"

namespace gks {

constexpr int NC = 4;             // conserved variables = right-hand-side columns
constexpr int NB = 5;             // coefficients per cell
constexpr int CB = NC * NB;       // doubles per cell in a solver vector
constexpr int KW = 4;             // ELL width of K (diagonal + 3 neighbours)
constexpr int LW = 3;             // ELL width of the strict lower / upper factors
constexpr int MAXM = 64;          // largest GMRES restart length
constexpr int NPROF = 24;         // profiled kernel classes
constexpr int MAXB = 16;          // handles per grouped launch
constexpr int GRAPH_A_CACHE = 8;  // solve graphs kept per handle
constexpr int MAXH = 5;           // earlier solutions kept for the extrapolated start

// State of the rule that adapts the points of the extrapolated start
// (points_rule).
struct PointsAdapt {
    int P = 0;                // points the starting guess takes
    int64_t step = 0;         // successful steps seen
    int64_t hold_until = 0;   // no trial before this step
    double r0[4] = {};        // starting residuals of the last steps at P
    int outer[4] = {};        // and their solves' Arnoldi steps
    int nr = 0;               // entries of r0 and outer filled
    int since = 0;            // steps at P since the last trial or change
    int prev = 0;             // the count before the running trial
    int fails = 0;            // trials in a row that did not start closer
    bool trial = false;       // this step tries prev - 1 or prev + 1 points
};

// State of the rule that adapts the mixed form's first-step sweep count
// (sweep_rule).
struct SweepAdapt {
    int q1 = 0;               // sweeps of the first outer step
    int64_t step = 0;         // successful steps seen
    int64_t hold_until = 0;   // no trial of a lower count before this step
    int ones = 0;             // solves in a row with one outer step
    int hard = 0;             // solves in a row with more than one
    int prev = 0;             // the count before the running trial
    int fails = 0;            // trials in a row that cost an outer step
    bool trial = false;       // this step tries a count one lower
};

struct Profile {
    bool on = false;
    int64_t launches[NPROF] = {0};
    double ms[NPROF] = {0};
    double bytes[NPROF] = {0};    // algorithmic bytes (what each launch must move)
    double flops[NPROF] = {0};
    std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> pending;
    std::vector<hipEvent_t> pool;
};

// Device-resident GMRES bookkeeping of one solve (one entry per column).
// The host reads only the leading Status block.
struct Status {
    double est[NC];               // |g_{k+1}| / ||R_c|| (estimate of the relative residual)
    double beta[NC];              // ||r_c|| at the start of the cycle (true residual)
    double beta0[NC];             // ||r_c|| of the starting guess (-1 until the first cycle starts)
    double bnorm[NC];             // ||R_c||
    int32_t k;                    // Arnoldi steps done in this cycle
    int32_t run;                  // 1 while the cycle continues (gates the iteration kernels)
    int32_t fin;                  // 1 once the cycle has ended (gates the end-of-cycle kernels)
    int32_t total;                // Arnoldi steps over all cycles of this solve
    int32_t cycles;               // cycles begun
    int32_t conv[NC];             // 1 once the estimate meets tol
    int32_t active[NC];           // 0 for a zero right-hand side
    int32_t its[NC];              // steps column c took part in before it converged
    int32_t reorths;              // Arnoldi steps of this solve that took the second Gram-Schmidt pass
};

// default of gks_params.reorth_tol
constexpr double REORTH_TOL_DEFAULT = 1e-8;

// largest relative residual of a solve's starting guess over the columns
// with a nonzero right-hand side
inline double start_resid(const Status& s) {
    double r = 0.0;
    for (int c = 0; c < NC; ++c)
        if (s.bnorm[c] > 0.0 && s.beta0[c] > 0.0) r = r > s.beta0[c] / s.bnorm[c] ? r : s.beta0[c] / s.bnorm[c];
    return r;
}

struct KrylovState {
    Status st;
    double tol;
    double scale[MAXM + 1][NC];   // v_j = scale_j * V_j (basis stored unnormalised)
    double h1[MAXM + 1][NC];      // first Gram-Schmidt pass
    double h2[MAXM + 1][NC];      // second pass
    double H[MAXM][MAXM + 1][NC]; // H[k][j]: column k after rotations
    double cs[MAXM][NC], sn[MAXM][NC];
    double g[MAXM + 1][NC];
    double y[MAXM][NC];
    double sq[NC];                // squared norms handed to the control kernel
    double reorth_tol;            // second Gram-Schmidt pass when |V^T w1| > reorth_tol |w1| (0: always)
    int32_t reorth;               // 1: the current Arnoldi step takes the second pass (gates it)
};

// Sliced storage of the BILU(0) factors (see the sweep kernels): per slice
// of 64 rows its first chunk and its number of slots; per chunk (one slot of
// one slice) 64 column indices.
struct SlicedIdx {
    const int32_t* col = nullptr;  // [chunk][64]
    const int32_t* off = nullptr;  // [slice] first chunk
    const int32_t* w = nullptr;    // [slice] slots
};

struct DevMesh {
    int nt = 0, nf = 0, nfb = 0;
    // faces (face order)
    int32_t* own = nullptr;       // [nf]
    int32_t* nbr = nullptr;       // [nf]  >= 0 cell, < 0: -(boundary row)
    double* fgeo = nullptr;       // [3][nf] nx, ny, S
    double* gpd = nullptr;        // [8][nf] (dx, dy) / h of GP g, side s at 2 (2 g + s) ..
    // cells (cell order)
    double* area = nullptr;       // [nt]
    double* cgeo = nullptr;       // [4][nt] 1/h, mxx, mxy, myy (second moments / h^2)
    int32_t* cface = nullptr;     // [3][nt] face f (owner) or ~f (neighbour)
    // boundary table
    int32_t* bc_kind = nullptr;   // [n_bc + 1]
    double* bc_state = nullptr;   // [n_bc + 1][4]
    int n_bc = 0;
    // solver (solver order)
    int n = 0;
    int np = 0;                   // row stride of the vector-packed matrices (n rounded up to 4)
    int32_t* iperm = nullptr;     // [nt] cell -> solver row
    int32_t* nbc = nullptr;       // [3][nt] face neighbours in cell order (self if none)
    double* a0c = nullptr;        // [3][5][nt] CLS row-0 coefficients per neighbour slot (cell order)
    double* Kval = nullptr;       // [KW][25][n]
    int32_t* Kcol = nullptr;      // [KW][n] (n = dummy)
    int32_t* worder = nullptr;    // [ceil(n / 64)] order in which the SpMV kernels take the 64-row
                                  // groups (multicolour: a spatial chunk of every colour in turn);
                                  // null: natural order
    float* Kval32 = nullptr;
    double* Lval = nullptr;       // sliced [chunk][25 * 64] strict lower factor blocks
    double* Uval = nullptr;       // sliced [chunk][25 * 64] strict upper factor blocks
    SlicedIdx Li{}, Ui{};         // their column indices and slice tables
    double* Dinv = nullptr;       // [25][np] inverted pivot blocks
    float* Lval32 = nullptr;      // sliced FP32: L, or Dinv K_L in the split form
    float* Uval32 = nullptr;      // sliced FP32: U, or Dinv K_U (U = K_U) in the split form
    float* Dinv32 = nullptr;
    float* E32 = nullptr;         // split form: [25][np] Dinv (D - K_D)
    bool split = false;           // mixed inner sweeps in the split form (cell graph without 3-cycles)
    std::vector<int32_t> lev_ptr; // host: rows of level l are [lev_ptr[l], lev_ptr[l+1])
    std::vector<int32_t> Lsbase, Usbase;  // host: first slice of each level
    std::vector<double> lev_Kb, lev_Lb, lev_Ub;  // host: stored K, L, U blocks per level
};

struct Work {
    double* X = nullptr;          // [n+1][CB] current solution (warm start)
    double* R = nullptr;          // [n+1][CB] right-hand side
    double* V = nullptr;          // [(m+1)][n+1][CB] Krylov basis
    float* Z = nullptr;           // [m][n+1][CB] flexible GMRES: preconditioned basis (FP32)
    float* yf = nullptr;          // [n+1][CB] mixed inner sweeps: forward result
    float* df = nullptr;          // [n+1][CB] mixed inner sweeps: correction
    float* bf = nullptr;          // [n+1][CB] mixed inner sweeps: FP32 right-hand side
    double* npart = nullptr;      // per-block partial sums of the fused norms: [4][blocks of 10 n threads]
    double* dpart = nullptr;      // per-block partial dots of the fused Gram-Schmidt passes
    double* H[MAXH] = {};         // [n][CB] earlier solutions, a ring
                                  // (ring_slots(prm) of them; newest at gks_mesh::hring)
    double* w = nullptr;          // [n+1][CB]
    double* t1 = nullptr;         // [n+1][CB]
    double* t2 = nullptr;         // [n+1][CB]
    double* t3 = nullptr;         // [n+1][CB]
    double* ones = nullptr;       // [MAXM + 1][NC] unit scale factors
    double* partial = nullptr;    // block partial sums
    int nblk_red = 0;             // blocks of the reduction kernels
    KrylovState* ks = nullptr;    // device
    double* U = nullptr;          // [(inner_iters+1)][n+1][CB] inner GMRES basis (mixed form, inner GMRES)
    float* T = nullptr;           // [inner_iters][n+1][CB] its preconditioned basis (FP32)
    KrylovState* ks_in = nullptr; // device: the inner GMRES state
    Status* st_host = nullptr;    // pinned mirror of ks->st
    double* Xcell = nullptr;
    int32_t* lim_list = nullptr;  // [nt] cells the limiter changes (allocated on first use)
    double* lim_buf = nullptr;    // [20][nt] their limited coefficients, by list position      // [4][5][nt] X in cell order (gks_step)
    double* F = nullptr;          // [4][nf]
    double* Wn = nullptr;         // [4][nt]
    double* Wint = nullptr;       // [4][nt] the step's copy of W (graph path)
    double* dt_dev = nullptr;     // [1]
    double* dtpart = nullptr;     // block minima of the CFL rule
    int32_t* counters = nullptr;  // [4] nonphysical count, ...
    int32_t* counters_host = nullptr;
    double* scal_host = nullptr;  // pinned scalars
};

}  // namespace gks

struct gks_mesh {
    gks_params prm;
    hipStream_t stream = nullptr;
    int device = 0;
    gks::DevMesh d;
    gks::Work w;
    gks::Profile prof;
    std::vector<int32_t> h_own, h_nbr;
    int n_levels = 0, n_colors = 0, rcm_bw = 0;
    int64_t dev_bytes = 0;
    std::vector<void*> allocs;
    bool have_x = false;
    bool capturing = false;       // a stream capture is in progress (no profiling events)
    bool own_stream = false;      // the handle created m->stream itself
    // captured step graphs (see gks_step): A = solve with a fixed iteration
    // budget and first-step sweep count (one graph per pair in gA_cache), B =
    // copy-out, flux, update; C[k] = Arnoldi step k of a cycle still running
    // after A, with the gated end of cycle (captured on first need)
    hipGraphExec_t gA = nullptr, gB = nullptr;
    std::vector<hipGraphExec_t> gC;
    int gA_budget = 0;            // Arnoldi steps captured in gA
    int gA_q1 = 0;                // first-step sweeps captured in gA
    struct GraphA {
        int budget, q1;
        hipGraphExec_t ex;
    };
    std::vector<GraphA> gA_cache; // solve graphs by (budget, first-step sweeps), gA among them
    // mixed form: Richardson sweeps of the first outer step, adapted between
    // steps (see adapt_first_sweeps)
    gks::SweepAdapt sw;
    // points of the extrapolated start, adapted between steps when
    // extrap_points is 0 (see points_rule)
    gks::PointsAdapt pts;
    int last_npts = 0;            // points the last starting guess took
    int budget = 0;               // steps wanted in gA for the next step
    int need_hist[8] = {0};       // first-cycle lengths of the last steps
    int need_n = 0;               // entries of need_hist filled
    int hist = 0;                 // solutions held in X and the ring w.H (extrapolated guess)
    int hring = 0;                // slot of w.H holding the newest earlier solution
    double dth[gks::MAXH + 1] = {}; // time steps taken from X, then from the ring's solutions
                                  // (newest first; hist of them are valid)
    int64_t graph_steps = 0;      // steps run through the graphs
    int capture_failures = 0;     // captures that failed (3 turn graphs off)
    int captures = 0;             // captures attempted
    double capture_ms = 0.0;      // host time in them
    std::string capture_err;      // the last capture failure
    void* scratch = nullptr;      // device address of the static limiter scratch on this
                                  // handle's device (gks_limit_noalloc), or null
    std::string scratch_err;      // why the scratch lookup failed
    std::string err;
};

namespace gks {

// thrown by a launcher whose kernel launch reported an error
struct LaunchError {
    hipError_t err;
    const char* kernel;
};

// kernel classes for profiling
enum Kc {
    KC_RHS = 0, KC_SPMV, KC_SPMV_RES, KC_ILU_FWD, KC_ILU_BWD, KC_DOTS, KC_AXPY_DOTS, KC_REORTH,
    KC_FINAL, KC_COMBINE, KC_AXPY, KC_COPYOUT, KC_FLUX, KC_UPDATE, KC_CFL, KC_MISC,
    KC_SPMV32, KC_ILU_FWD32, KC_ILU_BWD32, KC_EXTRAP, KC_LIMIT, KC_LIMIT_APPLY, KC_COUNT
};
extern const char* kc_names[NPROF];

// launchers (gks_kernels.hip); all enqueue on m->stream
// sq_out (device, 4 doubles): when given, also the per-column sums of R^2
void launch_rhs(gks_mesh* m, const double* W, double* sq_out = nullptr);
// gate: device flag; when non-null and zero the kernels return at once (used to
// unroll a fixed iteration budget into a captured graph).
void launch_spmv64(gks_mesh* m, const double* x, const double* xscale, double* y, const int32_t* gate = nullptr);
void launch_spmv64_f32x(gks_mesh* m, const float* x, double* y, const int32_t* gate = nullptr);
// sq_out: when given, also the per-column sums of y^2 (fused reduction)
void launch_resid(gks_mesh* m, const double* x, const double* b, double* y, const int32_t* gate = nullptr,
                  double* sq_out = nullptr);
void launch_ilu(gks_mesh* m, const double* in, const double* in_scale, double* tmp, double* out,
                const int32_t* gate = nullptr);
// z = P(s .* v): the mixed form's inner iteration, inner_iters sweeps
void launch_mx_precond(gks_mesh* m, const double* v, const double* vscale, float* z, const int32_t* gate = nullptr,
                       int q = 0);
// Richardson sweeps of the mixed form's preconditioner at Arnoldi step k of a
// cycle: the handle's first-step count (inner_iters_first, adapted) in the
// first step, else inner_iters
int outer_step_sweeps(const gks_mesh* m, int k);
// the rule's update after a successful step whose solve took outer_steps
// Arnoldi steps; top = the starting count
void sweep_rule(SweepAdapt& s, int outer_steps, int top);
// the handle's count after such a step, without changing the handle
int next_first_sweeps(const gks_mesh* m, int outer_steps);
// the rule applied to the handle (a no-op unless adaptation is on)
void adapt_first_sweeps(gks_mesh* m, int outer_steps);
// the points rule's update after a successful step whose start took used
// points and had relative residual r0, and whose solve took outer Arnoldi
// steps; tol = the solve tolerance
void points_rule(PointsAdapt& s, double r0, int used, int outer, double tol);
// the rule applied to the handle (a no-op unless extrap_points is 0)
void adapt_points(gks_mesh* m, double r0, int used, int outer);
void launch_dots_reduce(gks_mesh* m, int kc, const double* V, int64_t vstride, int nvec, const double* w,
                        const double* scale, double* out, const int32_t* gate = nullptr);
// second_pass: the gated second Gram-Schmidt pass (profiler class "reorth")
void launch_axpy(gks_mesh* m, const double* V, int64_t vstride, int nvec, const double* h, const double* scale,
                 const double* w, double* out, const int32_t* gate = nullptr, double* sq_out = nullptr,
                 bool second_pass = false);
// Fused Gram-Schmidt passes for nvec <= FUSED_DOTS_MAX basis vectors:
// y = K x together with out = scale .* (V^T y), and the update out = w - V h
// together with dots_out = scale .* (V^T out) and, with sq_out, the
// per-column squared norms of out.
constexpr int FUSED_DOTS_MAX = 8;
void launch_spmv64_dots(gks_mesh* m, const double* x, double* y, const double* V, int64_t vstride, int nvd,
                        const double* scale, double* out, const int32_t* gate = nullptr);
void launch_spmv64_f32x_dots(gks_mesh* m, const float* x, double* y, const double* V, int64_t vstride, int nvd,
                             const double* scale, double* out, const int32_t* gate = nullptr);
void launch_axpy_dots(gks_mesh* m, const double* V, int64_t vstride, int nvec, const double* h, const double* scale,
                      const double* w, double* out, double* dots_out, const int32_t* gate = nullptr,
                      double* sq_out = nullptr);
// nvec_dev: when non-null the number of vectors is min(nvec, *nvec_dev)
void launch_combine(gks_mesh* m, const double* V, int64_t vstride, int nvec, const double* y, const double* scale,
                    double* out, const int32_t* nvec_dev = nullptr, const int32_t* gate = nullptr);
// accum: out += the combination instead of out = it
void launch_combine_f32(gks_mesh* m, const float* V, int64_t vstride, int nvec, const double* y, const double* scale,
                        double* out, const int32_t* nvec_dev = nullptr, const int32_t* gate = nullptr,
                        bool accum = false);
void launch_acc(gks_mesh* m, double* X, const double* z, const int32_t* gate = nullptr);
// mode 0: norms of the right-hand side; 1: start of a cycle (true residual);
// 2: Arnoldi step (skipped once st.run is 0); 3: triangular solve for y.
// gated: skip unless st.fin is 1 (end-of-cycle work in a captured graph).
void launch_ctl(gks_mesh* m, int mode, bool gated = false);
// the control kernel on another Krylov state (the inner GMRES), restart mres
void launch_ctl_ks(gks_mesh* m, KrylovState* ks, int mode, int mres);
void launch_mask_cols(gks_mesh* m, double* X);
void launch_copyout(gks_mesh* m, const double* Xs, double* Xcell);
void launch_copyout_f32(gks_mesh* m, const float* Xs, double* Xcell);
void launch_copyin(gks_mesh* m, const double* Xcell, double* Xs);
// initial guess of a step's solve from the last solutions (order 0, 1, 2)
// and shift of the history
// earlier solutions kept for the starting guess: extrap_points - 1, or all
// MAXH slots when the point count adapts (extrap_points = 0)
inline int ring_slots(const gks_params& p) { return p.extrap_points > 0 ? p.extrap_points - 1 : MAXH; }
// point count a handle starts with: extrap_points, or when that is 0, 6 (3
// with the limiter on: limited cells switching between steps make the
// solutions less smooth in time)
inline int start_points(const gks_params& p) { return p.extrap_points > 0 ? p.extrap_points : (p.limiter ? 3 : 6); }
// starting guess from npts (1..extrap_points) solutions: X and npts - 1 ring
// slots; stores X in the ring and rotates it
void launch_extrap(gks_mesh* m, int npts);
// after a successful step of size dt
void push_step(gks_mesh* m, double dt);
void launch_flux(gks_mesh* m, const double* W, const double* X, const double* dt_dev, double* F);
// DWBAP limiter: Xout = limited X where IS_i >= threshold (count += limited cells)
// DWBAP limiter: cells whose indicator reaches threshold get limited
// coefficients in dst; with Xcopy set, X is first copied there for every
// cell (dst may then be Xcopy; otherwise dst already holds X, e.g. dst == X
// is allowed as nothing of X is read after the apply kernel).
void launch_limit(gks_mesh* m, const double* W, const double* X, double* Xcopy, double* dst, double threshold,
                  int variables, int32_t* count);
void launch_update(gks_mesh* m, const double* W, const double* F, double* Wn);
// Static scratch of gks_limit_noalloc (a file-scope device array of the
// kernel library): its address on the current device, looked up once per
// device (null on failure, err set); the limiter on it in two phases (1:
// copy X to Xout, clear and mark; 2: limit the listed cells and scatter);
// the device address of its count of limited cells.
void* scratch_device_ptr(std::string* err);

// ---------------------------------------------------------------- grouped launches (gks_batch_step)
// Each call launches its kernels once for all the handles given (at most
// MAXB = 16 per launch, more are split), each handle with the arguments and
// grid of its own launch, on stream st; see the single-handle launchers of
// the same names for what each computes.
struct BatchSlot {                // one handle's state as read back by the host
    Status st;
    int32_t counters[4];
    double dt;
};
void glaunch_gather(hipStream_t st, const std::vector<gks_mesh*>& ms, const std::vector<BatchSlot*>& out,
                    bool counters);
// counters = 0 and, where dt[r] > 0, the step's dt set to it
void glaunch_zero_counters(hipStream_t st, const std::vector<gks_mesh*>& ms, const std::vector<double>& dt);
void glaunch_cfl(hipStream_t st, const std::vector<gks_mesh*>& ms, const std::vector<const double*>& W);
void glaunch_extrap(hipStream_t st, const std::vector<gks_mesh*>& ms, const std::vector<int>& npts);
void glaunch_rhs(hipStream_t st, const std::vector<gks_mesh*>& ms, const std::vector<const double*>& W);
void glaunch_ctl(hipStream_t st, const std::vector<gks_mesh*>& ms, int mode);
void glaunch_mask_cols(hipStream_t st, const std::vector<gks_mesh*>& ms);
void glaunch_cycle_start(hipStream_t st, const std::vector<gks_mesh*>& ms);
void glaunch_arnoldi(hipStream_t st, const std::vector<gks_mesh*>& ms, int k);
void glaunch_end_cycle(hipStream_t st, const std::vector<gks_mesh*>& ms, const std::vector<int>& nvec);
void glaunch_flux_update(hipStream_t st, const std::vector<gks_mesh*>& ms, const std::vector<const double*>& W);
void glaunch_commit(hipStream_t st, const std::vector<gks_mesh*>& ms, const std::vector<double*>& W);
void launch_limit_noalloc(gks_mesh* m, void* scr, int phase, const double* W, const double* X, double* Xout,
                          double threshold, int variables);
int32_t* scratch_count(void* scr);
void launch_cfl(gks_mesh* m, const double* W, double* dt_out);
void launch_set_scalar(gks_mesh* m, double* p, double v);
void launch_zero(gks_mesh* m, double* p, int64_t count);
void launch_zero_i32(gks_mesh* m, int32_t* p, int count);
void launch_copy(gks_mesh* m, double* dst, const double* src, int64_t count);

void prof_begin(gks_mesh* m, int kc, double bytes = 0.0, double flops = 0.0);
void prof_end(gks_mesh* m, int kc);

}  // namespace gks
