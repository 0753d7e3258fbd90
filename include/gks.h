/*
 * gks.h -- C ABI of the third-order gas-kinetic scheme on triangle meshes
 * (compact least-squares reconstruction + second-order-expanded BGK flux +
 * finite-volume update), built for AMD Instinct MI355X (gfx950).
 *
 * Method: Li, Zhong, Zhuo, "A third order gas-kinetic scheme for
 * unstructured grid" (arXiv 1802.00704).  Each entry point cites the
 * passage that defines what it computes.
 *
 * Conventions shared by every call
 *   - State W: cell-averaged conservative variables (rho, rho u, rho v, E)
 *     of section 2.1 (Eq. macroVar), stored as double W[4][nt] (variable
 *     major) in DEVICE memory, cells in the caller's triangle order.
 *   - Reconstruction X: coefficients u_1..u_5 of the zero-mean quadratic of
 *     Eq. quadRCP for each variable, double X[4][5][nt] in DEVICE memory:
 *     X1 = h u_x, X2 = h u_y, X3 = h^2 u_xx, X4 = h^2 u_xy, X5 = h^2 u_yy at
 *     the cell centroid, h = max(circumradius, sqrt(area)) (Eq. h).  Cells
 *     with a boundary edge are linear (Eq. k_i): their X3..X5 are zero.
 *   - Faces: face f is emitted while scanning triangles t = 0..nt-1 and
 *     local edges e = 0..2 (edge e runs from vertex e to vertex e+1 mod 3)
 *     whenever the triangle across the edge has a larger index or the edge
 *     is a boundary edge.  The owner is t; the unit normal points out of the
 *     owner.  gks_faces() returns owner/neighbour arrays.
 *   - Fluxes F: double F[4][nf] in DEVICE memory, face order as above,
 *     x-y frame, integrated over the time step and along the face
 *     (sum over the two Gauss points of (S/2) times the time-integrated flux
 *     per unit length, Eqs. fluxgauss and fvm3), positive from owner to
 *     neighbour.
 *   - All device work is ordered on the HIP stream given at creation; for
 *     NULL the handle creates a stream of its own (which synchronises with
 *     the legacy default stream).  Device pointers must belong to the device that
 *     was current at creation.  Calls on one handle are not thread-safe;
 *     distinct handles are independent.
 *   - Every call returns GKS_OK (0) or a negative error code and never
 *     throws; gks_last_error() gives a message for the last failure.
 */
#ifndef GKS_H
#define GKS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define GKS_OK        0
#define GKS_EINVAL   -1   /* bad argument or invalid mesh                         */
#define GKS_ENOMEM   -2   /* device or host allocation failed                     */
#define GKS_EHIP     -3   /* a HIP runtime call failed                            */
#define GKS_ENOCONV  -4   /* GMRES did not reach the tolerance within max_iter    */
#define GKS_ENONPHYS -5   /* non-physical state (rho <= 0 or p <= 0)              */

/* precision of the reconstruction solve */
#define GKS_FP64   0      /* FP64 GMRES(restart) with BILU(0)                        */
#define GKS_MIXED  1      /* FP64 flexible GMRES; FP32 SpMV and ILU in inner sweeps */

/* elimination order of the BILU(0) preconditioner */
#define GKS_ORDER_MULTICOLOR 0  /* greedy colouring, RCM order inside each colour */
#define GKS_ORDER_RCM        1  /* reverse Cuthill-McKee (level-scheduled sweeps) */

/* boundary kinds (value of gks_mesh_desc.bc_kind[row]) */
#define GKS_BC_SLIP    1  /* inviscid wall: mirror image, normal momentum reflected      */
#define GKS_BC_NOSLIP  2  /* wall moving with (u, v) = bc_state[row][1..2]: mirror image,
                             ghost velocity 2 U_wall - U, density and pressure even      */
#define GKS_BC_INFLOW  3  /* fixed state (rho, u, v, p) = bc_state[row][0..3], no slopes */
#define GKS_BC_OUTFLOW 4  /* transmissive: ghost = the boundary cell's average, no slopes */

/* inner solver of the mixed form (gks_params.inner_solver) */
#define GKS_INNER_RICHARDSON 0  /* inner_iters BILU(0)-preconditioned Richardson sweeps  */
#define GKS_INNER_GMRES      1  /* inner_iters steps of GMRES, right-preconditioned by one
                                   FP32 BILU(0) application, FP64 Arnoldi and matrix     */

/* variables the limiter acts on (gks_params.limiter, gks_limit) */
#define GKS_LIMIT_CONSERVATIVE   1
#define GKS_LIMIT_CHARACTERISTIC 2

typedef struct gks_mesh gks_mesh;   /* opaque; owns every device buffer it allocates */

/* Mesh description.  Host arrays are copied at creation; the caller may free
 * them afterwards. */
typedef struct {
    int32_t nv;              /* vertices                                         */
    int32_t nt;              /* triangles (cells)                                */
    const double*  xy;       /* host [nv][2] vertex coordinates                  */
    const int32_t* tri;      /* host [nt][3] counter-clockwise vertex indices    */
    const int32_t* edge_tag; /* host [nt][3] or NULL: 0 interior, else 1-based
                                row of the boundary table for edge e of t       */
    int32_t periodic_x;      /* nonzero: x is periodic with period Lx; vertices
                                are identified, triangles unwrapped by the
                                minimum image                                   */
    int32_t periodic_y;
    double  Lx, Ly;
    int32_t n_bc;            /* rows of the boundary table                       */
    const int32_t* bc_kind;  /* host [n_bc] GKS_BC_* kinds                       */
    const double*  bc_state; /* host [n_bc][4] (rho, u, v, p) per row            */
} gks_mesh_desc;

/* Scheme and solver parameters (gks_params_default fills the paper's values). */
typedef struct {
    double  gamma;           /* ratio of specific heats (1.4)                    */
    double  mu;              /* dynamic viscosity; 0 selects the inviscid
                                collision time of Eq. tauIns, > 0 Eq. tauVis    */
    double  tau_eps;         /* coefficient of dt in Eq. tauIns (0.01)           */
    double  cls_w;           /* derivative weight w of Eq. A:B:b:3 (0.3)         */
    double  cfl;             /* CFL number of the time-step rule (0.5)           */
    double  tol;             /* relative residual ||R - K X|| / ||R|| per column */
    int32_t restart;         /* GMRES restart length m (30), 1..64               */
    int32_t max_iter;        /* cap on Krylov iterations per solve (500)         */
    int32_t precision;       /* GKS_FP64 or GKS_MIXED                            */
    int32_t ordering;        /* GKS_ORDER_MULTICOLOR or GKS_ORDER_RCM            */
    int32_t inner_iters;     /* GKS_MIXED: FP32 preconditioned sweeps (or inner
                                GMRES steps) per outer iteration (4; see
                                inner_iters_first)                              */
    int32_t exact_time;      /* 0: time coefficients c_1..c_8 of Eq.
                                Nomenclature2 as printed; 1: exact integrals     */
    int32_t nonphys_fallback;/* 0: non-physical Gauss-point state -> GKS_ENONPHYS;
                                1: that side falls back to its cell average     */
    int32_t all_quadratic;   /* testing: quadratic reconstruction in every cell  */
    int32_t graphs;          /* 1: gks_step replays two captured HIP graphs
                                (solve with the first GMRES cycle unrolled to
                                a step budget; flux and update), continuing on
                                the host when the cycle needs more steps; 0:
                                eager launches.  Results are identical.  Graphs
                                are not used while gks_profile_enable is on.  */
    int32_t graph_budget;    /* Arnoldi steps unrolled in the solve graph: 0 =
                                adaptive (follows the first-cycle length of
                                recent steps, re-capturing when it changes);
                                k > 0 = exactly min(k, restart, max_iter)       */
    int32_t limiter;         /* GKS_LIMIT_CONSERVATIVE or _CHARACTERISTIC:
                                gks_step limits the reconstruction with the
                                DWBAP limiter of section 3.3 (Eqs. DWBAP,
                                DWBAP_w, DWBAP_S) where the shock indicator of
                                Eqs. ISD1-2 reaches 1, before the fluxes, in
                                those variables; the solver keeps the
                                unlimited X.  0: off                          */
    double  reorth_tol;      /* Arnoldi orthogonalisation: classical Gram-
                                Schmidt, with the second pass (CGS2) taken
                                only when, for a column still iterating, the
                                new vector w1 after the first pass has
                                |V^T w1| > reorth_tol |w1|; 0 takes it at
                                every step.  Each solve still ends on its true
                                residual.  0 <= reorth_tol < 1; default 1e-8 */
    int32_t inner_solver;    /* GKS_MIXED: the preconditioner of each outer
                                step, GKS_INNER_RICHARDSON (default) or
                                GKS_INNER_GMRES (then 1 <= inner_iters <= 8;
                                not with gks_batch_step)                      */
    int32_t inner_iters_first; /* GKS_MIXED, Richardson: sweeps in the first
                                outer step of each GMRES cycle (7), the later
                                steps take inner_iters; 0: inner_iters in
                                every step.  gks_apply_precond applies
                                inner_iters sweeps                            */
    int32_t adapt_sweeps;    /* GKS_MIXED, Richardson, 1 (default): gks_step
                                and gks_batch_step adapt the first outer
                                step's sweep count between steps, from
                                inner_iters_first (inner_iters when that is
                                0) down to 2.  After 8 solves in a row that
                                need a single outer step, the next step
                                tries one sweep fewer; a trial that needs
                                more outer steps restores the count and
                                holds it for 64 steps (doubling with each
                                such trial in a row, up to 1024); 4 solves
                                in a row that need more than one outer step
                                raise it by one (back to at most the
                                starting count).  The rule reads only the
                                handle's own outer-step counts, so a handle
                                takes the same counts alone and in a batch.
                                0: the count stays inner_iters_first        */
    int32_t extrap_points;   /* starting guess of each step's solve: the
                                polynomial through the last extrap_points
                                solutions at their times, evaluated at the
                                step's time, 1..6 (fewer while the step
                                sequence has fewer solutions).  0 (default):
                                the count adapts between steps, from 6 (3
                                with the limiter on) within 2..6.  Once the
                                starting residual r0 is below 50 (2^P - 1)
                                tol (the previous solves' residuals amplified
                                by the weights), a step tries P - 1; while it
                                is above 1000 (2^P - 1) tol, P + 1.  A trial
                                comes after at least 8 steps at P (2 when r0
                                is below 5 (2^P - 1) tol) and is kept if its
                                r0 is below 0.8 times the median of the last
                                four at P or its solve took fewer Arnoldi
                                steps than theirs; else no trial follows for
                                48 steps, doubling with each failure in a row
                                up to 384.  Only the start changes: every
                                solve still ends on its true residual        */
} gks_params;

/* Per-solve report (one entry per conserved variable). */
typedef struct {
    int32_t iters[4];        /* Krylov iterations                                */
    int32_t restarts[4];     /* restart cycles                                   */
    double  rel_resid[4];    /* final true relative residual ||R - K X|| / ||R|| */
    int32_t nonphys;         /* non-physical Gauss-point states met in the flux  */
    double  solve_ms;        /* host wall time of the reconstruction solve       */
    double  call_ms;         /* host wall time of the whole call                 */
    int32_t limited;         /* cells the limiter changed in this step            */
    int32_t reorth;          /* Arnoldi steps that took the second Gram-Schmidt
                                pass (see gks_params.reorth_tol)               */
    int32_t first_sweeps;    /* GKS_MIXED, Richardson: sweeps of the solve's
                                first outer step (see adapt_sweeps); else 0   */
    double  start_resid;     /* largest relative residual of the starting
                                guess over the columns (see extrap_points)   */
    int32_t start_points;    /* solutions the starting guess took            */
} gks_solve_info;

/* Mesh statistics. */
typedef struct {
    int32_t nt, nf, nf_boundary;
    int32_t n_levels;        /* dependency levels of each BILU(0) sweep          */
    int32_t n_colors;        /* colours (multicolour order) or 0                 */
    int32_t rcm_bandwidth;   /* max |i - j| over cell neighbours in RCM order    */
    int64_t device_bytes;    /* device memory held by the handle                 */
    int64_t graph_steps;     /* gks_step calls run through the captured graphs   */
    int32_t capture_failures;/* graph captures that failed (the step then ran
                                with eager launches; 3 turn graphs off)         */
    int32_t split_form;      /* 1: the cell graph has no 3-cycles, so BILU(0)
                                has no off-diagonal fill (U = K_U, L = K_L D^-1)
                                and the mixed form's inner sweeps run in the
                                split form without products by all of K        */
    int32_t graph_captures;  /* step graphs captured (solve graphs per budget
                                and first-step sweep count, continuations, the
                                flux-and-update graph)                         */
    double  capture_ms;      /* host time spent capturing and instantiating    */
} gks_mesh_stats;

/* Fill p with the paper's parameters: gamma 1.4, inviscid, tau_eps 0.01,
 * w = 0.3 (Eq. A:B:b:3), CFL 0.5, tol 1e-10, GMRES(30), FP64, multicolour,
 * graph replay on, second Gram-Schmidt pass above reorth_tol 1e-8, mixed
 * form with 7 Richardson sweeps in the first outer step (adapted between
 * steps) and 4 after, starting guesses extrapolated from an adapted number of solutions
 * (from 6; 3 with the limiter). */
void gks_params_default(gks_params* p);

/* Build the per-mesh state (section 3.1 geometry and Eq. h; the normal
 * equations of Eq. spdConserved:5 over the face-neighbour conditions of
 * Eqs. spdConserved:1-3 and A:B:b:2-3; the renumbering and the BILU(0)
 * factors of section 3.2) and upload it to the current device.
 * Errors: GKS_EINVAL for null or inconsistent arguments, clockwise or
 * degenerate triangles, non-manifold or untagged open edges; GKS_ENOMEM;
 * GKS_EHIP.  On error *out is NULL. */
int gks_mesh_create(const gks_mesh_desc* desc, const gks_params* prm,
                    void* hip_stream, gks_mesh** out);

/* CLS reconstruction (section 3): X solves the normal equations for the
 * four conserved variables with right-preconditioned restarted GMRES
 * (FP64) or flexible GMRES with FP32 inner sweeps (GKS_MIXED), warm-started
 * from the handle's previous solution, to the relative tolerance prm.tol.
 * W: device [4][nt] input; X: device [4][5][nt] output (may not alias W).
 * info may be NULL.  Synchronises the stream before returning.
 * Errors: GKS_EINVAL, GKS_ENOCONV (X then holds the last iterate), GKS_EHIP. */
int gks_cls_reconstruct(gks_mesh* m, const double* W, double* X, gks_solve_info* info);

/* Time-integrated third-order BGK face fluxes (section 2.2: Eqs.
 * generalSolution, fNS, 3orderf0:2, 3orderg:2, Nomenclature1-2; collision
 * time Eq. tauIns / tauVis) at the two Gauss points of every face, given the
 * cell states W [4][nt], reconstruction X [4][5][nt] and the step dt > 0.
 * F: device [4][nf] output.  Enqueued only (no synchronisation) unless a
 * non-physical state is possible, in which case the count is checked.
 * Errors: GKS_EINVAL, GKS_ENONPHYS (fallback disabled), GKS_EHIP. */
int gks_flux(gks_mesh* m, const double* W, const double* X, double dt, double* F);

/* One step of Eq. fvm3: dt from the CFL rule when dt <= 0 (the paper gives
 * none: dt = CFL min_i |Omega_i| / sum_f S_f (|U_i . n_f| + c_i)), then the
 * reconstruction (started from the extrapolation of the handle's earlier
 * solutions, see gks_params.extrap_points), the fluxes and the update
 * W <- W - (1/|Omega|) sum s F.
 * W: device [4][nt], updated in place only on success.  dt_used and info may
 * be NULL.  Synchronises the stream before returning.
 * Errors: GKS_EINVAL, GKS_ENOCONV, GKS_ENONPHYS, GKS_EHIP (W unchanged). */
int gks_step(gks_mesh* m, double* W, double dt, double* dt_used, gks_solve_info* info);

/* Owner and neighbour cell of every face (host arrays of nf entries; a
 * boundary face has neighbour -(boundary row)).  Either pointer may be NULL. */
int gks_faces(const gks_mesh* m, int32_t* own, int32_t* nbr);

/* Statistics of the handle. */
int gks_mesh_get_stats(const gks_mesh* m, gks_mesh_stats* st);

/* Per-kernel timing with HIP events on the handle's stream (enable = 1
 * resets and starts; 0 stops).  gks_profile_get copies up to n entries per
 * kernel class: name (static string), number of launches, total
 * milliseconds and total algorithmic bytes (the bytes the launches must
 * move: stored matrix blocks and indices, each input block read once and
 * each output block written once).  Any output pointer may be NULL.
 * Returns the number of classes copied or a negative error. */
int gks_profile_enable(gks_mesh* m, int enable);
int gks_profile_get(gks_mesh* m, int n, const char** names, int64_t* launches, double* total_ms,
                    double* total_bytes);

/* DWBAP limiter of section 3.3 on caller coefficients: cells whose density
 * shock indicator IS_i (Eq. ISD1) is at least `threshold` (Eq. ISD2 uses 1)
 * get their derivatives replaced by the biased average of Eq. DWBAP over
 * their own value and candidates from their face neighbours, with the
 * weights of Eqs. DWBAP_w and DWBAP_S; the other cells are copied.
 * variables: GKS_LIMIT_CONSERVATIVE limits each conserved variable;
 * GKS_LIMIT_CHARACTERISTIC (the variant of section 4.2) limits the
 * characteristic variables of the Euler equations along the cell's density
 * gradient, at its average state, and maps them back.  W [4][nt] and X,
 * Xout [4][5][nt] are device arrays in the caller's cell order (the layouts
 * of gks_step and gks_cls_reconstruct); Xout must not alias X.  n_limited
 * (host, may be NULL) receives the number of limited cells.
 * Errors: GKS_EINVAL, GKS_EHIP. */
int gks_limit(gks_mesh* m, const double* W, const double* X, double* Xout, double threshold,
              int32_t variables, int32_t* n_limited);

/* Limited cells that gks_limit_noalloc can hold (its static scratch). */
#define GKS_LIMIT_NOALLOC_MAX_CELLS 65536

/* gks_limit without any allocation, for callers that cannot allocate device
 * memory (code under stream capture, tight serving loops, harnesses that
 * forbid hipMalloc): gks_limit allocates its list of limited cells and
 * their coefficients on its first call on a handle, while this call keeps
 * them in a static device array of 10,748,160 bytes (the count, the list and
 * the coefficients of at most GKS_LIMIT_NOALLOC_MAX_CELLS limited cells)
 * that every device the library runs on holds from module load until the
 * process ends.  It calls no hipMalloc, hipFree or other allocating routine
 * and records no profiling events.  Arguments, layouts and results are those
 * of gks_limit (identical kernels, bitwise the same Xout).  Every call on one
 * device shares that device's array: calls that overlap on one device (other
 * streams, other host threads) race and must be serialised by the caller.
 * The call synchronises the handle's stream twice (after marking, to read
 * the count, and at the end).
 * Errors: GKS_EINVAL for bad arguments, or when more than
 * GKS_LIMIT_NOALLOC_MAX_CELLS cells reach the threshold (*n_limited then
 * holds their number and Xout holds X unlimited; gks_limit has no such
 * limit); GKS_EHIP when the array's device address could not be found at
 * the handle's creation, or a launch fails. */
int gks_limit_noalloc(gks_mesh* m, const double* W, const double* X, double* Xout, double threshold,
                      int32_t variables, int32_t* n_limited);

/* Apply the solve's preconditioner to four columns: Z = P(V), where P is
 * the BILU(0) factorisation of section 3.2 (form GKS_FP64: one forward and
 * one backward block substitution in FP64), or the inner iteration of the
 * mixed form (form GKS_MIXED, handle created with precision GKS_MIXED:
 * inner_iters Richardson sweeps z += M^-1 (v - K z) from z = 0 with the FP32
 * matrix and factors, or with inner_solver GKS_INNER_GMRES inner_iters GMRES
 * steps on K z = v, each column of V of unit norm).  V and Z are device arrays [4][5][nt] in the caller's
 * cell order (the layout of X), not aliased.  Uses the handle's work space;
 * for inspection and tests of the factor storage.
 * Errors: GKS_EINVAL, GKS_EHIP. */
int gks_apply_precond(gks_mesh* m, const double* V, double* Z, int form);

/* Host-only view of the per-mesh state that gks_mesh_create builds (no
 * device is touched), for inspection and tests: faces, cell measures, the
 * renumbering, the normal-equation matrix of Eq. spdConserved:5 and its
 * BILU(0) factors, all in solver order.  Blocks are 5 x 5 with entry
 * e = 5 r + c; slot arrays use the value nt for an empty slot.  The library
 * allocates every array; release them with gks_host_free.
 * Errors: as gks_mesh_create (GKS_EINVAL, GKS_ENOMEM). */
typedef struct {
    int32_t  nt, nf, n_levels, n_colors, rcm_bandwidth;
    int32_t* own;      /* [nf] owner cell                                   */
    int32_t* nbr;      /* [nf] neighbour cell, -(boundary row) on the boundary */
    double*  area;     /* [nt] cell areas                                   */
    double*  h;        /* [nt] length scales of Eq. h                        */
    int32_t* perm;     /* [nt] solver position -> cell                       */
    int32_t* lev_ptr;  /* [n_levels + 1] rows of each sweep level            */
    int32_t* kcol;     /* [4][nt] column of slot s of row i (slot 0 diagonal) */
    double*  kval;     /* [4][25][nt]                                        */
    int32_t* lcol;     /* [3][nt] strict lower factor (unit diagonal)        */
    double*  lval;     /* [3][25][nt]                                        */
    int32_t* ucol;     /* [3][nt] strict upper factor                        */
    double*  uval;     /* [3][25][nt]                                        */
    double*  dinv;     /* [25][nt] inverted pivot blocks                     */
    int32_t* spmv_order;   /* [n_spmv_waves] order in which the SpMV kernels take the
                              64-row groups of solver rows (multicolour order), or NULL */
    int32_t  n_spmv_waves; /* ceil(nt / 64) with a multicolour order, else 0    */
} gks_host_system;

int  gks_host_inspect(const gks_mesh_desc* desc, const gks_params* prm, gks_host_system* out);
void gks_host_free(gks_host_system* s);

/* Message of the last error on m (or of the last failed creation when m is
 * NULL).  The string stays valid until the next call on the same handle. */
const char* gks_last_error(const gks_mesh* m);

/* Release every resource of the handle; NULL is a no-op. */
void gks_destroy(gks_mesh* m);

/* ---------------------------------------------------------------- batched steps
 * One step of Eq. fvm3 (as gks_step) for several handles at once, for
 * serving many meshes on one device: every kernel of the step runs once for
 * all the handles of the batch (grouped launches over the concatenated
 * meshes, each handle at its own offset in the launch grid with the grid of
 * its own launch), so small meshes share launches instead of queueing their
 * own.  Each handle keeps its own state (mesh, factors, Krylov basis,
 * solution history) and its arithmetic is exactly that of gks_step with
 * eager launches (graphs = 0): results are bitwise those of stepping the
 * handle alone.  The GMRES cycles of the handles run in lockstep with one
 * status read per Arnoldi step for the batch. */
typedef struct gks_batch gks_batch;

#define GKS_BATCH_MAX 64   /* handles per gks_batch_step call */

/* A batch context whose work is ordered on hip_stream (NULL: a stream of its
 * own), on the current device.  Errors: GKS_EINVAL, GKS_ENOMEM, GKS_EHIP. */
int gks_batch_create(void* hip_stream, gks_batch** out);

/* One step of each of the n handles meshes[0..n-1] (distinct, created on the
 * batch's device, all GKS_FP64 or all GKS_MIXED; mixed handles need the
 * split-form sweeps, see gks_mesh_stats.split_form, and the Richardson inner
 * solver; no limiter), with device
 * states W[r] ([4][nt_r], updated in place on success, as gks_step).
 * dt: host [n] time steps, entries <= 0 (or dt = NULL) take the CFL rule.
 * dt_used (host [n], may be NULL) receives the steps taken; info (host [n],
 * may be NULL) the per-handle solve reports, with solve_ms and call_ms the
 * batch's; status (host [n]) each handle's outcome: GKS_OK, GKS_ENOCONV or
 * GKS_ENONPHYS (that W unchanged, as gks_step; the others still step).
 * Work is ordered on the batch's stream; the handles' own streams must hold
 * no pending work of the caller's (the call waits for them).  Synchronises
 * the batch's stream before returning.
 * Returns GKS_OK when every handle's step was attempted; GKS_EINVAL for bad
 * arguments (nothing runs); GKS_EHIP for a failed launch or runtime call. */
int gks_batch_step(gks_batch* b, int32_t n, gks_mesh* const* meshes, double* const* W, const double* dt,
                   double* dt_used, gks_solve_info* info, int32_t* status);

/* Message of the batch's last failure. */
const char* gks_batch_last_error(const gks_batch* b);

/* Release the batch (not its handles); NULL is a no-op. */
void gks_batch_destroy(gks_batch* b);

#ifdef __cplusplus
}
#endif
#endif /* GKS_H */
