// HIP kernels of the reconstruction solve, the Gauss-point flux and the
// finite-volume update, for gfx950 (wave64).
//
// No floating-point atomics anywhere: every reduction writes per-block
// partial sums that a second kernel adds in a fixed order, so results are
// bitwise reproducible run to run.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdlib>
#include <mutex>

#include "gks_flux_device.h"
#include "gks_char_basis.h"
#include "gks_internal.h"

namespace gks {

const char* kc_names[NPROF] = {"rhs",       "spmv",       "spmv_resid", "ilu_fwd",  "ilu_bwd",
                               "dots",      "axpy_dots",  "reorth",     "finalize", "combine",
                               "axpy",      "copyout",    "flux",       "update",   "cfl",
                               "misc",      "spmv32",     "ilu_fwd32",  "ilu_bwd32", "extrap", "limit", "limit_apply", "", ""};

constexpr int TPB = 256;          // threads per block of the streaming kernels
constexpr int RED_CHUNK = FUSED_DOTS_MAX;   // vectors per block of the dot kernels

static inline int nblocks(int64_t n, int tpb = TPB) { return (int)((n + tpb - 1) / tpb); }
// grid of the Gram-Schmidt update (grid-stride beyond): about 8 blocks per
// CU, a multiple of 5 (k_axpy_dots needs a grid of a multiple of 10 threads)
// and of the 8 XCDs
constexpr int AXPY_BLOCKS = 2040;
// blocks of k_axpy_dots for n rows: a multiple of 5, at most AXPY_BLOCKS
static inline int axpy_dots_blocks(int n) { return (std::min(AXPY_BLOCKS, nblocks((int64_t)n * 10)) + 4) / 5 * 5; }

// The hardware hands consecutive workgroups of a grid to the 8 XCDs in turn,
// and each XCD has its own L2.  Row kernels gather neighbour blocks, so they
// renumber workgroups such that every XCD works on one contiguous range of
// rows and its neighbours stay in that XCD's L2.
constexpr int NXCD = 8;

// ------------------------------------------------------------------ launch grids
// Kernel bodies take their block index and grid size from a grid policy.
// Grid1 reads the hardware's (one mesh per launch).  GridV holds a block's
// virtual index and grid inside a grouped launch, which runs the same kernel
// for several meshes at once (Group below): each mesh's blocks see the grid
// its own launch would have, so they do exactly the same arithmetic, and
// block partials of reductions land where its own launch puts them.
struct Grid1 {
    __device__ __forceinline__ int b() const { return (int)blockIdx.x; }
    __device__ __forceinline__ int g() const { return (int)gridDim.x; }
};
struct GridV {
    int vb, vn;
    __device__ __forceinline__ int b() const { return vb; }
    __device__ __forceinline__ int g() const { return vn; }
};

// Arguments of a grouped launch, passed by value: per mesh r, its kernel
// arguments a[r], its first block start[r] (a multiple of NXCD, so that a
// block's XCD is the one its own launch would give it) and its grid nblk[r].
// Blocks between a mesh's grid and the next mesh's start do nothing.
template <class A>
struct Group {
    int n;
    int start[MAXB + 1];
    int nblk[MAXB];
    A a[MAXB];
};

// Mesh of this block in a grouped launch (or -1 for a padding block) and its
// virtual grid.  Uniform over the block: scalar loads of the kernel arguments.
template <class A>
__device__ __forceinline__ int group_locate(const Group<A>& g, GridV& vg) {
    const int b = (int)blockIdx.x;
    int r = 0;
    while (r + 1 < g.n && g.start[r + 1] <= b) ++r;
    vg.vb = b - g.start[r];
    vg.vn = g.nblk[r];
    return vg.vb < vg.vn ? r : -1;
}

template <class G = Grid1>
__device__ __forceinline__ int xcd_block(G grid = G()) {
    const int Gn = grid.g(), b = grid.b();
    const int q = Gn / NXCD, r = Gn % NXCD;
    const int x = b % NXCD, k = b / NXCD;
    return x * q + min(x, r) + k;
}
template <class G = Grid1>
__device__ __forceinline__ int xcd_row(G grid = G()) { return xcd_block(grid) * blockDim.x + threadIdx.x; }

// Row of a thread in the SpMV kernels.  With a wave order, the launch's
// waves take the 64-row groups in that order: in multicolour order it
// cycles through the colours chunk by chunk, so the rows that one XCD works
// on at a time cover one part of the mesh in every colour and the neighbour
// rows they gather (all in other colours) meet again in that XCD's L2.
// Waves past the table get rows past n (no work).
template <class G = Grid1>
__device__ __forceinline__ int spmv_row(const int32_t* __restrict__ worder, int n, G grid = G()) {
    const int r = xcd_row(grid);
    if (!worder) return r;
    const int nw = (n + 63) >> 6;
    const int g = r >> 6;   // wave-uniform
    const int w = g < nw ? __builtin_amdgcn_readfirstlane(worder[g]) : nw;
    return w * 64 + (r & 63);
}


// ------------------------------------------------------------------ block loads
// Matrix storage ("vector-packed"): for slot s of row i, entries e < 24 of the
// 5 x 5 block (e = 5 r + c) lie at  s*25*np + ((e / V) * np + i) * V + e % V
// and entry 24 at  s*25*np + 24*np + i,  with V = 16 bytes / sizeof(T) and the
// row stride np a multiple of 4.  A thread loads a block with 24 / V 16-byte
// loads plus one scalar, and a wave reads contiguous 1 KiB runs.
template <typename T> struct Vec16;
template <> struct Vec16<float> {
    using type = float4;
    static constexpr int N = 4;
    static __device__ __forceinline__ void put(float* o, const float4& v) { o[0] = v.x; o[1] = v.y; o[2] = v.z; o[3] = v.w; }
};
template <> struct Vec16<double> {
    using type = double2;
    static constexpr int N = 2;
    static __device__ __forceinline__ void put(double* o, const double2& v) { o[0] = v.x; o[1] = v.y; }
};

// Streams that a launch reads once (matrix blocks, factor blocks, Krylov
// basis vectors, rows of the input vector) are read with nontemporal loads,
// and the SpMV output with nontemporal stores: they bypass the L2 retention
// that the vectors read again by neighbouring rows (the SpMV's gathered x,
// the sweeps' solution) need.  The hints change no value: every result is
// bitwise the same with plain loads.  The builtins take clang vector types.
typedef float nvf4 __attribute__((ext_vector_type(4)));
typedef double nvd2 __attribute__((ext_vector_type(2)));
template <typename T> struct NV;
template <> struct NV<float> { using type = nvf4; static constexpr int N = 4; };
template <> struct NV<double> { using type = nvd2; static constexpr int N = 2; };

// load_block with nontemporal loads.
template <typename T>
__device__ __forceinline__ void load_block_nt(const T* __restrict__ val, int64_t np, int s, int i, T (&blk)[25]) {
    using VT = typename NV<T>::type;
    constexpr int V = NV<T>::N;
    const T* base = val + (int64_t)s * 25 * np;
    const VT* vb = reinterpret_cast<const VT*>(base);
#pragma unroll
    for (int g = 0; g < 24 / V; ++g) {
        const VT v = __builtin_nontemporal_load(vb + (int64_t)g * np + i);
#pragma unroll
        for (int e = 0; e < V; ++e) blk[g * V + e] = v[e];
    }
    blk[24] = __builtin_nontemporal_load(base + 24 * np + i);
}

template <typename T>
__device__ __forceinline__ void load_block(const T* __restrict__ val, int64_t np, int s, int i, T (&blk)[25]) {
    using VT = typename Vec16<T>::type;
    constexpr int V = Vec16<T>::N;
    const T* base = val + (int64_t)s * 25 * np;
    const VT* vb = reinterpret_cast<const VT*>(base);
#pragma unroll
    for (int g = 0; g < 24 / V; ++g) Vec16<T>::put(blk + g * V, vb[(int64_t)g * np + i]);
    blk[24] = base[24 * np + i];
}

// Per-column sums of squares of the values a thread produced, reduced over
// the block in a fixed order (wave butterfly, then the block's waves) to
// partial[c * gridDim.x + blockIdx.x].  Every thread of the block must call
// it (no early return before it); blockDim.x == TPB.
template <class G = Grid1>
__device__ __forceinline__ void block_sumsq4(const double (&s)[NC], double* __restrict__ partial, G grid = G()) {
    __shared__ double sh[NC][TPB / 64];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
    for (int c = 0; c < NC; ++c) {
        double v = s[c];
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
        if (lane == 0) sh[c][wid] = v;
    }
    __syncthreads();
    if (threadIdx.x < NC) {
        double t = 0.0;
#pragma unroll
        for (int q = 0; q < TPB / 64; ++q) t += sh[threadIdx.x][q];
        partial[(int64_t)threadIdx.x * grid.g() + grid.b()] = t;
    }
}

// ------------------------------------------------------------------ RHS
// R_i = sum_j a0_ij (W_j - W_i) for the four variables (Eq. A:B:b, b = C^T b).
// One thread per cell in the caller's order (W reads stay local); the
// 160-byte block goes to the cell's solver row.
// With partial != NULL the block also writes the per-column sums of R^2.
template <class GRID>
__device__ __forceinline__ void rhs_body(GRID grid, int nt, const int32_t* __restrict__ iperm, const int32_t* __restrict__ nbc, const double* __restrict__ a0c, const double* __restrict__ W, double* __restrict__ R, double* __restrict__ partial) {
    const int oi = xcd_row(grid);
    double sq[NC] = {0.0, 0.0, 0.0, 0.0};
    if (oi < nt) {
        double wi[NC];
#pragma unroll
        for (int c = 0; c < NC; ++c) wi[c] = W[(int64_t)c * nt + oi];
        double acc[NC][NB];
#pragma unroll
        for (int c = 0; c < NC; ++c)
#pragma unroll
            for (int l = 0; l < NB; ++l) acc[c][l] = 0.0;
#pragma unroll
        for (int s = 0; s < 3; ++s) {
            const int j = nbc[(int64_t)s * nt + oi];
            double a[NB];
#pragma unroll
            for (int l = 0; l < NB; ++l) a[l] = a0c[((int64_t)s * NB + l) * nt + oi];
#pragma unroll
            for (int c = 0; c < NC; ++c) {
                const double d = W[(int64_t)c * nt + j] - wi[c];
#pragma unroll
                for (int l = 0; l < NB; ++l) acc[c][l] += a[l] * d;
            }
        }
        // the row is 160 contiguous bytes at a 16-byte boundary: ten 16-byte stores
        double2* out = reinterpret_cast<double2*>(R + (int64_t)iperm[oi] * CB);
        const double* flat = &acc[0][0];
#pragma unroll
        for (int q = 0; q < CB / 2; ++q) out[q] = make_double2(flat[2 * q], flat[2 * q + 1]);
#pragma unroll
        for (int c = 0; c < NC; ++c)
#pragma unroll
            for (int l = 0; l < NB; ++l) sq[c] += acc[c][l] * acc[c][l];
    }
    if (partial) block_sumsq4(sq, partial, grid);
}

__global__ void __launch_bounds__(TPB) k_rhs(int nt, const int32_t* __restrict__ iperm,
                                             const int32_t* __restrict__ nbc, const double* __restrict__ a0c,
                                             const double* __restrict__ W, double* __restrict__ R,
                                             double* __restrict__ partial) {
    rhs_body(Grid1(), nt, iperm, nbc, a0c, W, R, partial);
}

struct RhsArgs {
    int nt;
    const int32_t* iperm;
    const int32_t* nbc;
    const double* a0c;
    const double* W;
    double* R;
    double* partial;
};

__global__ void __launch_bounds__(TPB) kg_rhs(Group<RhsArgs> g) {
    GridV v;
    const int r = group_locate(g, v);
    if (r < 0) return;
    const RhsArgs& a = g.a[r];
    rhs_body(v, a.nt, a.iperm, a.nbc, a.a0c, a.W, a.R, a.partial);
}


// Row-major [.][CB] vectors of a wave's rows [i0, i0 + nr) pass through the
// wave's LDS area: lanes copy 16-byte chunks lane-contiguously to or from
// global memory, and each lane reads or writes its own row in LDS.  Every
// lane of the wave must take part (rows past nr are neither read nor
// written in global memory).  rows_load reads with nontemporal loads.
template <typename T>
__device__ __forceinline__ void rows_load(const T* __restrict__ a, int64_t i0, int nr, float4* st, int lane,
                                          T (&v)[CB]) {
    constexpr int K = CB * (int)sizeof(T) / 16;   // 16-byte chunks per row
    const nvf4* src = reinterpret_cast<const nvf4*>(a + i0 * CB);
    const int nc = nr * K;
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const int c = k * 64 + lane;
        if (c < nc) {
            const nvf4 v = __builtin_nontemporal_load(src + c);
            st[c] = make_float4(v[0], v[1], v[2], v[3]);
        }
    }
    __builtin_amdgcn_wave_barrier();
    const T* my = reinterpret_cast<const T*>(st + lane * K);
#pragma unroll
    for (int q = 0; q < CB; ++q) v[q] = my[q];
    __builtin_amdgcn_wave_barrier();
}

// rows_store with nontemporal global stores (the SpMV output).
template <typename T>
__device__ __forceinline__ void rows_store_nt(T* __restrict__ a, int64_t i0, int nr, float4* st, int lane,
                                              const T (&v)[CB]) {
    constexpr int K = CB * (int)sizeof(T) / 16;
    T* my = reinterpret_cast<T*>(st + lane * K);
#pragma unroll
    for (int q = 0; q < CB; ++q) my[q] = v[q];
    __builtin_amdgcn_wave_barrier();
    nvf4* dst = reinterpret_cast<nvf4*>(a + i0 * CB);
    const int nc = nr * K;
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const int c = k * 64 + lane;
        if (c < nc) {
            const float4 w = st[c];
            nvf4 nv;
            nv[0] = w.x; nv[1] = w.y; nv[2] = w.z; nv[3] = w.w;
            __builtin_nontemporal_store(nv, dst + c);
        }
    }
    __builtin_amdgcn_wave_barrier();
}

template <typename T>
__device__ __forceinline__ void rows_store(T* __restrict__ a, int64_t i0, int nr, float4* st, int lane,
                                           const T (&v)[CB]) {
    constexpr int K = CB * (int)sizeof(T) / 16;
    T* my = reinterpret_cast<T*>(st + lane * K);
#pragma unroll
    for (int q = 0; q < CB; ++q) my[q] = v[q];
    __builtin_amdgcn_wave_barrier();
    float4* dst = reinterpret_cast<float4*>(a + i0 * CB);
    const int nc = nr * K;
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const int c = k * 64 + lane;
        if (c < nc) dst[c] = st[c];
    }
    __builtin_amdgcn_wave_barrier();
}

// ------------------------------------------------------------------ SpMV
// y = K (s .* x)   or   y = b - K x   (RESID), block-ELL, thread per row.
// In RESID mode xscale (when not null) scales b instead: y = s .* b - K x.
// MT: matrix element type; XT: element type of the input vector x.
// In RESID mode with partial != NULL the block also writes the per-column
// sums of y^2 (no early return then: every thread reaches the reduction).
template <class GRID, typename T, typename XT, bool RESID>
__device__ __forceinline__ void spmv_body(GRID grid, int n, int np, const T* __restrict__ val, const int32_t* __restrict__ col, const int32_t* __restrict__ worder, const XT* __restrict__ x, const double* __restrict__ xscale, const double* __restrict__ b, double* __restrict__ y, const int32_t* __restrict__ gate, double* __restrict__ partial) {
    if (gate && *gate == 0) return;
    __shared__ float4 stage[TPB / 64][64 * 2 * CB / 4];   // a wave's 64 FP64 rows
    const int i = spmv_row(worder, n, grid);
    const int lane = threadIdx.x & 63;
    const int64_t i0 = (int64_t)i - lane;                  // first row of the wave
    const int nr = (int)max((int64_t)0, min((int64_t)64, (int64_t)n - i0));
    if (nr == 0 && !(RESID && partial)) return;            // the whole wave is past the rows
    const bool valid = lane < nr;
    float4* st = stage[threadIdx.x >> 6];
    double sq[NC] = {0.0, 0.0, 0.0, 0.0};
    double acc[CB];
#pragma unroll
    for (int q = 0; q < CB; ++q) acc[q] = 0.0;
    if (valid) {
#pragma unroll
        for (int s = 0; s < KW; ++s) {
            const int j = col[(int64_t)s * n + i];
            const XT* xj = x + (int64_t)j * CB;
            double xv[CB];
#pragma unroll
            for (int q = 0; q < CB; ++q) xv[q] = (double)xj[q];
            T blk[25];
            load_block_nt(val, np, s, i, blk);
#pragma unroll
            for (int c = 0; c < NC; ++c)
#pragma unroll
                for (int r = 0; r < NB; ++r)
#pragma unroll
                    for (int q = 0; q < NB; ++q) acc[c * NB + r] += (double)blk[r * NB + q] * xv[c * NB + q];
        }
    }
    double out[CB];
    if (RESID) {
        double bi[CB];
        rows_load(b, i0, nr, st, lane, bi);
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            const double sc = xscale ? xscale[c] : 1.0;
#pragma unroll
            for (int r = 0; r < NB; ++r) {
                const double v = sc * bi[c * NB + r] - acc[c * NB + r];
                out[c * NB + r] = v;
                if (valid) sq[c] += v * v;
            }
        }
    } else {
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            const double sc = xscale ? xscale[c] : 1.0;
#pragma unroll
            for (int r = 0; r < NB; ++r) out[c * NB + r] = sc * acc[c * NB + r];
        }
    }
    if (nr > 0) rows_store_nt(y, i0, nr, st, lane, out);
    if (RESID && partial) block_sumsq4(sq, partial, grid);
}

template <typename T, typename XT, bool RESID>
__global__ void __launch_bounds__(TPB) k_spmv(int n, int np, const T* __restrict__ val, const int32_t* __restrict__ col,
                                              const int32_t* __restrict__ worder,
                                              const XT* __restrict__ x, const double* __restrict__ xscale,
                                              const double* __restrict__ b, double* __restrict__ y,
    const int32_t* __restrict__ gate, double* __restrict__ partial = nullptr) {
    spmv_body<Grid1, T, XT, RESID>(Grid1(), n, np, val, col, worder, x, xscale, b, y, gate, partial);
}

template <typename T, typename XT>
struct SpmvArgs {
    int n;
    int np;
    const T* val;
    const int32_t* col;
    const int32_t* worder;
    const XT* x;
    const double* xscale;
    const double* b;
    double* y;
    const int32_t* gate;
    double* partial;
};

template <typename T, typename XT, bool RESID>
__global__ void __launch_bounds__(TPB) kg_spmv(Group<SpmvArgs<T, XT>> g) {
    GridV v;
    const int r = group_locate(g, v);
    if (r < 0) return;
    const SpmvArgs<T, XT>& a = g.a[r];
    spmv_body<GridV, T, XT, RESID>(v, a.n, a.np, a.val, a.col, a.worder, a.x, a.xscale, a.b, a.y, a.gate, a.partial);
}


// Per-column dot products d[j][c] (j < nj <= RED_CHUNK) of a thread, reduced
// over the block in a fixed order to partial[(j * NC + c) * gridDim.x +
// blockIdx.x].  Every thread of the block must call it.
template <class G = Grid1>
__device__ __forceinline__ void block_dots(const double (&d)[RED_CHUNK][NC], int nj, double* __restrict__ partial,
                                           G grid = G()) {
    __shared__ double sh[RED_CHUNK * NC][TPB / 64];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
    for (int j = 0; j < RED_CHUNK; ++j)
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            double v = d[j][c];
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
            if (lane == 0) sh[j * NC + c][wid] = v;
        }
    __syncthreads();
    if (threadIdx.x < nj * NC) {
        double t = 0.0;
#pragma unroll
        for (int q = 0; q < TPB / 64; ++q) t += sh[threadIdx.x][q];
        const int j = threadIdx.x / NC, c = threadIdx.x % NC;
        partial[((int64_t)j * NC + c) * grid.g() + grid.b()] = t;
    }
}

// y = K x (FP64 K) and, in the same pass, the first Gram-Schmidt products
// V_j . y for j < nvd <= RED_CHUNK (block partials to dpart).  y leaves
// through the wave's LDS area, and the products run over the wave's
// contiguous rows in 16-byte pairs, so every V_j read is lane-contiguous.
template <class GRID, typename XT>
__device__ __forceinline__ void spmv_dots_body(GRID grid, int n, int np, const double* __restrict__ val, const int32_t* __restrict__ col, const int32_t* __restrict__ worder, const XT* __restrict__ x, double* __restrict__ y, const double* __restrict__ V, int64_t vstride, int nvd, double* __restrict__ dpart, const int32_t* __restrict__ gate) {
    if (gate && *gate == 0) return;
    __shared__ float4 stage[TPB / 64][64 * 2 * CB / 4];   // a wave's 64 FP64 rows
    const int i = spmv_row(worder, n, grid);
    const int lane = threadIdx.x & 63;
    const int64_t i0 = (int64_t)i - lane;
    const int nr = (int)max((int64_t)0, min((int64_t)64, (int64_t)n - i0));
    float4* st = stage[threadIdx.x >> 6];
    double d[RED_CHUNK][NC];
#pragma unroll
    for (int j = 0; j < RED_CHUNK; ++j)
#pragma unroll
        for (int c = 0; c < NC; ++c) d[j][c] = 0.0;
    double acc[CB];
#pragma unroll
    for (int q = 0; q < CB; ++q) acc[q] = 0.0;
    if (lane < nr) {
#pragma unroll
        for (int s = 0; s < KW; ++s) {
            const int j = col[(int64_t)s * n + i];
            const XT* xj = x + (int64_t)j * CB;
            double xv[CB];
#pragma unroll
            for (int q = 0; q < CB; ++q) xv[q] = (double)xj[q];
            double blk[25];
            load_block_nt(val, np, s, i, blk);
#pragma unroll
            for (int c = 0; c < NC; ++c)
#pragma unroll
                for (int r = 0; r < NB; ++r)
#pragma unroll
                    for (int q = 0; q < NB; ++q) acc[c * NB + r] += blk[r * NB + q] * xv[c * NB + q];
        }
    }
    if (nr > 0) {
        rows_store(y, i0, nr, st, lane, acc);   // the staged y stays in LDS
        const double2* ys = reinterpret_cast<const double2*>(st);
        const int npair = nr * (CB / 2);
#pragma unroll
        for (int k = 0; k < CB / 2; ++k) {
            const int c = k * 64 + lane;   // pair c: elements 2c, 2c + 1 of the wave's rows
            if (c >= npair) continue;
            const int e = (2 * c) % CB;
            const int c0 = e / NB, c1 = (e + 1) / NB;
            const double2 yv = ys[c];
#pragma unroll
            for (int j = 0; j < RED_CHUNK; ++j) {
                if (j < nvd) {
                    const nvd2 vn = __builtin_nontemporal_load(reinterpret_cast<const nvd2*>(V + (int64_t)j * vstride + i0 * CB) + c);
                    const double2 vv = make_double2(vn[0], vn[1]);
#pragma unroll
                    for (int cc = 0; cc < NC; ++cc)
                        d[j][cc] += (cc == c0 ? vv.x * yv.x : 0.0) + (cc == c1 ? vv.y * yv.y : 0.0);
                }
            }
        }
    }
    block_dots(d, nvd, dpart, grid);
}

template <typename XT>
__global__ void __launch_bounds__(TPB) k_spmv_dots(int n, int np, const double* __restrict__ val,
                                                   const int32_t* __restrict__ col, const int32_t* __restrict__ worder,
                                                   const XT* __restrict__ x,
                                                   double* __restrict__ y, const double* __restrict__ V,
                                                   int64_t vstride, int nvd, double* __restrict__ dpart,
                                                   const int32_t* __restrict__ gate) {
    spmv_dots_body<Grid1, XT>(Grid1(), n, np, val, col, worder, x, y, V, vstride, nvd, dpart, gate);
}

template <typename XT>
struct SpmvDotsArgs {
    int n;
    int np;
    const double* val;
    const int32_t* col;
    const int32_t* worder;
    const XT* x;
    double* y;
    const double* V;
    int64_t vstride;
    int nvd;
    double* dpart;
    const int32_t* gate;
};

template <typename XT>
__global__ void __launch_bounds__(TPB) kg_spmv_dots(Group<SpmvDotsArgs<XT>> g) {
    GridV v;
    const int r = group_locate(g, v);
    if (r < 0) return;
    const SpmvDotsArgs<XT>& a = g.a[r];
    spmv_dots_body<GridV, XT>(v, a.n, a.np, a.val, a.col, a.worder, a.x, a.y, a.V, a.vstride, a.nvd, a.dpart, a.gate);
}


// out = w - sum_j h_j[c] scale_j[c] V_j and, in the same pass, the second
// Gram-Schmidt products V_j . out for j < nvec <= RED_CHUNK (block partials
// to dpart).  Grid-stride over 16-byte groups (pair p of a 20-double row);
// the launch makes the grid a multiple of 10 threads, so each thread keeps
// one pair position, hence fixed columns c0, c1 and fixed coefficients.
// out may alias w.  With sqpart != NULL the block also writes the
// per-column sums of out^2 (the norms that decide the second pass).
template <class GRID>
__device__ __forceinline__ void axpy_dots_body(GRID grid, int n, const double* __restrict__ V, int64_t vstride, int nvec, const double* __restrict__ h, const double* __restrict__ scale, const double* w, double* out, double* __restrict__ dpart, const int32_t* __restrict__ gate, double* __restrict__ sqpart) {
    if (gate && *gate == 0) return;
    double sq[NC] = {0.0, 0.0, 0.0, 0.0};
    const int64_t npair = (int64_t)n * 10;
    const int64_t t0 = (int64_t)grid.b() * blockDim.x + threadIdx.x;
    const int p = (int)(t0 % 10);
    const int c0 = (2 * p) / NB, c1 = (2 * p + 1) / NB;
    double hs0[RED_CHUNK], hs1[RED_CHUNK], d0[RED_CHUNK], d1[RED_CHUNK];
#pragma unroll
    for (int j = 0; j < RED_CHUNK; ++j) {
        hs0[j] = j < nvec ? h[j * NC + c0] * scale[j * NC + c0] : 0.0;
        hs1[j] = j < nvec ? h[j * NC + c1] * scale[j * NC + c1] : 0.0;
        d0[j] = 0.0;
        d1[j] = 0.0;
    }
    for (int64_t t = t0; t < npair; t += (int64_t)grid.g() * blockDim.x) {
        const int64_t off = (t / 10) * CB + 2 * p;
        const double2 w2 = *reinterpret_cast<const double2*>(w + off);
        double a0 = w2.x, a1 = w2.y;
        double2 vv[RED_CHUNK];
#pragma unroll
        for (int j = 0; j < RED_CHUNK; ++j) {
            if (j < nvec) {
                {
                    const nvd2 vn = __builtin_nontemporal_load(reinterpret_cast<const nvd2*>(V + (int64_t)j * vstride + off));
                    vv[j] = make_double2(vn[0], vn[1]);
                }
                a0 -= hs0[j] * vv[j].x;
                a1 -= hs1[j] * vv[j].y;
            }
        }
        *reinterpret_cast<double2*>(out + off) = make_double2(a0, a1);
#pragma unroll
        for (int j = 0; j < RED_CHUNK; ++j) {
            if (j < nvec) {
                d0[j] += vv[j].x * a0;
                d1[j] += vv[j].y * a1;
            }
        }
        if (sqpart) {
#pragma unroll
            for (int c = 0; c < NC; ++c) sq[c] += (c == c0 ? a0 * a0 : 0.0) + (c == c1 ? a1 * a1 : 0.0);
        }
    }
    double d[RED_CHUNK][NC];
#pragma unroll
    for (int j = 0; j < RED_CHUNK; ++j)
#pragma unroll
        for (int c = 0; c < NC; ++c) d[j][c] = (c == c0 ? d0[j] : 0.0) + (c == c1 ? d1[j] : 0.0);
    block_dots(d, nvec, dpart, grid);
    if (sqpart) block_sumsq4(sq, sqpart, grid);
}

__global__ void __launch_bounds__(TPB) k_axpy_dots(int n, const double* __restrict__ V, int64_t vstride, int nvec,
                                                   const double* __restrict__ h, const double* __restrict__ scale,
                                                   const double* w, double* out, double* __restrict__ dpart,
                                                   const int32_t* __restrict__ gate, double* __restrict__ sqpart) {
    axpy_dots_body(Grid1(), n, V, vstride, nvec, h, scale, w, out, dpart, gate, sqpart);
}

struct AxpyDotsArgs {
    int n;
    const double* V;
    int64_t vstride;
    int nvec;
    const double* h;
    const double* scale;
    const double* w;
    double* out;
    double* dpart;
    const int32_t* gate;
    double* sqpart;
};

__global__ void __launch_bounds__(TPB) kg_axpy_dots(Group<AxpyDotsArgs> g) {
    GridV v;
    const int r = group_locate(g, v);
    if (r < 0) return;
    const AxpyDotsArgs& a = g.a[r];
    axpy_dots_body(v, a.n, a.V, a.vstride, a.nvec, a.h, a.scale, a.w, a.out, a.dpart, a.gate, a.sqpart);
}


// ------------------------------------------------------------------ BILU(0) sweeps
// Factor storage ("sliced"): the rows of one dependency level are cut into
// slices of 64 consecutive rows, one wavefront each.  Slice k holds w[k]
// slots; slot s of the slice is a chunk of 64 blocks in the vector-packed
// layout with row stride 64, plus 64 column indices.  The host sorts the
// rows of a level by their number of lower (upper) neighbours, so a slice's
// width is nearly every row's exact count and padding is rare; padded slots
// point at the zero dummy row with zero blocks.  A wave reads its slice's
// width and first chunk once (scalar), so the slot loop is uniform.
struct SliceRef {
    int64_t ch0;   // first chunk of the slice
    int w;         // slots in the slice
    int lane;      // row within the slice
};

__device__ __forceinline__ SliceRef slice_ref(const SlicedIdx& S, int sbase, int rl) {
    const int sl = sbase + (rl >> 6);
    SliceRef r;
    r.ch0 = __builtin_amdgcn_readfirstlane(S.off[sl]);
    r.w = __builtin_amdgcn_readfirstlane(S.w[sl]);
    r.lane = rl & 63;
    return r;
}

// acc_c -= B x_c for the four columns, B a 5 x 5 block
template <typename T, typename XT, typename ACC>
__device__ __forceinline__ void block_sub(ACC (&acc)[CB], const T (&blk)[25], const XT (&x)[CB]) {
#pragma unroll
    for (int c = 0; c < NC; ++c)
#pragma unroll
        for (int r = 0; r < NB; ++r)
#pragma unroll
            for (int q = 0; q < NB; ++q) acc[c * NB + r] -= (ACC)blk[r * NB + q] * (ACC)x[c * NB + q];
}

// acc -= sum over the slice's slots of F_is x_{col(s)}
template <typename T, typename XT, typename ACC>
__device__ __forceinline__ void slice_sub(ACC (&acc)[CB], const T* __restrict__ val, const int32_t* __restrict__ col,
                                          const SliceRef& sr, const XT* __restrict__ x) {
#pragma unroll
    for (int s = 0; s < LW; ++s) {
        if (s >= sr.w) break;
        const int64_t ch = sr.ch0 + s;
        const int j = col[ch * 64 + sr.lane];
        const XT* xj = x + (int64_t)j * CB;
        XT xv[CB];
#pragma unroll
        for (int q = 0; q < CB; ++q) xv[q] = xj[q];
        T blk[25];
        load_block_nt(val + ch * 25 * 64, 64, 0, sr.lane, blk);
        block_sub(acc, blk, xv);
    }
}

// As slice_sub, with x_j read from xlo for columns j < split, else from x.
template <typename T, typename XT, typename ACC>
__device__ __forceinline__ void slice_sub_split(ACC (&acc)[CB], const T* __restrict__ val,
                                                const int32_t* __restrict__ col, const SliceRef& sr,
                                                const XT* __restrict__ xlo, const XT* __restrict__ x, int split) {
#pragma unroll
    for (int s = 0; s < LW; ++s) {
        if (s >= sr.w) break;
        const int64_t ch = sr.ch0 + s;
        const int j = col[ch * 64 + sr.lane];
        const XT* xj = (j < split ? xlo : x) + (int64_t)j * CB;
        XT xv[CB];
#pragma unroll
        for (int q = 0; q < CB; ++q) xv[q] = xj[q];
        T blk[25];
        load_block_nt(val + ch * 25 * 64, 64, 0, sr.lane, blk);
        block_sub(acc, blk, xv);
    }
}

// As slice_sub, with x_j = xs .* xlo_j (per-column scale xs, none if null)
// for columns j < split, else x_j.
template <typename T, typename ACC>
__device__ __forceinline__ void slice_sub_lo(ACC (&acc)[CB], const T* __restrict__ val,
                                             const int32_t* __restrict__ col, const SliceRef& sr,
                                             const double* __restrict__ xlo, const double* __restrict__ xs,
                                             const double* __restrict__ x, int split) {
#pragma unroll
    for (int s = 0; s < LW; ++s) {
        if (s >= sr.w) break;
        const int64_t ch = sr.ch0 + s;
        const int j = col[ch * 64 + sr.lane];
        const bool lo = j < split;
        const double* xj = (lo ? xlo : x) + (int64_t)j * CB;
        double xv[CB];
#pragma unroll
        for (int q = 0; q < CB; ++q) xv[q] = xj[q];
        if (lo && xs) {
#pragma unroll
            for (int c = 0; c < NC; ++c)
#pragma unroll
                for (int r = 0; r < NB; ++r) xv[c * NB + r] *= xs[c];
        }
        T blk[25];
        load_block_nt(val + ch * 25 * 64, 64, 0, sr.lane, blk);
        block_sub(acc, blk, xv);
    }
}

// forward  y_i = s .* v_i - sum_{k<i} L_ik y_k            (unit lower factor)
// backward z_i = Dinv_i (y_i - sum_{j>i} U_ij z_j)
// over the rows [r0, r1) of one dependency level.  Rows of level 0 (rows
// [0, zrows)) have no lower neighbours, so their y is s .* v: the forward
// pass skips them and reads s .* v where it gathers them, and their backward
// pass reads v with the scale.  Rows of the last level have no upper
// neighbours: its forward pass (LAST) writes z_i = Dinv_i y_i directly.
template <class GRID, bool LAST>
__device__ __forceinline__ void ilu_fwd_body(GRID grid, int np, int r0, int r1, int sbase, int zrows, SlicedIdx Li, const double* __restrict__ Lv, const double* __restrict__ Dinv, const double* __restrict__ v, const double* __restrict__ vscale, double* __restrict__ y, double* __restrict__ z, const int32_t* __restrict__ gate) {
    if (gate && *gate == 0) return;
    __shared__ float4 stage[TPB / 64][64 * 2 * CB / 4];   // a wave's 64 FP64 rows
    const int rl = xcd_row(grid);
    const int lane = threadIdx.x & 63;
    const int64_t i0 = (int64_t)r0 + rl - lane;            // first row of the wave
    if (i0 >= r1) return;                                   // the whole wave is past the level
    const int nr = (int)min((int64_t)64, (int64_t)r1 - i0);
    float4* st = stage[threadIdx.x >> 6];
    double acc[CB];
    rows_load(v, i0, nr, st, lane, acc);
#pragma unroll
    for (int c = 0; c < NC; ++c) {
        const double sc = vscale ? vscale[c] : 1.0;
#pragma unroll
        for (int r = 0; r < NB; ++r) acc[c * NB + r] *= sc;
    }
    if (lane < nr) slice_sub_lo(acc, Lv, Li.col, slice_ref(Li, sbase, rl), v, vscale, (const double*)y, zrows);
    if (LAST) {
        double zi[CB];
#pragma unroll
        for (int q = 0; q < CB; ++q) zi[q] = 0.0;
        if (lane < nr) {
            double d[25];
            load_block_nt(Dinv, np, 0, (int)i0 + lane, d);
#pragma unroll
            for (int c = 0; c < NC; ++c)
#pragma unroll
                for (int r = 0; r < NB; ++r) {
                    double t = 0.0;
#pragma unroll
                    for (int q = 0; q < NB; ++q) t += d[r * NB + q] * acc[c * NB + q];
                    zi[c * NB + r] = t;
                }
        }
        rows_store(z, i0, nr, st, lane, zi);
    } else {
        rows_store(y, i0, nr, st, lane, acc);
    }
}

template <bool LAST>
__global__ void __launch_bounds__(TPB) k_ilu_fwd(int np, int r0, int r1, int sbase, int zrows, SlicedIdx Li,
                                                 const double* __restrict__ Lv, const double* __restrict__ Dinv,
                                                 const double* __restrict__ v, const double* __restrict__ vscale,
                                                 double* __restrict__ y, double* __restrict__ z,
                                                 const int32_t* __restrict__ gate) {
    ilu_fwd_body<Grid1, LAST>(Grid1(), np, r0, r1, sbase, zrows, Li, Lv, Dinv, v, vscale, y, z, gate);
}

struct IluFwdArgs {
    int np;
    int r0;
    int r1;
    int sbase;
    int zrows;
    SlicedIdx Li;
    const double* Lv;
    const double* Dinv;
    const double* v;
    const double* vscale;
    double* y;
    double* z;
    const int32_t* gate;
};

template <bool LAST>
__global__ void __launch_bounds__(TPB) kg_ilu_fwd(Group<IluFwdArgs> g) {
    GridV v;
    const int r = group_locate(g, v);
    if (r < 0) return;
    const IluFwdArgs& a = g.a[r];
    ilu_fwd_body<GridV, LAST>(v, a.np, a.r0, a.r1, a.sbase, a.zrows, a.Li, a.Lv, a.Dinv, a.v, a.vscale, a.y, a.z, a.gate);
}


template <class GRID>
__device__ __forceinline__ void ilu_bwd_body(GRID grid, int np, int r0, int r1, int sbase, SlicedIdx Ui, const double* __restrict__ Uv, const double* __restrict__ Dinv, const double* __restrict__ y, const double* __restrict__ yscale, double* __restrict__ z, const int32_t* __restrict__ gate) {
    if (gate && *gate == 0) return;
    __shared__ float4 stage[TPB / 64][64 * 2 * CB / 4];
    const int rl = xcd_row(grid);
    const int lane = threadIdx.x & 63;
    const int64_t i0 = (int64_t)r0 + rl - lane;
    if (i0 >= r1) return;
    const int nr = (int)min((int64_t)64, (int64_t)r1 - i0);
    float4* st = stage[threadIdx.x >> 6];
    const int i = (int)i0 + lane;
    double acc[CB];
    rows_load(y, i0, nr, st, lane, acc);
    if (yscale) {
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            const double sc = yscale[c];
#pragma unroll
            for (int r = 0; r < NB; ++r) acc[c * NB + r] *= sc;
        }
    }
    double zi[CB];
#pragma unroll
    for (int q = 0; q < CB; ++q) zi[q] = 0.0;
    if (lane < nr) {
        slice_sub(acc, Uv, Ui.col, slice_ref(Ui, sbase, rl), z);
        double d[25];
        load_block_nt(Dinv, np, 0, i, d);
#pragma unroll
        for (int c = 0; c < NC; ++c)
#pragma unroll
            for (int r = 0; r < NB; ++r) {
                double t = 0.0;
#pragma unroll
                for (int q = 0; q < NB; ++q) t += d[r * NB + q] * acc[c * NB + q];
                zi[c * NB + r] = t;
            }
    }
    rows_store(z, i0, nr, st, lane, zi);
}

__global__ void __launch_bounds__(TPB) k_ilu_bwd(int np, int r0, int r1, int sbase, SlicedIdx Ui,
                                                 const double* __restrict__ Uv, const double* __restrict__ Dinv,
                                                 const double* __restrict__ y, const double* __restrict__ yscale,
                                                 double* __restrict__ z, const int32_t* __restrict__ gate) {
    ilu_bwd_body(Grid1(), np, r0, r1, sbase, Ui, Uv, Dinv, y, yscale, z, gate);
}

struct IluBwdArgs {
    int np;
    int r0;
    int r1;
    int sbase;
    SlicedIdx Ui;
    const double* Uv;
    const double* Dinv;
    const double* y;
    const double* yscale;
    double* z;
    const int32_t* gate;
};

__global__ void __launch_bounds__(TPB) kg_ilu_bwd(Group<IluBwdArgs> g) {
    GridV v;
    const int r = group_locate(g, v);
    if (r < 0) return;
    const IluBwdArgs& a = g.a[r];
    ilu_bwd_body(v, a.np, a.r0, a.r1, a.sbase, a.Ui, a.Uv, a.Dinv, a.y, a.yscale, a.z, a.gate);
}


// ------------------------------------------------------------------ mixed-precision inner sweeps
// One BILU(0)-preconditioned Richardson sweep z <- z + M^-1 (b - K z) with
// the FP32 matrix and factors and FP32 vectors (20 floats per cell), where
// b = FP32(s .* v) is formed once, by the first sweep:
//   forward  (rows of one level)  y_i = r_i - sum_{k<i} L_ik y_k,
//            r_i = b_i - sum_s K_is z_s      (FIRST: z = 0, r_i = b_i)
//   backward (rows of one level)  d_i = Dinv_i (y_i - sum_{j>i} U_ij d_j),
//            z_i += d_i                        (FIRST: z_i = d_i, d is z)
// z is not modified during the forward levels, so the residual needs no
// separate pass.  Sums are accumulated in ACC.
template <bool FIRST, typename ACC>
__global__ void __launch_bounds__(TPB) k_mx_fwd(int n, int np, int r0, int r1, int sbase, const float* __restrict__ Kv,
                                                const int32_t* __restrict__ Kc, SlicedIdx Li,
                                                const float* __restrict__ Lv, const double* __restrict__ v,
                                                const double* __restrict__ vscale, float* __restrict__ b,
                                                const float* __restrict__ z, float* __restrict__ y,
                                                const int32_t* __restrict__ gate) {
    if (gate && *gate == 0) return;
    const int rl = xcd_row();
    const int i = r0 + rl;
    if (i >= r1) return;
    ACC acc[CB];
    float* bi = b + (int64_t)i * CB;
    if (FIRST) {
        const double* vi = v + (int64_t)i * CB;
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            const double sc = vscale[c];
#pragma unroll
            for (int r = 0; r < NB; ++r) {
                const float t = (float)(sc * vi[c * NB + r]);
                bi[c * NB + r] = t;
                acc[c * NB + r] = (ACC)t;
            }
        }
    } else {
#pragma unroll
        for (int q = 0; q < CB; ++q) acc[q] = (ACC)bi[q];
#pragma unroll
        for (int s = 0; s < KW; ++s) {
            const int j = Kc[(int64_t)s * n + i];
            const float* zj = z + (int64_t)j * CB;
            float zv[CB];
#pragma unroll
            for (int q = 0; q < CB; ++q) zv[q] = zj[q];
            float blk[25];
            load_block(Kv, np, s, i, blk);
            block_sub(acc, blk, zv);
        }
    }
    slice_sub(acc, Lv, Li.col, slice_ref(Li, sbase, rl), y);
    float* yi = y + (int64_t)i * CB;
#pragma unroll
    for (int q = 0; q < CB; ++q) yi[q] = (float)acc[q];
}

template <bool FIRST, typename ACC>
__global__ void __launch_bounds__(TPB) k_mx_bwd(int np, int r0, int r1, int sbase, SlicedIdx Ui,
                                                const float* __restrict__ Uv, const float* __restrict__ Dinv,
                                                const float* __restrict__ y, float* __restrict__ d,
                                                float* __restrict__ z, const int32_t* __restrict__ gate) {
    if (gate && *gate == 0) return;
    const int rl = xcd_row();
    const int i = r0 + rl;
    if (i >= r1) return;
    float* dd = FIRST ? z : d;
    ACC acc[CB];
    const float* yi = y + (int64_t)i * CB;
#pragma unroll
    for (int q = 0; q < CB; ++q) acc[q] = (ACC)yi[q];
    slice_sub(acc, Uv, Ui.col, slice_ref(Ui, sbase, rl), dd);
    float dg[25];
    load_block(Dinv, np, 0, i, dg);
    float di[CB];
#pragma unroll
    for (int c = 0; c < NC; ++c)
#pragma unroll
        for (int r = 0; r < NB; ++r) {
            ACC t = 0;
#pragma unroll
            for (int q = 0; q < NB; ++q) t += (ACC)dg[r * NB + q] * acc[c * NB + q];
            di[c * NB + r] = (float)t;
        }
    float* zi = z + (int64_t)i * CB;
    if (FIRST) {
#pragma unroll
        for (int q = 0; q < CB; ++q) zi[q] = di[q];
    } else {
        float* dout = d + (int64_t)i * CB;
#pragma unroll
        for (int q = 0; q < CB; ++q) {
            dout[q] = di[q];
            zi[q] = zi[q] + di[q];
        }
    }
}

// ------------------------------------------------------------------ split-form inner sweeps
// When the cell graph has no 3-cycles, BILU(0) has no off-diagonal fill, so
// M = (D + K_L) D^-1 (D + K_U) with D the pivot blocks and K_L, K_U the
// strict block triangles of K.  The Richardson sweep z <- z + M^-1 (b - K z)
// is then  (D + K_L) w = b + E z + K_L D^-1 K_U z,  (D + K_U) z' = D w,
// E = D - K_D, and the previous backward solve gives D^-1 K_U z = w_prev - z
// (Eisenstat's observation), so no product with all of K is needed.  The
// blocks are stored scaled from the left by the row's pivot inverse
// (L'_ik = Dinv_i K_ik, U'_ij = Dinv_i K_ij, G_i = Dinv_i E_i) and the first
// sweep keeps b'_i = Dinv_i b_i, so later sweeps never touch Dinv:
//   forward  w_i = b'_i + G_i z_i - sum_{k<i} L'_ik t_k,
//            t_i = w_i - w_prev_i + z_i           (first sweep: z = 0, t = w)
//   backward z'_i = w_i - sum_{j>i} U'_ij z'_j
// The last level has no upper neighbours (z'_i = w_i, set by the forward
// kernel).  Level 0 has no lower neighbours, so its pivots are untouched by
// the elimination: G = 0 there, w = b' in every sweep and t = z after the
// first.  Level 0 therefore has a forward pass only in the first sweep, which
// stores b' alone; later levels gather b' (first sweep) or z (later sweeps)
// for level-0 neighbours, and level 0's backward pass reads b' as its w.
template <typename ACC>
__device__ __forceinline__ void block_mul(float (&out)[CB], const float (&blk)[25], const ACC (&x)[CB]) {
#pragma unroll
    for (int c = 0; c < NC; ++c)
#pragma unroll
        for (int r = 0; r < NB; ++r) {
            ACC t = 0;
#pragma unroll
            for (int q = 0; q < NB; ++q) t += (ACC)blk[r * NB + q] * x[c * NB + q];
            out[c * NB + r] = (float)t;
        }
}

// acc += blk x (x FP32)
template <typename ACC>
__device__ __forceinline__ void block_add(ACC (&acc)[CB], const float (&blk)[25], const float (&x)[CB]) {
#pragma unroll
    for (int c = 0; c < NC; ++c)
#pragma unroll
        for (int r = 0; r < NB; ++r)
#pragma unroll
            for (int q = 0; q < NB; ++q) acc[c * NB + r] += (ACC)blk[r * NB + q] * (ACC)x[c * NB + q];
}

template <class GRID, bool FIRST, bool LAST, typename ACC>
__device__ __forceinline__ void es_fwd_body(GRID grid, int np, int r0, int r1, int sbase, int zrows, SlicedIdx Li, const float* __restrict__ KLv, const float* __restrict__ G, const float* __restrict__ Dinv, const double* __restrict__ v, const double* __restrict__ vscale, float* __restrict__ b, float* __restrict__ t, float* __restrict__ w, float* __restrict__ z, const int32_t* __restrict__ gate) {
    if (gate && *gate == 0) return;
    constexpr int SK = FIRST ? 2 * CB / 4 : CB / 4;   // 16-byte chunks per staged row (FP64 v first)
    __shared__ float4 stage[TPB / 64][64 * SK];
    const int rl = xcd_row(grid);
    const int lane = threadIdx.x & 63;
    const int64_t i0 = (int64_t)r0 + rl - lane;       // first row of the wave
    if (i0 >= r1) return;                              // the whole wave is past the level
    const int nr = (int)min((int64_t)64, (int64_t)r1 - i0);
    const bool valid = lane < nr;
    const int i = (int)i0 + lane;
    float4* st = stage[threadIdx.x >> 6];
    ACC acc[CB];
    float zi[CB];
    if (FIRST) {
        double vi[CB];
        rows_load(v, i0, nr, st, lane, vi);
        ACC x[CB];
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            const double sc = vscale[c];
#pragma unroll
            for (int r = 0; r < NB; ++r) x[c * NB + r] = (ACC)(float)(sc * vi[c * NB + r]);
        }
        float bs[CB];
#pragma unroll
        for (int q = 0; q < CB; ++q) bs[q] = 0.0f;
        if (valid) {
            float db[25];
            load_block_nt(Dinv, np, 0, i, db);
            block_mul(bs, db, x);
        }
        rows_store(b, i0, nr, st, lane, bs);
#pragma unroll
        for (int q = 0; q < CB; ++q) acc[q] = (ACC)bs[q];
    } else {
        float bl[CB];
        rows_load(z, i0, nr, st, lane, zi);
        rows_load(b, i0, nr, st, lane, bl);
#pragma unroll
        for (int q = 0; q < CB; ++q) acc[q] = (ACC)bl[q];
        if (valid) {
            float gb[25];
            load_block_nt(G, np, 0, i, gb);
            block_add(acc, gb, zi);
        }
    }
    // lower neighbours: for rows of level 0 (rows [0, zrows)) b' in the
    // first sweep (their w) and z later (their t); for the others w in the
    // first sweep and t later
    if (valid) {
        if (FIRST)
            slice_sub_split(acc, KLv, Li.col, slice_ref(Li, sbase, rl), (const float*)b, (const float*)w, zrows);
        else
            slice_sub_split(acc, KLv, Li.col, slice_ref(Li, sbase, rl), (const float*)z, (const float*)t, zrows);
    }
    float wi[CB];
#pragma unroll
    for (int q = 0; q < CB; ++q) wi[q] = (float)acc[q];
    if (!FIRST && !LAST) {
        float wprev[CB], ti[CB];
        rows_load(w, i0, nr, st, lane, wprev);
#pragma unroll
        for (int q = 0; q < CB; ++q) ti[q] = wi[q] - wprev[q] + zi[q];
        rows_store(t, i0, nr, st, lane, ti);
    }
    // rows of the last level have no upper neighbours: z = w, and no later
    // pass reads their w; level 0's w is b', already stored
    if (LAST)
        rows_store(z, i0, nr, st, lane, wi);
    else if (!(FIRST && r1 <= zrows))
        rows_store(w, i0, nr, st, lane, wi);
}

template <bool FIRST, bool LAST, typename ACC>
__global__ void __launch_bounds__(TPB) k_es_fwd(int np, int r0, int r1, int sbase, int zrows, SlicedIdx Li,
                                                const float* __restrict__ KLv, const float* __restrict__ G,
                                                const float* __restrict__ Dinv, const double* __restrict__ v,
                                                const double* __restrict__ vscale, float* __restrict__ b,
                                                float* __restrict__ t, float* __restrict__ w,
                                                float* __restrict__ z, const int32_t* __restrict__ gate) {
    es_fwd_body<Grid1, FIRST, LAST, ACC>(Grid1(), np, r0, r1, sbase, zrows, Li, KLv, G, Dinv, v, vscale, b, t, w, z, gate);
}

struct EsFwdArgs {
    int np;
    int r0;
    int r1;
    int sbase;
    int zrows;
    SlicedIdx Li;
    const float* KLv;
    const float* G;
    const float* Dinv;
    const double* v;
    const double* vscale;
    float* b;
    float* t;
    float* w;
    float* z;
    const int32_t* gate;
};

template <bool FIRST, bool LAST, typename ACC>
__global__ void __launch_bounds__(TPB) kg_es_fwd(Group<EsFwdArgs> g) {
    GridV v;
    const int r = group_locate(g, v);
    if (r < 0) return;
    const EsFwdArgs& a = g.a[r];
    es_fwd_body<GridV, FIRST, LAST, ACC>(v, a.np, a.r0, a.r1, a.sbase, a.zrows, a.Li, a.KLv, a.G, a.Dinv, a.v, a.vscale, a.b, a.t, a.w, a.z, a.gate);
}


template <class GRID, typename ACC>
__device__ __forceinline__ void es_bwd_body(GRID grid, int r0, int r1, int sbase, SlicedIdx Ui, const float* __restrict__ KUv, const float* __restrict__ w, float* __restrict__ z, const int32_t* __restrict__ gate) {
    if (gate && *gate == 0) return;
    __shared__ float4 stage[TPB / 64][64 * CB / 4];
    const int rl = xcd_row(grid);
    const int lane = threadIdx.x & 63;
    const int64_t i0 = (int64_t)r0 + rl - lane;
    if (i0 >= r1) return;
    const int nr = (int)min((int64_t)64, (int64_t)r1 - i0);
    const bool valid = lane < nr;
    const int i = (int)i0 + lane;
    float4* st = stage[threadIdx.x >> 6];
    float wi[CB];
    rows_load(w, i0, nr, st, lane, wi);
    ACC acc[CB];
#pragma unroll
    for (int q = 0; q < CB; ++q) acc[q] = (ACC)wi[q];
    if (valid) slice_sub(acc, KUv, Ui.col, slice_ref(Ui, sbase, rl), z);   // acc = w_i - sum U'_ij z'_j
    float zn[CB];
#pragma unroll
    for (int q = 0; q < CB; ++q) zn[q] = (float)acc[q];
    rows_store(z, i0, nr, st, lane, zn);
}

// At most 128 VGPRs (four waves per SIMD): the backward sweep fits them
// without spills and the extra wave hides more of its gather latency.
template <typename ACC>
__global__ void __launch_bounds__(TPB, 4) k_es_bwd(int r0, int r1, int sbase, SlicedIdx Ui,
                                                const float* __restrict__ KUv, const float* __restrict__ w,
                                                float* __restrict__ z, const int32_t* __restrict__ gate) {
    es_bwd_body<Grid1, ACC>(Grid1(), r0, r1, sbase, Ui, KUv, w, z, gate);
}

struct EsBwdArgs {
    int r0;
    int r1;
    int sbase;
    SlicedIdx Ui;
    const float* KUv;
    const float* w;
    float* z;
    const int32_t* gate;
};

template <typename ACC>
__global__ void __launch_bounds__(TPB, 4) kg_es_bwd(Group<EsBwdArgs> g) {
    GridV v;
    const int r = group_locate(g, v);
    if (r < 0) return;
    const EsBwdArgs& a = g.a[r];
    es_bwd_body<GridV, ACC>(v, a.r0, a.r1, a.sbase, a.Ui, a.KUv, a.w, a.z, a.gate);
}


// ------------------------------------------------------------------ reductions
// Per-column dot products p_j = V_j . w for j in a chunk of RED_CHUNK vectors
// (blockIdx.y selects the chunk).  Each block writes its partial sums to
// partial[(j * NC + c) * nblk + blockIdx.x].
template <class GRID>
__device__ __forceinline__ void dots_body(GRID grid, int n, const double* __restrict__ V, int64_t vstride, int nvec, const double* __restrict__ w, double* __restrict__ partial, const int32_t* __restrict__ gate) {
    if (gate && *gate == 0) return;
    __shared__ double sh[RED_CHUNK * NC][TPB / 64];
    const int j0 = blockIdx.y * RED_CHUNK;
    const int nj = min(RED_CHUNK, nvec - j0);
    double acc[RED_CHUNK][NC];
#pragma unroll
    for (int j = 0; j < RED_CHUNK; ++j)
#pragma unroll
        for (int c = 0; c < NC; ++c) acc[j][c] = 0.0;
    for (int i = grid.b() * blockDim.x + threadIdx.x; i < n; i += grid.g() * blockDim.x) {
        double wv[CB];
        const double* wi = w + (int64_t)i * CB;
#pragma unroll
        for (int q = 0; q < CB; ++q) wv[q] = wi[q];
#pragma unroll
        for (int j = 0; j < RED_CHUNK; ++j) {
            if (j < nj) {
                const double* vi = V + (int64_t)(j0 + j) * vstride + (int64_t)i * CB;
#pragma unroll
                for (int c = 0; c < NC; ++c)
#pragma unroll
                    for (int l = 0; l < NB; ++l) acc[j][c] += vi[c * NB + l] * wv[c * NB + l];
            }
        }
    }
    // wave reduction (fixed butterfly order), then across the block's waves
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
    for (int j = 0; j < RED_CHUNK; ++j)
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            double v = acc[j][c];
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
            if (lane == 0) sh[j * NC + c][wid] = v;
        }
    __syncthreads();
    if (threadIdx.x < nj * NC) {
        double s = 0.0;
#pragma unroll
        for (int q = 0; q < TPB / 64; ++q) s += sh[threadIdx.x][q];
        const int j = threadIdx.x / NC, c = threadIdx.x % NC;
        partial[((int64_t)(j0 + j) * NC + c) * grid.g() + grid.b()] = s;
    }
}

__global__ void __launch_bounds__(TPB) k_dots(int n, const double* __restrict__ V, int64_t vstride, int nvec,
                                              const double* __restrict__ w, double* __restrict__ partial,
    const int32_t* __restrict__ gate) {
    dots_body(Grid1(), n, V, vstride, nvec, w, partial, gate);
}

struct DotsArgs {
    int n;
    const double* V;
    int64_t vstride;
    int nvec;
    const double* w;
    double* partial;
    const int32_t* gate;
};

__global__ void __launch_bounds__(TPB) kg_dots(Group<DotsArgs> g) {
    GridV v;
    const int r = group_locate(g, v);
    if (r < 0) return;
    const DotsArgs& a = g.a[r];
    dots_body(v, a.n, a.V, a.vstride, a.nvec, a.w, a.partial, a.gate);
}


// Vector kernels over the Krylov basis map one 16-byte group of a cell's 20
// values to a thread (10 threads per cell for FP64, 5 for FP32), so each load
// instruction of a wave reads 1 KiB of contiguous memory and several basis
// vectors are in flight per thread.  Value q of a cell belongs to column q / 5.
template <typename VT>
struct Grp {
    static constexpr int E = 16 / sizeof(VT);   // values per thread
    static constexpr int T = CB / E;            // threads per cell
};

// out = w - sum_j h_j[c] scale_j[c] V_j   (out may alias w).  With partial
// != NULL the block also writes the per-column sums of out^2.
template <class GRID>
__device__ __forceinline__ void axpy_body(GRID grid, int n, const double* __restrict__ V, int64_t vstride, int nvec, const double* __restrict__ h, const double* __restrict__ scale, const double* w, double* out, const int32_t* __restrict__ gate, double* __restrict__ partial) {
    if (gate && *gate == 0) return;
    double sq[NC] = {0.0, 0.0, 0.0, 0.0};
    const int64_t npair = (int64_t)n * 10;
    for (int64_t t = (int64_t)grid.b() * blockDim.x + threadIdx.x; t < npair; t += (int64_t)grid.g() * blockDim.x) {
        const int64_t i = t / 10;
        const int p = (int)(t - i * 10);
        const int c0 = (2 * p) / NB, c1 = (2 * p + 1) / NB;
        const int64_t off = i * CB + 2 * p;
        const double2 w2 = *reinterpret_cast<const double2*>(w + off);
        double a0 = w2.x, a1 = w2.y;
#pragma unroll 4
        for (int j = 0; j < nvec; ++j) {
            const nvd2 vn = __builtin_nontemporal_load(reinterpret_cast<const nvd2*>(V + (int64_t)j * vstride + off));
            const double2 v = make_double2(vn[0], vn[1]);
            a0 -= h[j * NC + c0] * scale[j * NC + c0] * v.x;
            a1 -= h[j * NC + c1] * scale[j * NC + c1] * v.y;
        }
        *reinterpret_cast<double2*>(out + off) = make_double2(a0, a1);
        // columns of a pair: c0 == c1 except for pairs straddling a column
#pragma unroll
        for (int c = 0; c < NC; ++c) sq[c] += (c == c0 ? a0 * a0 : 0.0) + (c == c1 ? a1 * a1 : 0.0);
    }
    if (partial) block_sumsq4(sq, partial, grid);
}

__global__ void __launch_bounds__(TPB) k_axpy(int n, const double* __restrict__ V, int64_t vstride, int nvec,
                                              const double* __restrict__ h, const double* __restrict__ scale,
                                              const double* w, double* out,
    const int32_t* __restrict__ gate, double* __restrict__ partial) {
    axpy_body(Grid1(), n, V, vstride, nvec, h, scale, w, out, gate, partial);
}

struct AxpyArgs {
    int n;
    const double* V;
    int64_t vstride;
    int nvec;
    const double* h;
    const double* scale;
    const double* w;
    double* out;
    const int32_t* gate;
    double* partial;
};

__global__ void __launch_bounds__(TPB) kg_axpy(Group<AxpyArgs> g) {
    GridV v;
    const int r = group_locate(g, v);
    if (r < 0) return;
    const AxpyArgs& a = g.a[r];
    axpy_body(v, a.n, a.V, a.vstride, a.nvec, a.h, a.scale, a.w, a.out, a.gate, a.partial);
}


// out = sum_j y_j[c] scale_j[c] V_j
// out = sum_j y_j scale_j V_j, or out += that sum (ACCUM: the mixed form's
// X += Z y in one pass)
template <class GRID, typename VT, bool ACCUM, typename OT = double>
__device__ __forceinline__ void combine_body(GRID grid, int n, const VT* __restrict__ V, int64_t vstride, int nvec, const double* __restrict__ y, const double* __restrict__ scale, OT* __restrict__ out, const int32_t* __restrict__ nvec_dev, const int32_t* __restrict__ gate) {
    if (gate && *gate == 0) return;
    if (nvec_dev) nvec = min(nvec, *nvec_dev);
    constexpr int E = Grp<VT>::E, TC = Grp<VT>::T;
    const int64_t t = (int64_t)grid.b() * blockDim.x + threadIdx.x;
    const int64_t i = t / TC;
    const int p = (int)(t - i * TC);
    if (i >= n) return;
    int col[E];
#pragma unroll
    for (int e = 0; e < E; ++e) col[e] = (E * p + e) / NB;
    const int64_t off = i * CB + E * p;
    double acc[E];
#pragma unroll
    for (int e = 0; e < E; ++e) acc[e] = 0.0;
#pragma unroll 4
    for (int j = 0; j < nvec; ++j) {
        VT v[E];
        {
            const typename NV<VT>::type vn =
                __builtin_nontemporal_load(reinterpret_cast<const typename NV<VT>::type*>(V + (int64_t)j * vstride + off));
#pragma unroll
            for (int e = 0; e < E; ++e) v[e] = vn[e];
        }
#pragma unroll
        for (int e = 0; e < E; ++e) acc[e] += y[j * NC + col[e]] * scale[j * NC + col[e]] * (double)v[e];
    }
#pragma unroll
    for (int e = 0; e < E; ++e) {
        if (ACCUM)
            out[off + e] += (OT)acc[e];
        else
            out[off + e] = (OT)acc[e];
    }
}

template <typename VT, bool ACCUM = false>
__global__ void __launch_bounds__(TPB) k_combine(int n, const VT* __restrict__ V, int64_t vstride, int nvec,
                                                 const double* __restrict__ y, const double* __restrict__ scale,
                                                 double* __restrict__ out, const int32_t* __restrict__ nvec_dev,
                                                 const int32_t* __restrict__ gate) {
    combine_body<Grid1, VT, ACCUM>(Grid1(), n, V, vstride, nvec, y, scale, out, nvec_dev, gate);
}

// z = sum_j y_j scale_j T_j into an FP32 vector (the inner GMRES result)
__global__ void __launch_bounds__(TPB) k_combine_f32out(int n, const float* __restrict__ V, int64_t vstride, int nvec,
                                                        const double* __restrict__ y, const double* __restrict__ scale,
                                                        float* __restrict__ out, const int32_t* __restrict__ nvec_dev,
                                                        const int32_t* __restrict__ gate) {
    combine_body<Grid1, float, false, float>(Grid1(), n, V, vstride, nvec, y, scale, out, nvec_dev, gate);
}

template <typename VT>
struct CombineArgs {
    int n;
    const VT* V;
    int64_t vstride;
    int nvec;
    const double* y;
    const double* scale;
    double* out;
    const int32_t* nvec_dev;
    const int32_t* gate;
};

template <typename VT, bool ACCUM = false>
__global__ void __launch_bounds__(TPB) kg_combine(Group<CombineArgs<VT>> g) {
    GridV v;
    const int r = group_locate(g, v);
    if (r < 0) return;
    const CombineArgs<VT>& a = g.a[r];
    combine_body<GridV, VT, ACCUM>(v, a.n, a.V, a.vstride, a.nvec, a.y, a.scale, a.out, a.nvec_dev, a.gate);
}


// X += z
template <class GRID>
__device__ __forceinline__ void acc_body(GRID grid, int64_t len, double* __restrict__ X, const double* __restrict__ z, const int32_t* __restrict__ gate) {
    if (gate && *gate == 0) return;
    const int64_t i = (int64_t)grid.b() * blockDim.x + threadIdx.x;
    if (i < len) X[i] += z[i];
}

__global__ void __launch_bounds__(TPB) k_acc(int64_t len, double* __restrict__ X, const double* __restrict__ z,
                                             const int32_t* __restrict__ gate) {
    acc_body(Grid1(), len, X, z, gate);
}

struct AccArgs {
    int64_t len;
    double* X;
    const double* z;
    const int32_t* gate;
};

__global__ void __launch_bounds__(TPB) kg_acc(Group<AccArgs> g) {
    GridV v;
    const int r = group_locate(g, v);
    if (r < 0) return;
    const AccArgs& a = g.a[r];
    acc_body(v, a.len, a.X, a.z, a.gate);
}


// Sum partials of nval values in a fixed order: one wave per value.
// mode 0: out[v] = sum;  mode 1: out[v] = sum * scale[v]
// One block per value: each thread sums a strided subset with four
// independent accumulators (loads in flight), then the block reduces them;
// the order is fixed, so results are reproducible.
template <class GRID>
__device__ __forceinline__ void sum_partials_body(GRID grid, int nval, int nblk, const double* __restrict__ partial, const double* __restrict__ scale, double* __restrict__ out, const int32_t* __restrict__ gate) {
    if (gate && *gate == 0) return;
    __shared__ double sh[TPB / 64];
    const int v = grid.b();
    const double* p = partial + (int64_t)v * nblk;
    double a[4] = {0.0, 0.0, 0.0, 0.0};
    int b = threadIdx.x;
    for (; b + 3 * TPB < nblk; b += 4 * TPB) {
#pragma unroll
        for (int k = 0; k < 4; ++k) a[k] += p[b + k * TPB];
    }
    for (int k = 0; b < nblk; b += TPB, ++k) a[k & 3] += p[b];
    double s = (a[0] + a[1]) + (a[2] + a[3]);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
    if (lane == 0) sh[wid] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
#pragma unroll
        for (int q = 0; q < TPB / 64; ++q) t += sh[q];
        out[v] = scale ? t * scale[v] : t;
    }
}

__global__ void __launch_bounds__(TPB) k_sum_partials(int nval, int nblk, const double* __restrict__ partial,
                                                      const double* __restrict__ scale, double* __restrict__ out,
    const int32_t* __restrict__ gate) {
    sum_partials_body(Grid1(), nval, nblk, partial, scale, out, gate);
}

struct SumArgs {
    int nval;
    int nblk;
    const double* partial;
    const double* scale;
    double* out;
    const int32_t* gate;
};

__global__ void __launch_bounds__(TPB) kg_sum_partials(Group<SumArgs> g) {
    GridV v;
    const int r = group_locate(g, v);
    if (r < 0) return;
    const SumArgs& a = g.a[r];
    sum_partials_body(v, a.nval, a.nblk, a.partial, a.scale, a.out, a.gate);
}


// ------------------------------------------------------------------ GMRES bookkeeping (one wave)
// mode 0 (BNORM):   ||R_c|| from sq, active = ||R_c|| > 0
// mode 1 (BETA):    start of a cycle from ||r_c||^2: beta, scale_0, g, k = 0
// mode 2 (ARNOLDI): column k of H from h1 + h2 and ||w||^2, Givens rotation,
//                   residual estimate, k += 1
// mode 3 (SOLVE):   y = R^{-1} g over the first k columns
template <class GRID>
__device__ __forceinline__ void gmres_ctl_body(GRID grid, int mode, KrylovState* __restrict__ ks, int mres, int gated) {
    if (mode == 4) {
        // Whether the second Gram-Schmidt pass runs (ks->reorth gates it):
        // it does when, for a column still iterating, the first pass left
        // the new vector w1 measurably non-orthogonal to the basis,
        // |V^T w1| > reorth_tol |w1| (the second products h2 and the squared
        // norm sq of w1 are in place).  reorth_tol = 0 always takes it (CGS2).
        __shared__ int need[NC];
        const int c = threadIdx.x;
        const int run = ks->st.run;
        if (c < NC) {
            int nd = 1;
            if (ks->reorth_tol > 0.0) {
                double hh = 0.0;
                for (int j = 0; j <= ks->st.k; ++j) hh += ks->h2[j][c] * ks->h2[j][c];
                const double t = ks->reorth_tol;
                nd = ks->st.active[c] && !ks->st.conv[c] && hh > t * t * ks->sq[c];
            }
            need[c] = nd;
        }
        __syncthreads();
        if (c == 0) {
            int any = 0;
            for (int q = 0; q < NC; ++q) any |= need[q];
            const int r = run && any;
            ks->reorth = r;
            ks->st.reorths += r;
        }
        return;
    }
    if (mode == 2 && ks->st.run == 0) return;   // the cycle has ended
    if (gated && ks->st.fin == 0) return;        // end-of-cycle work while the cycle still runs
    const int c = threadIdx.x;
    const int k = ks->st.k;
    const int conv_in = c < NC ? ks->st.conv[c] : 1;
    __syncthreads();
    if (c < NC) {
        Status& st = ks->st;
        if (mode == 0) {
            const double b = sqrt(ks->sq[c]);
            st.bnorm[c] = b;
            st.active[c] = b > 0.0;
            st.its[c] = 0;
            st.beta0[c] = -1.0;
        } else if (mode == 1) {
            const double b = sqrt(ks->sq[c]);
            st.beta[c] = b;
            if (st.beta0[c] < 0.0) st.beta0[c] = b;
            ks->scale[0][c] = b > 0.0 ? 1.0 / b : 0.0;
            for (int j = 0; j <= MAXM; ++j) ks->g[j][c] = 0.0;
            ks->g[0][c] = b;
            const double bn = st.bnorm[c];
            st.est[c] = bn > 0.0 ? b / bn : 0.0;
            st.conv[c] = (!st.active[c]) || b <= ks->tol * bn;
        } else if (mode == 2) {
            // column of H: the products of the passes that ran
            double col[MAXM + 1];
            const int two = ks->reorth;
            for (int j = 0; j <= k; ++j) col[j] = two ? ks->h1[j][c] + ks->h2[j][c] : ks->h1[j][c];
            const double hn = sqrt(ks->sq[c]);
            col[k + 1] = hn;
            ks->scale[k + 1][c] = hn > 0.0 ? 1.0 / hn : 0.0;
            for (int j = 0; j < k; ++j) {
                const double t = ks->cs[j][c] * col[j] + ks->sn[j][c] * col[j + 1];
                col[j + 1] = -ks->sn[j][c] * col[j] + ks->cs[j][c] * col[j + 1];
                col[j] = t;
            }
            const double d = hypot(col[k], col[k + 1]);
            double cs = 1.0, sn = 0.0;
            if (d > 0.0) {
                cs = col[k] / d;
                sn = col[k + 1] / d;
            }
            ks->cs[k][c] = cs;
            ks->sn[k][c] = sn;
            col[k] = d;
            col[k + 1] = 0.0;
            for (int j = 0; j <= k + 1; ++j) ks->H[k][j][c] = col[j];
            const double gk = ks->g[k][c];
            ks->g[k + 1][c] = -sn * gk;
            ks->g[k][c] = cs * gk;
            const double bn = st.bnorm[c];
            const double e = bn > 0.0 ? fabs(ks->g[k + 1][c]) / bn : 0.0;
            st.est[c] = e;
            st.conv[c] = (!st.active[c]) || e <= ks->tol;
            if (!conv_in) st.its[c] = st.total + 1;
        } else if (mode == 3) {
            for (int j = k - 1; j >= 0; --j) {
                double s = ks->g[j][c];
                for (int q = j + 1; q < k; ++q) s -= ks->H[q][j][c] * ks->y[q][c];
                const double d = ks->H[j][j][c];
                ks->y[j][c] = d != 0.0 ? s / d : 0.0;
            }
        }
    }
    __syncthreads();
    if (c == 0) {
        int all = 1;
        for (int q = 0; q < NC; ++q) all &= ks->st.conv[q];
        if (mode == 0) {
            ks->st.total = 0;
            ks->st.cycles = 0;
            ks->st.reorths = 0;
        }
        if (mode == 1) {
            ks->st.k = 0;
            ks->st.run = !all;
            ks->st.fin = 0;
            ks->st.cycles += !all;
        }
        if (mode == 2) {
            ks->st.k = k + 1;
            ks->st.total += 1;
            ks->st.run = !all && (k + 1 < mres);
            ks->st.fin = !ks->st.run;
        }
    }
}

__global__ void __launch_bounds__(64) k_gmres_ctl(int mode, KrylovState* __restrict__ ks, int mres, int gated) {
    gmres_ctl_body(Grid1(), mode, ks, mres, gated);
}

// Start of an inner GMRES solve on the unit vector s .* v: residual norm 1
// in every column, basis scale s, no column converged (the inner tolerance
// is 0: the solve runs its fixed number of steps).
__global__ void __launch_bounds__(64) k_inner_init(KrylovState* __restrict__ ki, const double* __restrict__ vscale,
                                                   const int32_t* __restrict__ gate) {
    if (gate && *gate == 0) return;
    const int c = threadIdx.x;
    if (c < NC) {
        ki->scale[0][c] = vscale[c];
        for (int j = 0; j <= MAXM; ++j) ki->g[j][c] = 0.0;
        ki->g[0][c] = 1.0;
        ki->st.bnorm[c] = 1.0;
        ki->st.beta[c] = 1.0;
        ki->st.est[c] = 1.0;
        ki->st.active[c] = 1;
        ki->st.conv[c] = 0;
        ki->st.its[c] = 0;
    }
    if (c == 0) {
        ki->st.k = 0;
        ki->st.run = 1;
        ki->st.fin = 0;
        ki->st.total = 0;
        ki->st.cycles = 1;
        ki->st.reorths = 0;
    }
}

struct CtlArgs {
    int mode;
    KrylovState* ks;
    int mres;
    int gated;
};

__global__ void __launch_bounds__(64) kg_gmres_ctl(Group<CtlArgs> g) {
    GridV v;
    const int r = group_locate(g, v);
    if (r < 0) return;
    const CtlArgs& a = g.a[r];
    gmres_ctl_body(v, a.mode, a.ks, a.mres, a.gated);
}


// ------------------------------------------------------------------ layout conversion
// X in the caller's layout [4][5][nt] from the solver vector: one thread per
// cell in the caller's order (coalesced writes, one 160-byte read).
template <class GRID, typename T>
__device__ __forceinline__ void copyout_body(GRID grid, int nt, const int32_t* __restrict__ iperm, const T* __restrict__ Xs, double* __restrict__ Xc) {
    const int oi = xcd_row(grid);
    if (oi >= nt) return;
    const T* xi = Xs + (int64_t)iperm[oi] * CB;
#pragma unroll
    for (int q = 0; q < CB; ++q) Xc[(int64_t)q * nt + oi] = (double)xi[q];
}

template <typename T>
__global__ void __launch_bounds__(TPB) k_copyout(int nt, const int32_t* __restrict__ iperm,
                                                 const T* __restrict__ Xs, double* __restrict__ Xc) {
    copyout_body<Grid1, T>(Grid1(), nt, iperm, Xs, Xc);
}

template <typename T>
struct CopyoutArgs {
    int nt;
    const int32_t* iperm;
    const T* Xs;
    double* Xc;
};

template <typename T>
__global__ void __launch_bounds__(TPB) kg_copyout(Group<CopyoutArgs<T>> g) {
    GridV v;
    const int r = group_locate(g, v);
    if (r < 0) return;
    const CopyoutArgs<T>& a = g.a[r];
    copyout_body<GridV, T>(v, a.nt, a.iperm, a.Xs, a.Xc);
}


// Initial guess for the next step's solve: the polynomial through the last
// npts solutions at their times, evaluated at the current time:
// g = c[0] x + c[1] h0 + c[2] h1 + ..., with x the last solution, h0, h1, ...
// the earlier ones (newest first) and c the Lagrange weights the host
// computes from the step sizes (at uniform steps the alternating binomial
// ones: x; 2x - h0; 3x - 3h0 + h1; ...).  The earlier solutions are kept in
// FP64 in a ring: the larger coefficients of the longer
// polynomials would amplify the rounding of FP32 copies above the
// extrapolation error of smooth flows.  x goes into the ring's oldest slot
// (hout, which may be the slot read as the oldest term: each element is read
// before it is overwritten).
struct ExtrapArgs {
    int64_t len;
    int npts;
    double c[MAXH + 1];     // weights of x, h0, h1, ...
    double* X;
    const double* h[MAXH];  // newest first
    double* hout;           // null without a ring
};

template <class GRID>
__device__ __forceinline__ void extrap_body(GRID grid, const ExtrapArgs& a) {
    const int64_t e = (int64_t)grid.b() * blockDim.x + threadIdx.x;
    if (e >= a.len) return;
    const double x = a.X[e];
    double g = a.c[0] * x;
    for (int i = 1; i < a.npts; ++i) g = fma(a.c[i], a.h[i - 1][e], g);
    a.X[e] = g;
    if (a.hout) a.hout[e] = x;
}

__global__ void __launch_bounds__(TPB) k_extrap(ExtrapArgs a) { extrap_body(Grid1(), a); }

__global__ void __launch_bounds__(TPB) kg_extrap(Group<ExtrapArgs> g) {
    GridV v;
    const int r = group_locate(g, v);
    if (r < 0) return;
    extrap_body(v, g.a[r]);
}


// solver vector from the caller's layout [4][5][nt] (inverse of k_copyout)
__global__ void __launch_bounds__(TPB) k_copyin(int nt, const int32_t* __restrict__ iperm,
                                                const double* __restrict__ Xc, double* __restrict__ Xs) {
    const int oi = xcd_row();
    if (oi >= nt) return;
    double* xi = Xs + (int64_t)iperm[oi] * CB;
#pragma unroll
    for (int q = 0; q < CB; ++q) xi[q] = Xc[(int64_t)q * nt + oi];
}

__global__ void k_set(double* p, double v) { *p = v; }

__global__ void __launch_bounds__(TPB) k_zero(int64_t len, double* __restrict__ p) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < len) p[i] = 0.0;
}

template <class GRID>
__device__ __forceinline__ void copy_body(GRID grid, int64_t len, double* __restrict__ d, const double* __restrict__ s) {
    const int64_t i = (int64_t)grid.b() * blockDim.x + threadIdx.x;
    if (i < len) d[i] = s[i];
}

__global__ void __launch_bounds__(TPB) k_copy(int64_t len, double* __restrict__ d, const double* __restrict__ s) {
    copy_body(Grid1(), len, d, s);
}

struct CopyArgs {
    int64_t len;
    double* d;
    const double* s;
};

__global__ void __launch_bounds__(TPB) kg_copy(Group<CopyArgs> g) {
    GridV v;
    const int r = group_locate(g, v);
    if (r < 0) return;
    const CopyArgs& a = g.a[r];
    copy_body(v, a.len, a.d, a.s);
}


// zero the inactive columns of X (a zero right-hand side has X = 0)
template <class GRID>
__device__ __forceinline__ void mask_cols_body(GRID grid, int n, double* __restrict__ X, const KrylovState* __restrict__ ks) {
    const int i = grid.b() * blockDim.x + threadIdx.x;
    if (i >= n) return;
#pragma unroll
    for (int c = 0; c < NC; ++c)
        if (!ks->st.active[c])
#pragma unroll
            for (int l = 0; l < NB; ++l) X[(int64_t)i * CB + c * NB + l] = 0.0;
}

__global__ void __launch_bounds__(TPB) k_mask_cols(int n, double* __restrict__ X, const KrylovState* __restrict__ ks) {
    mask_cols_body(Grid1(), n, X, ks);
}

struct MaskArgs {
    int n;
    double* X;
    const KrylovState* ks;
};

__global__ void __launch_bounds__(TPB) kg_mask_cols(Group<MaskArgs> g) {
    GridV v;
    const int r = group_locate(g, v);
    if (r < 0) return;
    const MaskArgs& a = g.a[r];
    mask_cols_body(v, a.n, a.X, a.ks);
}


// ------------------------------------------------------------------ flux
struct FluxArgs {
    int nf, nt;
    const int32_t* own;
    const int32_t* nbr;
    const double* fgeo;
    const double* gpd;
    const double* cgeo;
    const int32_t* bc_kind;
    const double* bc_state;
    const double* W;
    const double* X;
    const double* dt;
    double* F;
    int32_t* nonphys;
    gksdev::FluxParams fp;
    int fallback;
};

// Cell polynomial value, gradient and Hessian at offset (dx, dy) (in units of
// h), rotated into the face frame: Wloc and d[5][4] = n, t, nn, nt, tt.
__device__ __forceinline__ void gp_state(const FluxArgs& a, int cell, double dx, double dy, double nx, double ny,
                                         double Wloc[4], double d[5][4]) {
    const int nt = a.nt;
    const double ih = a.cgeo[cell];
    const double mxx = a.cgeo[nt + cell], mxy = a.cgeo[2 * nt + cell], myy = a.cgeo[3 * nt + cell];
    const double phi[5] = {dx, dy, 0.5 * (dx * dx - mxx), dx * dy - mxy, 0.5 * (dy * dy - myy)};
    double Q[4], Qx[4], Qy[4], Qxx[4], Qxy[4], Qyy[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        double X[5];
#pragma unroll
        for (int l = 0; l < 5; ++l) X[l] = a.X[(int64_t)(v * 5 + l) * nt + cell];
        double q = a.W[(int64_t)v * nt + cell];
#pragma unroll
        for (int l = 0; l < 5; ++l) q += X[l] * phi[l];
        Q[v] = q;
        Qx[v] = (X[0] + X[2] * dx + X[3] * dy) * ih;
        Qy[v] = (X[1] + X[3] * dx + X[4] * dy) * ih;
        Qxx[v] = X[2] * ih * ih;
        Qxy[v] = X[3] * ih * ih;
        Qyy[v] = X[4] * ih * ih;
    }
    const double tx = -ny, ty = nx;
    double loc[6][4];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        loc[0][v] = Q[v];
        loc[1][v] = nx * Qx[v] + ny * Qy[v];
        loc[2][v] = tx * Qx[v] + ty * Qy[v];
        loc[3][v] = nx * nx * Qxx[v] + 2.0 * nx * ny * Qxy[v] + ny * ny * Qyy[v];
        loc[4][v] = nx * tx * Qxx[v] + (nx * ty + ny * tx) * Qxy[v] + ny * ty * Qyy[v];
        loc[5][v] = tx * tx * Qxx[v] + 2.0 * tx * ty * Qxy[v] + ty * ty * Qyy[v];
    }
    // rotate the momentum pair into (n, t)
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        const double mx = loc[k][1], my = loc[k][2];
        loc[k][1] = mx * nx + my * ny;
        loc[k][2] = -mx * ny + my * nx;
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        Wloc[v] = loc[0][v];
#pragma unroll
        for (int k = 0; k < 5; ++k) d[k][v] = loc[k + 1][v];
    }
}

__device__ __forceinline__ bool physical(const double W[4], double gamma) {
    return W[0] > 0.0 && gksdev::pressure(W, gamma) > 0.0;
}

__device__ __forceinline__ void cell_average_local(const FluxArgs& a, int cell, double nx, double ny, double W[4],
                                                   double d[5][4]) {
    const double m0 = a.W[(int64_t)1 * a.nt + cell], m1 = a.W[(int64_t)2 * a.nt + cell];
    W[0] = a.W[cell];
    W[1] = m0 * nx + m1 * ny;
    W[2] = -m0 * ny + m1 * nx;
    W[3] = a.W[(int64_t)3 * a.nt + cell];
#pragma unroll
    for (int k = 0; k < 5; ++k)
#pragma unroll
        for (int v = 0; v < 4; ++v) d[k][v] = 0.0;
}

// Ghost state beyond a boundary face (face frame), from the interior side o.
// Walls mirror the one-sided polynomial, inflow is the fixed state, and
// outflow is the cell's own average with zero derivatives (zeroth-order
// extrapolation: the kinetic flux then stays upwind for a characteristic
// entering through a subsonic outflow).
__device__ __forceinline__ void ghost(const FluxArgs& a, int row, int o, const double WL[4], const double dL[5][4],
                                      double nx, double ny, double WR[4], double dR[5][4]) {
    const int kind = a.bc_kind[row];
    const double* st = a.bc_state + 4 * row;
    if (kind == GKS_BC_SLIP || kind == GKS_BC_NOSLIP) {
        double Lm[4][4] = {{1, 0, 0, 0}, {0, -1, 0, 0}, {0, 0, 1, 0}, {0, 0, 0, 1}};
        if (kind == GKS_BC_NOSLIP) {
            const double wn = st[1] * nx + st[2] * ny;
            const double wt = -st[1] * ny + st[2] * nx;
            Lm[1][0] = 2.0 * wn;
            Lm[2][0] = 2.0 * wt;
            Lm[2][2] = -1.0;
            Lm[3][0] = 2.0 * (wn * wn + wt * wt);
            Lm[3][1] = -2.0 * wn;
            Lm[3][2] = -2.0 * wt;
        }
        // mirror: one sign per normal differentiation (n: -, t: +, nn: +, nt: -, tt: +)
        const double sg[5] = {-1.0, 1.0, 1.0, -1.0, 1.0};
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            double s = 0.0;
#pragma unroll
            for (int q = 0; q < 4; ++q) s += Lm[r][q] * WL[q];
            WR[r] = s;
#pragma unroll
            for (int k = 0; k < 5; ++k) {
                double t = 0.0;
#pragma unroll
                for (int q = 0; q < 4; ++q) t += Lm[r][q] * dL[k][q];
                dR[k][r] = sg[k] * t;
            }
        }
    } else if (kind == GKS_BC_INFLOW) {
        const double rho = st[0], u = st[1], v = st[2], p = st[3];
        const double mx = rho * u, my = rho * v;
        WR[0] = rho;
        WR[1] = mx * nx + my * ny;
        WR[2] = -mx * ny + my * nx;
        WR[3] = p / (a.fp.gamma - 1.0) + 0.5 * rho * (u * u + v * v);
#pragma unroll
        for (int k = 0; k < 5; ++k)
#pragma unroll
            for (int q = 0; q < 4; ++q) dR[k][q] = 0.0;
    } else {  // outflow
        cell_average_local(a, o, nx, ny, WR, dR);
    }
}

// One thread per Gauss point; lanes 2f and 2f+1 hold the two points of face f.
template <class GRID>
__device__ __forceinline__ void flux_body(GRID grid, const FluxArgs& a) {
    const int64_t t = (int64_t)grid.b() * blockDim.x + threadIdx.x;
    const int f = (int)(t >> 1);
    const int g = (int)(t & 1);
    const bool valid = f < a.nf;
    double F[4] = {0.0, 0.0, 0.0, 0.0};
    double nx = 1.0, ny = 0.0, S = 0.0;
    if (valid) {
        nx = a.fgeo[f];
        ny = a.fgeo[a.nf + f];
        S = a.fgeo[2 * (int64_t)a.nf + f];
        const int o = a.own[f];
        const int nb = a.nbr[f];
        double WL[4], dL[5][4], WR[4], dR[5][4];
        gp_state(a, o, a.gpd[(int64_t)(4 * g + 0) * a.nf + f], a.gpd[(int64_t)(4 * g + 1) * a.nf + f], nx, ny, WL, dL);
        int bad = 0;
        if (!physical(WL, a.fp.gamma)) {
            ++bad;
            cell_average_local(a, o, nx, ny, WL, dL);
        }
        if (nb >= 0) {
            gp_state(a, nb, a.gpd[(int64_t)(4 * g + 2) * a.nf + f], a.gpd[(int64_t)(4 * g + 3) * a.nf + f], nx, ny,
                     WR, dR);
            if (!physical(WR, a.fp.gamma)) {
                ++bad;
                cell_average_local(a, nb, nx, ny, WR, dR);
            }
        } else {
            ghost(a, -nb, o, WL, dL, nx, ny, WR, dR);
        }
        if (bad) atomicAdd(a.nonphys, bad);
        gksdev::gp_flux(F, WL, dL, WR, dR, *a.dt, a.fp);
    }
    // back to (x, y), weight S/2, sum the two Gauss points of the face
    double Fx[4];
    Fx[0] = 0.5 * S * F[0];
    Fx[1] = 0.5 * S * (F[1] * nx - F[2] * ny);
    Fx[2] = 0.5 * S * (F[1] * ny + F[2] * nx);
    Fx[3] = 0.5 * S * F[3];
#pragma unroll
    for (int q = 0; q < 4; ++q) Fx[q] += __shfl_xor(Fx[q], 1, 64);
    if (valid && g == 0) {
#pragma unroll
        for (int q = 0; q < 4; ++q) a.F[(int64_t)q * a.nf + f] = Fx[q];
    }
}

__global__ void __launch_bounds__(128) k_flux(FluxArgs a) { flux_body(Grid1(), a); }

__global__ void __launch_bounds__(128) kg_flux(Group<FluxArgs> g) {
    GridV v;
    const int r = group_locate(g, v);
    if (r < 0) return;
    flux_body(v, g.a[r]);
}

// ------------------------------------------------------------------ update (Eq. fvm3)
template <class GRID>
__device__ __forceinline__ void update_body(GRID grid, int nt, int nf, const int32_t* __restrict__ cface, const double* __restrict__ area, const double* __restrict__ W, const double* __restrict__ F, double* __restrict__ Wn, double gamma, int32_t* __restrict__ nonphys) {
    const int i = grid.b() * blockDim.x + threadIdx.x;
    if (i >= nt) return;
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const int code = cface[(int64_t)k * nt + i];
        const int f = code >= 0 ? code : ~code;
        const double s = code >= 0 ? -1.0 : 1.0;
#pragma unroll
        for (int q = 0; q < 4; ++q) acc[q] += s * F[(int64_t)q * nf + f];
    }
    const double ia = 1.0 / area[i];
    double w[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        w[q] = W[(int64_t)q * nt + i] + acc[q] * ia;
        Wn[(int64_t)q * nt + i] = w[q];
    }
    if (!(w[0] > 0.0 && gksdev::pressure(w, gamma) > 0.0)) atomicAdd(nonphys, 1);
}

__global__ void __launch_bounds__(TPB) k_update(int nt, int nf, const int32_t* __restrict__ cface,
                                                const double* __restrict__ area, const double* __restrict__ W,
                                                const double* __restrict__ F, double* __restrict__ Wn,
                                                double gamma, int32_t* __restrict__ nonphys) {
    update_body(Grid1(), nt, nf, cface, area, W, F, Wn, gamma, nonphys);
}

struct UpdateArgs {
    int nt;
    int nf;
    const int32_t* cface;
    const double* area;
    const double* W;
    const double* F;
    double* Wn;
    double gamma;
    int32_t* nonphys;
};

__global__ void __launch_bounds__(TPB) kg_update(Group<UpdateArgs> g) {
    GridV v;
    const int r = group_locate(g, v);
    if (r < 0) return;
    const UpdateArgs& a = g.a[r];
    update_body(v, a.nt, a.nf, a.cface, a.area, a.W, a.F, a.Wn, a.gamma, a.nonphys);
}


// ------------------------------------------------------------------ CFL
template <class GRID>
__device__ __forceinline__ void cfl_body(GRID grid, int nt, int nf, const int32_t* __restrict__ cface, const double* __restrict__ area, const double* __restrict__ fgeo, const double* __restrict__ W, double gamma, double* __restrict__ partial) {
    __shared__ double sh[TPB / 64];
    double best = INFINITY;
    for (int i = grid.b() * blockDim.x + threadIdx.x; i < nt; i += grid.g() * blockDim.x) {
        const double rho = W[i], u = W[(int64_t)nt + i] / rho, v = W[2 * (int64_t)nt + i] / rho;
        const double p = (gamma - 1.0) * (W[3 * (int64_t)nt + i] - 0.5 * rho * (u * u + v * v));
        const double c = sqrt(gamma * p / rho);
        double den = 0.0;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const int code = cface[(int64_t)k * nt + i];
            const int f = code >= 0 ? code : ~code;
            den += fgeo[2 * (int64_t)nf + f] * (fabs(u * fgeo[f] + v * fgeo[nf + f]) + c);
        }
        best = fmin(best, area[i] / den);
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) best = fmin(best, __shfl_xor(best, off, 64));
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = best;
    __syncthreads();
    if (threadIdx.x == 0) {
        double b = sh[0];
        for (int q = 1; q < TPB / 64; ++q) b = fmin(b, sh[q]);
        partial[grid.b()] = b;
    }
}

__global__ void __launch_bounds__(TPB) k_cfl(int nt, int nf, const int32_t* __restrict__ cface,
                                             const double* __restrict__ area, const double* __restrict__ fgeo,
                                             const double* __restrict__ W, double gamma,
                                             double* __restrict__ partial) {
    cfl_body(Grid1(), nt, nf, cface, area, fgeo, W, gamma, partial);
}

struct CflArgs {
    int nt;
    int nf;
    const int32_t* cface;
    const double* area;
    const double* fgeo;
    const double* W;
    double gamma;
    double* partial;
};

__global__ void __launch_bounds__(TPB) kg_cfl(Group<CflArgs> g) {
    GridV v;
    const int r = group_locate(g, v);
    if (r < 0) return;
    const CflArgs& a = g.a[r];
    cfl_body(v, a.nt, a.nf, a.cface, a.area, a.fgeo, a.W, a.gamma, a.partial);
}


__device__ __forceinline__ void cfl_final_body(int nblk, const double* __restrict__ partial, double cfl,
                                               double* __restrict__ dt);

__global__ void k_cfl_final(int nblk, const double* __restrict__ partial, double cfl, double* __restrict__ dt) {
    cfl_final_body(nblk, partial, cfl, dt);
}

struct CflFinalArgs {
    int nblk;
    const double* partial;
    double cfl;
    double* dt;
};

__global__ void __launch_bounds__(64) kg_cfl_final(Group<CflFinalArgs> g) {
    GridV v;
    const int r = group_locate(g, v);
    if (r < 0) return;
    const CflFinalArgs& a = g.a[r];
    cfl_final_body(a.nblk, a.partial, a.cfl, a.dt);
}

__device__ __forceinline__ void cfl_final_body(int nblk, const double* __restrict__ partial, double cfl,
                                               double* __restrict__ dt) {
    double b = INFINITY;
    for (int q = threadIdx.x; q < nblk; q += 64) b = fmin(b, partial[q]);
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) b = fmin(b, __shfl_xor(b, off, 64));
    if (threadIdx.x == 0) *dt = cfl * b;
}

// ================================================================== launchers

void prof_begin(gks_mesh* m, int kc, double bytes, double flops) {
    if (!m->prof.on || m->capturing) return;
    m->prof.bytes[kc] += bytes;
    m->prof.flops[kc] += flops;
    hipEvent_t a, b;
    if (m->prof.pool.size() >= 2) {
        a = m->prof.pool.back();
        m->prof.pool.pop_back();
        b = m->prof.pool.back();
        m->prof.pool.pop_back();
    } else {
        (void)hipEventCreate(&a);
        (void)hipEventCreate(&b);
    }
    (void)hipEventRecord(a, m->stream);
    m->prof.pending.push_back({kc, {a, b}});
}

void prof_end(gks_mesh* m, int kc) {
    (void)kc;
    if (!m->prof.on || m->capturing || m->prof.pending.empty()) return;
    (void)hipEventRecord(m->prof.pending.back().second.second, m->stream);
}

// Algorithmic bytes per row of the solver kernels (four columns, FP64
// vectors of 160 bytes per cell): matrix blocks and indices as stored, each
// input vector block read once, each output block written once.
constexpr double VB = CB * 8.0;
inline double spmv_bytes(int n, int esz, bool resid) { return n * (KW * 25.0 * esz + KW * 4.0 + (resid ? 3 : 2) * VB); }

// ------------------------------------------------------------------ DWBAP limiter
// Section 3.3: where the density shock indicator IS_i (Eq. ISD1) reaches
// the threshold (1 in Eq. ISD2), the derivatives of every conserved variable
// are replaced by L = tan(sum_j w_j atan(u_j)) over the cell's own value and
// candidates from its face neighbours (Eq. DWBAP), with weights
// w_j ~ (mean distance from r_j to the cell's face midpoints / h_i)^-S and
// S = 1 / (sqrt(chi + 1e-8) + 0.05), chi = std / mean of the neighbours'
// pressures (Eqs. DWBAP_w, DWBAP_S).  Hierarchical candidates: second
// derivatives from the neighbours' second derivatives; first derivatives
// from the cell averages of the remainder u - q_i (q_i: the cell's quadratic
// part with limited second derivatives): the plane through the cell and each
// pair of neighbours, a pair weighing the mean of its two neighbours'
// weights, or in a wall cell (fewer than three neighbours) the gradient
// along each neighbour's direction alone.  One thread per cell (cell order); the indicator
// needs the neighbours' density polynomials only, and the full neighbour
// data is read for limited cells alone.
struct LimArgs {
    int nt, nf;
    const int32_t* own;
    const int32_t* nbr;
    const int32_t* cface;
    const int32_t* nbc;   // [3][nt] face neighbour per slot (the cell itself: boundary)
    const double* a0c;    // [3][5][nt] averages over the neighbour of the cell's basis
    const double* gpd;
    const double* cgeo;
    const double* W;
    const double* X;      // unlimited coefficients [20][nt]
    double* Xcopy;        // mark: when set, receives X for every cell
    double gamma, threshold;
    int all_quadratic;
    int charvars;         // 1: limit characteristic variables, 0: conserved ones
    int32_t* count;       // number of limited cells (list length)
    int32_t* list;        // [cap] limited cells, in no particular order
    double* lbuf;         // [20][lstride] limited coefficients of list entry k at column k
    double* dst;          // scatter target [20][nt]
    int cap;              // entries the list holds (nt, or the static scratch's limit);
                          // the count goes on past it, entries beyond are not stored
    int lstride;          // column stride of lbuf (>= the entries processed)
};

// Face-neighbour stencil of cell i: interior neighbours, their slots and
// centroid offsets (r_j - r_i) / h_i.
__device__ __forceinline__ int lim_stencil(const LimArgs& a, int i, int nb[3], int slot[3], double dc[3][2]) {
    const int nt = a.nt;
    int J = 0;
    for (int s = 0; s < 3; ++s) {
        const int j = a.nbc[(int64_t)s * nt + i];
        if (j == i) continue;
        nb[J] = j;
        slot[J] = s;
        dc[J][0] = a.a0c[((int64_t)s * 5 + 0) * nt + i];
        dc[J][1] = a.a0c[((int64_t)s * 5 + 1) * nt + i];
        ++J;
    }
    return J;
}

// Shock indicator of Eq. ISD1 on the density, for every cell; limited cells
// are appended to the list.  With Xcopy set, X is copied for every cell.
__global__ void __launch_bounds__(TPB) k_limit_mark(LimArgs a) {
    const int i = xcd_row();
    if (i >= a.nt) return;
    const int nt = a.nt;
    if (a.Xcopy) {
#pragma unroll
        for (int l = 0; l < 20; ++l) a.Xcopy[(int64_t)l * nt + i] = a.X[(int64_t)l * nt + i];
    }
    int nb[3], slot[3];
    double dc[3][2];
    const int J = lim_stencil(a, i, nb, slot, dc);
    if (J == 0) return;
    const int ki = (J < 3 && !a.all_quadratic) ? 1 : 2;
    const double ihi = a.cgeo[i], hi = 1.0 / ihi;
    const double mxx = a.cgeo[nt + i], mxy = a.cgeo[2 * nt + i], myy = a.cgeo[3 * nt + i];
    const double Wi0 = a.W[i];
    const double own = Wi0 - 0.5 * mxx * a.X[(int64_t)2 * nt + i] - mxy * a.X[(int64_t)3 * nt + i] -
                       0.5 * myy * a.X[(int64_t)4 * nt + i];
    double num = 0.0, umax = Wi0;
    for (int n = 0; n < J; ++n) {
        const int j = nb[n];
        const double ihj = a.cgeo[j];
        const double dx = -dc[n][0] * hi * ihj, dy = -dc[n][1] * hi * ihj;   // (r_i - r_j) / h_j
        const double mxj = a.cgeo[nt + j], mxyj = a.cgeo[2 * nt + j], myj = a.cgeo[3 * nt + j];
        double vj = a.W[j];
        const double phi[5] = {dx, dy, 0.5 * (dx * dx - mxj), dx * dy - mxyj, 0.5 * (dy * dy - myj)};
#pragma unroll
        for (int l = 0; l < 5; ++l) vj += a.X[(int64_t)l * nt + j] * phi[l];
        num += fabs(own - vj);
        umax = fmax(umax, a.W[j]);
    }
    const double hk = ki == 2 ? hi * sqrt(hi) : hi;   // h_i^((k+1)/2)
    if (num / (J * hk * umax) >= a.threshold) {
        const int pos = atomicAdd(a.count, 1);
        if (pos < a.cap) a.list[pos] = i;
    }
}

using gksdev::CharBasis;

// Biased average of Eq. DWBAP over the valid candidates (q = 0..3, in order).
__device__ __forceinline__ double dwbap4(const double u[4], const double w[4], const bool ok[4]) {
    double s = 0.0;
#pragma unroll
    for (int q = 0; q < 4; ++q)
        if (ok[q]) s += w[q] * atan(u[q]);
    return tan(s);
}

// Limit one derivative of the four variables: cand[q][v] is candidate q of
// variable v (overwritten), ok[q] whether it exists; out[v] the limited
// derivative.  Conserved variables one by one, or characteristic variables
// mapped back.
__device__ __forceinline__ void limit_vec(double cand[4][4], const double w[4], const bool ok[4], bool charvars,
                                          const CharBasis& cb, double out[4]) {
    if (charvars) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            if (!ok[q]) continue;
            double y[4];
            cb.to_char(cand[q], y);
#pragma unroll
            for (int k = 0; k < 4; ++k) cand[q][k] = y[k];
        }
    }
    double lim[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        double u[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) u[q] = cand[q][k];
        lim[k] = dwbap4(u, w, ok);
    }
    if (charvars)
        cb.from_char(lim, out);
    else
#pragma unroll
        for (int k = 0; k < 4; ++k) out[k] = lim[k];
}

// The DWBAP limiter on the listed cells (grid-stride over the list): the
// limited coefficients of entry k go to column k of lbuf.  Neighbours stay
// in their slots (ok[] marks the interior ones; candidate 1 + s belongs to
// slot s), so every array index is a compile-time constant.
__global__ void __launch_bounds__(64) k_limit_apply(LimArgs a) {
    const int cnt = min(*a.count, a.cap);
    const int nt = a.nt;
    for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < cnt; k += gridDim.x * blockDim.x) {
        const int i = a.list[k];
        const double ihi = a.cgeo[i], hi = 1.0 / ihi;
        int nb[3];
        bool ok[4];
        double dc[3][2];
        int J = 0;
        ok[0] = true;
#pragma unroll
        for (int s = 0; s < 3; ++s) {
            nb[s] = a.nbc[(int64_t)s * nt + i];
            ok[s + 1] = nb[s] != i;
            dc[s][0] = a.a0c[((int64_t)s * 5 + 0) * nt + i];
            dc[s][1] = a.a0c[((int64_t)s * 5 + 1) * nt + i];
            J += ok[s + 1];
        }
        const int ki = (J < 3 && !a.all_quadratic) ? 1 : 2;
        // weights of Eqs. DWBAP_w, DWBAP_S; distances in units of h_i to the
        // midpoints of the interior faces
        double w[4];
        {
            double mid[3][2];
            bool mok[3];
            int nm = 0;
#pragma unroll
            for (int e = 0; e < 3; ++e) {
                const int cf = a.cface[(int64_t)e * nt + i];
                const int f = cf >= 0 ? cf : ~cf;
                const int side = cf >= 0 ? 0 : 1;
                mok[e] = (side == 0 ? a.nbr[f] : a.own[f]) >= 0;
                const int64_t nf = a.nf;
                mid[e][0] = 0.5 * (a.gpd[(2 * side) * nf + f] + a.gpd[(4 + 2 * side) * nf + f]);
                mid[e][1] = 0.5 * (a.gpd[(2 * side + 1) * nf + f] + a.gpd[(4 + 2 * side + 1) * nf + f]);
                nm += mok[e];
            }
            double p[3], pbar = 0.0;
#pragma unroll
            for (int s = 0; s < 3; ++s) {
                p[s] = 0.0;
                if (!ok[s + 1]) continue;
                const int j = nb[s];
                const double r = a.W[j], mu = a.W[(int64_t)nt + j], mv = a.W[(int64_t)2 * nt + j];
                const double E = a.W[(int64_t)3 * nt + j];
                p[s] = (a.gamma - 1.0) * (E - 0.5 * (mu * mu + mv * mv) / r);
                pbar += p[s];
            }
            pbar /= J;
            double var = 0.0;
#pragma unroll
            for (int s = 0; s < 3; ++s)
                if (ok[s + 1]) var += (p[s] - pbar) * (p[s] - pbar);
            const double chi = sqrt(var / J) / pbar;
            const double S = 1.0 / (sqrt(chi + 1e-8) + 0.05);
            double wsum = 0.0;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                w[q] = 0.0;
                if (!ok[q]) continue;
                const double cx = q == 0 ? 0.0 : dc[q - 1][0], cy = q == 0 ? 0.0 : dc[q - 1][1];
                double D = 0.0;
#pragma unroll
                for (int e = 0; e < 3; ++e)
                    if (mok[e]) D += hypot(cx - mid[e][0], cy - mid[e][1]);
                w[q] = pow(D / nm, -S);
                wsum += w[q];
            }
#pragma unroll
            for (int q = 0; q < 4; ++q) w[q] /= wsum;
        }
        double Wi[4], Xi[4][5];
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            Wi[v] = a.W[(int64_t)v * nt + i];
#pragma unroll
            for (int l = 0; l < 5; ++l) Xi[v][l] = a.X[(int64_t)(v * 5 + l) * nt + i];
        }
        const bool cv = a.charvars != 0;
        CharBasis cb;
        if (cv) cb.init(Wi, Xi[0][0], Xi[0][1], a.gamma);
        double cand[4][4], out[4];
        // second derivatives: own and the neighbours' (limited in place)
        if (ki == 2) {
#pragma unroll
            for (int l = 0; l < 3; ++l) {
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    cand[0][v] = Xi[v][2 + l] * ihi * ihi;
#pragma unroll
                    for (int s = 0; s < 3; ++s) {
                        cand[s + 1][v] = 0.0;
                        if (!ok[s + 1]) continue;
                        const double ihj = a.cgeo[nb[s]];
                        cand[s + 1][v] = a.X[(int64_t)(v * 5 + 2 + l) * nt + nb[s]] * (ihj * ihj);
                    }
                }
                limit_vec(cand, w, ok, cv, cb, out);
#pragma unroll
                for (int v = 0; v < 4; ++v) Xi[v][2 + l] = out[v] * hi * hi;
            }
        }
        // first derivatives from remainder averages: with three neighbours
        // the plane through each neighbour pair (weighing the pair's mean
        // weight); in a wall cell the gradient along each neighbour's
        // direction alone
        double rem[3][4];
#pragma unroll
        for (int s = 0; s < 3; ++s) {
#pragma unroll
            for (int v = 0; v < 4; ++v) rem[s][v] = 0.0;
            if (!ok[s + 1]) continue;
            const int64_t b = (int64_t)s * 5;
            const double a3 = a.a0c[(b + 2) * nt + i], a4 = a.a0c[(b + 3) * nt + i], a5 = a.a0c[(b + 4) * nt + i];
#pragma unroll
            for (int v = 0; v < 4; ++v)
                rem[s][v] = (a.W[(int64_t)v * nt + nb[s]] - Wi[v]) - (Xi[v][2] * a3 + Xi[v][3] * a4 + Xi[v][4] * a5);
        }
        const bool pairs = J == 3;
        double w1[4];
        w1[0] = w[0];
#pragma unroll
        for (int s = 0; s < 3; ++s) w1[s + 1] = pairs ? 0.5 * (w[s + 1] + w[(s + 1) % 3 + 1]) : w[s + 1];
#pragma unroll
        for (int l = 0; l < 2; ++l) {
#pragma unroll
            for (int s = 0; s < 3; ++s) {
#pragma unroll
                for (int v = 0; v < 4; ++v) cand[s + 1][v] = 0.0;
                if (!ok[s + 1]) continue;
                if (!pairs) {
                    const double dd = dc[s][0] * dc[s][0] + dc[s][1] * dc[s][1];
#pragma unroll
                    for (int v = 0; v < 4; ++v) cand[s + 1][v] = rem[s][v] * dc[s][l] / dd * ihi;
                    continue;
                }
                const int m2 = (s + 1) % 3;
                const double a11 = dc[s][0], a12 = dc[s][1], a21 = dc[m2][0], a22 = dc[m2][1];
                const double det = a11 * a22 - a12 * a21;
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    double gcomp;
                    if (fabs(det) < 1e-12)
                        gcomp = Xi[v][l];
                    else if (l == 0)
                        gcomp = (a22 * rem[s][v] - a12 * rem[m2][v]) / det;
                    else
                        gcomp = (a11 * rem[m2][v] - a21 * rem[s][v]) / det;
                    cand[s + 1][v] = gcomp * ihi;
                }
            }
#pragma unroll
            for (int v = 0; v < 4; ++v) cand[0][v] = Xi[v][l] * ihi;
            limit_vec(cand, w1, ok, cv, cb, out);
#pragma unroll
            for (int v = 0; v < 4; ++v) Xi[v][l] = out[v] * hi;
        }
#pragma unroll
        for (int v = 0; v < 4; ++v)
#pragma unroll
            for (int l = 0; l < 5; ++l) a.lbuf[(int64_t)(v * 5 + l) * a.lstride + k] = Xi[v][l];
    }
}

// Limited coefficients of the listed cells into their places in dst.
__global__ void __launch_bounds__(TPB) k_limit_scatter(LimArgs a) {
    const int cnt = min(*a.count, a.cap);
    const int nt = a.nt;
    for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < cnt; k += gridDim.x * blockDim.x) {
        const int i = a.list[k];
#pragma unroll
        for (int l = 0; l < 20; ++l) a.dst[(int64_t)l * nt + i] = a.lbuf[(int64_t)l * a.lstride + k];
    }
}

static inline void check_launch(int kc) {
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) throw LaunchError{e, kc_names[kc]};
}

#define PROFB(kc, bytes, ...)        \
    do {                             \
        prof_begin(m, kc, bytes);    \
        __VA_ARGS__;                 \
        check_launch(kc);            \
        prof_end(m, kc);             \
    } while (0)
#define PROF(kc, ...) PROFB(kc, 0.0, __VA_ARGS__)



void launch_rhs(gks_mesh* m, const double* W, double* sq_out) {
    const int nt = m->d.nt;
    const int nb = nblocks(nt);
    double* part = sq_out ? m->w.npart : nullptr;
    PROFB(KC_RHS, nt * (3 * (4.0 + 40.0) + 4.0 + 4 * 8.0 * 4 + VB), hipLaunchKernelGGL(k_rhs, dim3(nb), dim3(TPB), 0, m->stream, nt, m->d.iperm, m->d.nbc,
                                    m->d.a0c, W, m->w.R, part));
    if (sq_out)
        PROF(KC_FINAL, hipLaunchKernelGGL(k_sum_partials, dim3(NC), dim3(TPB), 0, m->stream, NC, nb, part, nullptr, sq_out,
                                          nullptr));
}

void launch_spmv64(gks_mesh* m, const double* x, const double* xscale, double* y, const int32_t* gate) {
    const int n = m->d.n;
    PROFB(KC_SPMV, spmv_bytes(n, 8, false), hipLaunchKernelGGL((k_spmv<double, double, false>), dim3(nblocks(n)), dim3(TPB), 0, m->stream, n, m->d.np,
                                         m->d.Kval, m->d.Kcol, m->d.worder, x, xscale, nullptr, y, gate));
}

void launch_spmv64_f32x(gks_mesh* m, const float* x, double* y, const int32_t* gate) {
    const int n = m->d.n;
    PROFB(KC_SPMV, n * (KW * 25.0 * 8 + KW * 4.0 + VB / 2 + VB), hipLaunchKernelGGL((k_spmv<double, float, false>), dim3(nblocks(n)), dim3(TPB), 0, m->stream, n, m->d.np,
                                         m->d.Kval, m->d.Kcol, m->d.worder, x, nullptr, nullptr, y, gate));
}

// y = K x with the products V_j . y (j < nvd <= RED_CHUNK) reduced to
// out[j * NC + c] * scale[j * NC + c]
template <typename XT>
static void spmv_dots(gks_mesh* m, const XT* x, double* y, const double* V, int64_t vstride, int nvd,
                      const double* scale, double* out, const int32_t* gate) {
    const int n = m->d.n;
    const int nb = nblocks(n);
    const double by = n * (KW * 25.0 * 8 + KW * 4.0 + (double)sizeof(XT) * CB + VB + nvd * VB);
    PROFB(KC_SPMV, by, hipLaunchKernelGGL(k_spmv_dots<XT>, dim3(nb), dim3(TPB), 0, m->stream, n, m->d.np, m->d.Kval,
                                          m->d.Kcol, m->d.worder, x, y, V, vstride, nvd, m->w.dpart, gate));
    PROF(KC_FINAL, hipLaunchKernelGGL(k_sum_partials, dim3(nvd * NC), dim3(TPB), 0, m->stream, nvd * NC, nb, m->w.dpart,
                                      scale, out, gate));
}

void launch_spmv64_dots(gks_mesh* m, const double* x, double* y, const double* V, int64_t vstride, int nvd,
                        const double* scale, double* out, const int32_t* gate) {
    spmv_dots<double>(m, x, y, V, vstride, nvd, scale, out, gate);
}

void launch_spmv64_f32x_dots(gks_mesh* m, const float* x, double* y, const double* V, int64_t vstride, int nvd,
                             const double* scale, double* out, const int32_t* gate) {
    spmv_dots<float>(m, x, y, V, vstride, nvd, scale, out, gate);
}

void launch_axpy_dots(gks_mesh* m, const double* V, int64_t vstride, int nvec, const double* h, const double* scale,
                      const double* w, double* out, double* dots_out, const int32_t* gate, double* sq_out) {
    const int n = m->d.n;
    // a multiple of 5 blocks of 256 threads: the grid is a multiple of 10 threads
    const int nb = axpy_dots_blocks(n);
    double* part = sq_out ? m->w.npart : nullptr;
    PROFB(KC_AXPY_DOTS, (double)n * (nvec + 2) * VB, hipLaunchKernelGGL(k_axpy_dots, dim3(nb), dim3(TPB), 0, m->stream, n, V, vstride,
                                                                   nvec, h, scale, w, out, m->w.dpart, gate, part));
    PROF(KC_FINAL, hipLaunchKernelGGL(k_sum_partials, dim3(nvec * NC), dim3(TPB), 0, m->stream, nvec * NC, nb, m->w.dpart,
                                      scale, dots_out, gate));
    if (sq_out)
        PROF(KC_FINAL, hipLaunchKernelGGL(k_sum_partials, dim3(NC), dim3(TPB), 0, m->stream, NC, nb, part, nullptr, sq_out,
                                          gate));
}

void launch_resid(gks_mesh* m, const double* x, const double* b, double* y, const int32_t* gate, double* sq_out) {
    const int n = m->d.n;
    const int nb = nblocks(n);
    double* part = sq_out ? m->w.npart : nullptr;
    PROFB(KC_SPMV_RES, spmv_bytes(n, 8, true), hipLaunchKernelGGL((k_spmv<double, double, true>), dim3(nb), dim3(TPB), 0, m->stream, n, m->d.np,
                                         m->d.Kval, m->d.Kcol, m->d.worder, x, nullptr, b, y, gate, part));
    if (sq_out)
        PROF(KC_FINAL, hipLaunchKernelGGL(k_sum_partials, dim3(NC), dim3(TPB), 0, m->stream, NC, nb, part, nullptr, sq_out,
                                          gate));
}

// The mixed form's inner iteration z = P(s .* v): q (default inner_iters) BILU(0)-
// preconditioned Richardson sweeps in FP32, in the split form when the
// handle has it (see k_es_fwd/k_es_bwd), else the general fused sweeps
// (k_mx_fwd/k_mx_bwd).  Bytes: stored blocks (100 B FP32, 4 B index) of each
// level plus per row its own vectors (80 B FP32, 160 B FP64 v).
// Block size of a level's sweep launch: TPB threads once the level has rows
// for two such blocks per CU, else one-wave blocks, so that the waves of a
// small level spread over every CU (the sweeps have no block-wide
// reductions; their LDS areas are per wave).
static inline int sweep_tpb(int64_t rows) { return rows >= 2 * 256 * (int64_t)TPB ? TPB : 64; }

static void mx_sweeps_general(gks_mesh* m, const double* v, const double* vscale, float* z, const int32_t* gate, int q) {
    using ACC = double;
    const DevMesh& D = m->d;
    float* b = m->w.bf;
    float* y = m->w.yf;
    float* d = m->w.df;
    const auto& lp = D.lev_ptr;
    const int nl = (int)lp.size() - 1;
    const double VF = VB / 2;
    for (int sw = 0; sw < q; ++sw) {
        const bool first = sw == 0;
        for (int l = 0; l < nl; ++l) {
            const int r0 = lp[l], r1 = lp[l + 1];
            if (r1 <= r0) continue;
            const int rows = r1 - r0;
            const double lb = D.lev_Lb[l] * 104.0;
            if (first)
                PROFB(KC_ILU_FWD32, lb + rows * (VB + 2 * VF),
                      hipLaunchKernelGGL((k_mx_fwd<true, ACC>), dim3(nblocks(rows, sweep_tpb(rows))), dim3(sweep_tpb(rows)), 0, m->stream, D.n, D.np,
                                         r0, r1, D.Lsbase[l], D.Kval32, D.Kcol, D.Li, D.Lval32, v, vscale, b, z, y, gate));
            else
                PROFB(KC_ILU_FWD32, lb + D.lev_Kb[l] * 104.0 + rows * 3 * VF,
                      hipLaunchKernelGGL((k_mx_fwd<false, ACC>), dim3(nblocks(rows, sweep_tpb(rows))), dim3(sweep_tpb(rows)), 0, m->stream, D.n, D.np,
                                         r0, r1, D.Lsbase[l], D.Kval32, D.Kcol, D.Li, D.Lval32, v, vscale, b, z, y, gate));
        }
        for (int l = nl - 1; l >= 0; --l) {
            const int r0 = lp[l], r1 = lp[l + 1];
            if (r1 <= r0) continue;
            const int rows = r1 - r0;
            const double ub = D.lev_Ub[l] * 104.0;
            if (first)
                PROFB(KC_ILU_BWD32, ub + rows * (100.0 + 2 * VF),
                      hipLaunchKernelGGL((k_mx_bwd<true, ACC>), dim3(nblocks(rows, sweep_tpb(rows))), dim3(sweep_tpb(rows)), 0, m->stream, D.np, r0,
                                         r1, D.Usbase[l], D.Ui, D.Uval32, D.Dinv32, y, d, z, gate));
            else
                PROFB(KC_ILU_BWD32, ub + rows * (100.0 + 4 * VF),
                      hipLaunchKernelGGL((k_mx_bwd<false, ACC>), dim3(nblocks(rows, sweep_tpb(rows))), dim3(sweep_tpb(rows)), 0, m->stream, D.np, r0,
                                         r1, D.Usbase[l], D.Ui, D.Uval32, D.Dinv32, y, d, z, gate));
        }
    }
}

static void mx_sweeps_split(gks_mesh* m, const double* v, const double* vscale, float* z, const int32_t* gate, int q) {
    using ACC = double;
    const DevMesh& D = m->d;
    float* b = m->w.bf;
    float* w = m->w.yf;
    float* t = m->w.df;
    const auto& lp = D.lev_ptr;
    const int nl = (int)lp.size() - 1;
    const double VF = VB / 2;
    auto fwd = [&](int l, bool first) {
        const int r0 = lp[l], r1 = lp[l + 1];
        if (r1 <= r0) return;
        const int rows = r1 - r0;
        const bool last = l == nl - 1;
        // blocks: Dinv K_L, and Dinv (first sweep) or Dinv E; vectors: v read
        // and b' written (first) or b', z read; then w written (z on the last
        // level); w_prev read and t written on the middle levels
        // (the first sweep's level 0 writes b' alone: its w is b')
        const bool wout = last || !(first && l == 0);
        const double by = D.lev_Lb[l] * 104.0 + rows * (100.0 + (first ? VB + VF : 2 * VF) + (wout ? VF : 0.0)) +
                          rows * VF * (!first && !last ? 2 : 0);
        const int tb = sweep_tpb(rows);
        const dim3 g(nblocks(rows, tb)), bl(tb);
        if (first && last)
            PROFB(KC_ILU_FWD32, by, hipLaunchKernelGGL((k_es_fwd<true, true, ACC>), g, bl, 0, m->stream, D.np, r0, r1,
                                                     D.Lsbase[l], lp[1], D.Li, D.Lval32, D.E32, D.Dinv32, v, vscale, b, t, w, z, gate));
        else if (first)
            PROFB(KC_ILU_FWD32, by, hipLaunchKernelGGL((k_es_fwd<true, false, ACC>), g, bl, 0, m->stream, D.np, r0, r1,
                                                     D.Lsbase[l], lp[1], D.Li, D.Lval32, D.E32, D.Dinv32, v, vscale, b, t, w, z, gate));
        else if (last)
            PROFB(KC_ILU_FWD32, by, hipLaunchKernelGGL((k_es_fwd<false, true, ACC>), g, bl, 0, m->stream, D.np, r0, r1,
                                                     D.Lsbase[l], lp[1], D.Li, D.Lval32, D.E32, D.Dinv32, v, vscale, b, t, w, z, gate));
        else
            PROFB(KC_ILU_FWD32, by, hipLaunchKernelGGL((k_es_fwd<false, false, ACC>), g, bl, 0, m->stream, D.np, r0, r1,
                                                     D.Lsbase[l], lp[1], D.Li, D.Lval32, D.E32, D.Dinv32, v, vscale, b, t, w, z, gate));
    };
    auto bwd = [&](int l) {
        const int r0 = lp[l], r1 = lp[l + 1];
        if (r1 <= r0) return;
        const int rows = r1 - r0;
        // blocks: Dinv K_U; vectors: w read, z written
        const double by = D.lev_Ub[l] * 104.0 + rows * 2 * VF;
        const int tb = sweep_tpb(rows);
        const dim3 g(nblocks(rows, tb)), bl(tb);
        PROFB(KC_ILU_BWD32, by, hipLaunchKernelGGL((k_es_bwd<ACC>), g, bl, 0, m->stream, r0, r1, D.Usbase[l], D.Ui,
                                                 D.Uval32, l == 0 ? b : w, z, gate));
    };
    for (int sw = 0; sw < q; ++sw) {
        const bool first = sw == 0;
        // Level 0's forward pass of a later sweep changes nothing: its rows
        // have no lower neighbours, so E = D - K_D = 0 there, w stays b' and
        // t = w - w_prev + z is z, which the next levels gather directly.
        for (int l = (first || nl < 2) ? 0 : 1; l < nl; ++l) fwd(l, first);
        for (int l = nl - 2; l >= 0; --l) bwd(l);
    }
}

static void mx_sweeps(gks_mesh* m, const double* v, const double* vscale, float* z, const int32_t* gate, int q) {
    if (m->d.split)
        mx_sweeps_split(m, v, vscale, z, gate, q);
    else
        mx_sweeps_general(m, v, vscale, z, gate, q);
}

// Inner GMRES of the mixed form (inner_solver = GKS_INNER_GMRES): z
// approximately solves K z = s .* v by inner_iters steps of GMRES from z = 0,
// right-preconditioned by one FP32 BILU(0) application (the first of the
// split-form or general sweeps), with the FP64 matrix and an FP64 Arnoldi
// process (classical Gram-Schmidt with the selective second pass), its own
// basis U, preconditioned basis T (FP32) and Krylov state.  s .* v has unit
// norm (an outer basis vector), so the inner residual starts at 1.  No host
// read: the step count is fixed, and a breakdown (an exact inner solution)
// stops the inner control step from advancing.  z = sum_j y_j t_j in FP32.
static void launch_inner_gmres(gks_mesh* m, const double* v, const double* vscale, float* z, const int32_t* gate) {
    Work& w = m->w;
    KrylovState* ki = w.ks_in;
    const int mi = m->prm.inner_iters;
    const int n = m->d.n;
    const int64_t vs = (int64_t)(n + 1) * CB;
    PROFB(KC_MISC, 2.0 * vs * sizeof(double), hipLaunchKernelGGL(k_copy, dim3(nblocks(vs)), dim3(TPB), 0, m->stream, vs, w.U, v));
    PROF(KC_MISC, hipLaunchKernelGGL(k_inner_init, dim3(1), dim3(64), 0, m->stream, ki, vscale, gate));
    for (int j = 0; j < mi; ++j) {
        const double* uj = w.U + (int64_t)j * vs;
        double* uj1 = w.U + (int64_t)(j + 1) * vs;
        float* tj = w.T + (int64_t)j * vs;
        mx_sweeps(m, uj, &ki->scale[j][0], tj, gate, 1);
        launch_spmv64_f32x_dots(m, tj, w.w, w.U, vs, j + 1, &ki->scale[0][0], &ki->h1[0][0], gate);
        launch_axpy_dots(m, w.U, vs, j + 1, &ki->h1[0][0], &ki->scale[0][0], w.w, uj1, &ki->h2[0][0], gate, ki->sq);
        launch_ctl_ks(m, ki, 4, mi);
        launch_axpy(m, w.U, vs, j + 1, &ki->h2[0][0], &ki->scale[0][0], uj1, uj1, &ki->reorth, ki->sq, true);
        launch_ctl_ks(m, ki, 2, mi);
    }
    launch_ctl_ks(m, ki, 3, mi);
    const dim3 g(nblocks((int64_t)n * Grp<float>::T)), b(TPB);
    PROFB(KC_COMBINE, (double)n * (mi * VB / 2 + VB / 2),
          hipLaunchKernelGGL((k_combine_f32out), g, b, 0, m->stream, n, w.T, vs, mi, &ki->y[0][0], w.ones, z, &ki->st.k, gate));
}

void launch_mx_precond(gks_mesh* m, const double* v, const double* vscale, float* z, const int32_t* gate, int q) {
    if (m->prm.inner_solver == GKS_INNER_GMRES)
        launch_inner_gmres(m, v, vscale, z, gate);
    else
        mx_sweeps(m, v, vscale, z, gate, q > 0 ? q : m->prm.inner_iters);
}

int outer_step_sweeps(const gks_mesh* m, int k) {
    return k == 0 ? m->sw.q1 : m->prm.inner_iters;
}

// FP64 BILU(0) solve out = M^-1 (s .* in), level by level.  Bytes: stored
// blocks (200 B, 4 B index) plus per row in/out vectors (and Dinv).
void launch_ilu(gks_mesh* m, const double* in, const double* in_scale, double* tmp, double* out, const int32_t* gate) {
    const DevMesh& D = m->d;
    const auto& lp = D.lev_ptr;
    const int nl = (int)lp.size() - 1;
    // level 0 (no lower neighbours: y = s .* v) has no forward launch
    // when later levels read it from v
    const int l0 = nl >= 2 ? 1 : 0;
    const int zrows = l0 ? lp[1] : 0;
    // the last level's forward pass also applies its pivot inverse (no upper
    // neighbours), so its backward pass has no launch
    for (int l = l0; l < nl; ++l) {
        const int r0 = lp[l], r1 = lp[l + 1];
        if (r1 <= r0) continue;
        const dim3 g(nblocks(r1 - r0, sweep_tpb(r1 - r0))), b(sweep_tpb(r1 - r0));
        if (l == nl - 1)
            PROFB(KC_ILU_FWD, D.lev_Lb[l] * 204.0 + (r1 - r0) * (200.0 + 2.0 * VB),
                  hipLaunchKernelGGL(k_ilu_fwd<true>, g, b, 0, m->stream, D.np, r0, r1, D.Lsbase[l], zrows, D.Li, D.Lval,
                                     D.Dinv, in, in_scale, tmp, out, gate));
        else
            PROFB(KC_ILU_FWD, D.lev_Lb[l] * 204.0 + (r1 - r0) * 2.0 * VB,
                  hipLaunchKernelGGL(k_ilu_fwd<false>, g, b, 0, m->stream, D.np, r0, r1, D.Lsbase[l], zrows, D.Li, D.Lval,
                                     D.Dinv, in, in_scale, tmp, out, gate));
    }
    for (int l = nl - 2; l >= 0; --l) {
        const int r0 = lp[l], r1 = lp[l + 1];
        if (r1 <= r0) continue;
        const bool from_v = l == 0 && l0 == 1;
        PROFB(KC_ILU_BWD, D.lev_Ub[l] * 204.0 + (r1 - r0) * (200.0 + 2.0 * VB),
              hipLaunchKernelGGL(k_ilu_bwd, dim3(nblocks(r1 - r0, sweep_tpb(r1 - r0))), dim3(sweep_tpb(r1 - r0)), 0, m->stream, D.np, r0, r1, D.Usbase[l],
                                 D.Ui, D.Uval, D.Dinv, from_v ? in : tmp, from_v ? in_scale : nullptr, out, gate));
    }
}

// partial sums of V_j . w for j < nvec into m->w.partial, then reduce
// (times scale_j when scale != NULL) into out[j * NC + c].
void launch_dots_reduce(gks_mesh* m, int kc, const double* V, int64_t vstride, int nvec, const double* w,
                        const double* scale, double* out, const int32_t* gate) {
    const int n = m->d.n;
    const int nb = m->w.nblk_red;
    const int nch = (nvec + RED_CHUNK - 1) / RED_CHUNK;
    PROFB(kc, (double)n * (nvec + 1) * VB, hipLaunchKernelGGL(k_dots, dim3(nb, nch), dim3(TPB), 0, m->stream, n, V, vstride, nvec, w,
                                m->w.partial, gate));
    const int nval = nvec * NC;
    PROF(KC_FINAL, hipLaunchKernelGGL(k_sum_partials, dim3(nval), dim3(TPB), 0, m->stream, nval, nb,
                                      m->w.partial, scale, out, gate));
}

void launch_axpy(gks_mesh* m, const double* V, int64_t vstride, int nvec, const double* h, const double* scale,
                 const double* w, double* out, const int32_t* gate, double* sq_out, bool second_pass) {
    const int n = m->d.n;
    const int nb = std::min(AXPY_BLOCKS, nblocks((int64_t)n * 10));   // grid-stride beyond
    double* part = sq_out ? m->w.npart : nullptr;
    // The second Gram-Schmidt pass is gated on the device (ks->reorth), so
    // whether it moves its bytes is unknown here: its own class, no bytes.
    PROFB(second_pass ? KC_REORTH : KC_AXPY_DOTS, second_pass ? 0.0 : (double)n * (nvec + 2) * VB,
          hipLaunchKernelGGL(k_axpy, dim3(nb), dim3(TPB), 0, m->stream, n, V, vstride, nvec, h, scale, w, out, gate, part));
    if (sq_out)
        PROF(KC_FINAL, hipLaunchKernelGGL(k_sum_partials, dim3(NC), dim3(TPB), 0, m->stream, NC, nb, part, nullptr, sq_out,
                                          gate));
}

void launch_combine(gks_mesh* m, const double* V, int64_t vstride, int nvec, const double* y, const double* scale,
                    double* out, const int32_t* nvec_dev, const int32_t* gate) {
    const int n = m->d.n;
    PROFB(KC_COMBINE, (double)n * (nvec + 1) * VB, hipLaunchKernelGGL(k_combine<double>, dim3(nblocks((int64_t)n * Grp<double>::T)), dim3(TPB), 0, m->stream, n, V, vstride, nvec,
                                        y, scale, out, nvec_dev, gate));
}

void launch_combine_f32(gks_mesh* m, const float* V, int64_t vstride, int nvec, const double* y, const double* scale,
                        double* out, const int32_t* nvec_dev, const int32_t* gate, bool accum) {
    const int n = m->d.n;
    const dim3 g(nblocks((int64_t)n * Grp<float>::T)), b(TPB);
    // bytes: the FP32 basis vectors read, out written (and read when accumulating)
    const double by = (double)n * (nvec * VB / 2 + (accum ? 2 : 1) * VB);
    if (accum)
        PROFB(KC_COMBINE, by, hipLaunchKernelGGL((k_combine<float, true>), g, b, 0, m->stream, n, V, vstride, nvec, y,
                                                 scale, out, nvec_dev, gate));
    else
        PROFB(KC_COMBINE, by, hipLaunchKernelGGL((k_combine<float, false>), g, b, 0, m->stream, n, V, vstride, nvec, y,
                                                 scale, out, nvec_dev, gate));
}

void launch_acc(gks_mesh* m, double* X, const double* z, const int32_t* gate) {
    const int64_t len = (int64_t)m->d.n * CB;
    PROFB(KC_AXPY, (double)len * 24.0, hipLaunchKernelGGL(k_acc, dim3(nblocks(len)), dim3(TPB), 0, m->stream, len, X, z, gate));
}

void launch_ctl_ks(gks_mesh* m, KrylovState* ks, int mode, int mres) {
    PROF(KC_MISC, hipLaunchKernelGGL(k_gmres_ctl, dim3(1), dim3(64), 0, m->stream, mode, ks, mres, 0));
}

void launch_ctl(gks_mesh* m, int mode, bool gated) {
    PROF(KC_MISC, hipLaunchKernelGGL(k_gmres_ctl, dim3(1), dim3(64), 0, m->stream, mode, m->w.ks, m->prm.restart,
                                     gated ? 1 : 0));
}

void launch_mask_cols(gks_mesh* m, double* X) {
    const int n = m->d.n;
    PROF(KC_MISC, hipLaunchKernelGGL(k_mask_cols, dim3(nblocks(n)), dim3(TPB), 0, m->stream, n, X, m->w.ks));
}

void launch_copyout(gks_mesh* m, const double* Xs, double* Xcell) {
    const int nt = m->d.nt;
    PROFB(KC_COPYOUT, (double)nt * (4.0 + 2 * VB), hipLaunchKernelGGL(k_copyout<double>, dim3(nblocks(nt)), dim3(TPB), 0, m->stream, nt,
                                        m->d.iperm, Xs, Xcell));
}

void launch_copyout_f32(gks_mesh* m, const float* Xs, double* Xcell) {
    const int nt = m->d.nt;
    PROF(KC_COPYOUT, hipLaunchKernelGGL(k_copyout<float>, dim3(nblocks(nt)), dim3(TPB), 0, m->stream, nt, m->d.iperm, Xs, Xcell));
}

// Arguments of the extrapolation for npts solutions; rotates the handle's
// ring (the slot receiving X becomes the newest).
static ExtrapArgs extrap_args(gks_mesh* m, int npts) {
    const int S = ring_slots(m->prm);
    ExtrapArgs a{};
    a.len = (int64_t)m->d.n * CB;
    // the solutions used must have their step sizes (a reconstruction
    // outside the step sequence clears them)
    int known = 0;
    while (known < S + 1 && m->dth[known] > 0.0) ++known;
    a.npts = std::max(1, std::min(std::min(std::min(npts, S + 1), m->pts.P), known));
    m->last_npts = a.npts;
    // Lagrange weights at time 0 of the solutions at tau_0 = -dth[0],
    // tau_i = tau_{i-1} - dth[i]
    double tau[MAXH + 1];
    double t = 0.0;
    for (int i = 0; i < a.npts; ++i) tau[i] = t -= m->dth[i];
    for (int i = 0; i < a.npts; ++i) {
        double w = 1.0;
        for (int j = 0; j < a.npts; ++j)
            if (j != i) w *= (0.0 - tau[j]) / (tau[i] - tau[j]);
        a.c[i] = w;
    }
    a.X = m->w.X;
    for (int i = 0; i < S; ++i) a.h[i] = m->w.H[(m->hring + i) % S];
    if (S > 0) {
        a.hout = m->w.H[(m->hring + S - 1) % S];
        m->hring = (m->hring + S - 1) % S;
    }
    return a;
}

void push_step(gks_mesh* m, double dt) {
    for (int i = MAXH; i > 0; --i) m->dth[i] = m->dth[i - 1];
    m->dth[0] = dt;
}

// algorithmic bytes: X read and written, the ring slots read, one written
static double extrap_bytes(const ExtrapArgs& a) {
    return (double)a.len * (16.0 + 8.0 * (a.npts - 1) + (a.hout ? 8.0 : 0.0));
}

void launch_extrap(gks_mesh* m, int npts) {
    const ExtrapArgs a = extrap_args(m, npts);
    PROFB(KC_EXTRAP, extrap_bytes(a), hipLaunchKernelGGL(k_extrap, dim3(nblocks(a.len)), dim3(TPB), 0, m->stream, a));
}

void launch_copyin(gks_mesh* m, const double* Xcell, double* Xs) {
    const int nt = m->d.nt;
    PROF(KC_MISC, hipLaunchKernelGGL(k_copyin, dim3(nblocks(nt)), dim3(TPB), 0, m->stream, nt, m->d.iperm, Xcell, Xs));
}

void launch_flux(gks_mesh* m, const double* W, const double* X, const double* dt_dev, double* F) {
    FluxArgs a;
    a.nf = m->d.nf;
    a.nt = m->d.nt;
    a.own = m->d.own;
    a.nbr = m->d.nbr;
    a.fgeo = m->d.fgeo;
    a.gpd = m->d.gpd;
    a.cgeo = m->d.cgeo;
    a.bc_kind = m->d.bc_kind;
    a.bc_state = m->d.bc_state;
    a.W = W;
    a.X = X;
    a.dt = dt_dev;
    a.F = F;
    a.nonphys = m->w.counters;
    a.fp.gamma = m->prm.gamma;
    a.fp.K = 2.0 / (m->prm.gamma - 1.0) - 2.0;
    a.fp.mu = m->prm.mu;
    a.fp.eps = m->prm.tau_eps;
    a.fp.exact_time = m->prm.exact_time;
    a.fallback = m->prm.nonphys_fallback;
    const int64_t nthr = 2 * (int64_t)a.nf;
    PROFB(KC_FLUX, (double)a.nf * (2 * (32.0 + 160.0 + 32.0) + 8.0 + 24.0 + 64.0 + 32.0), hipLaunchKernelGGL(k_flux, dim3(nblocks(nthr, 128)), dim3(128), 0, m->stream, a));
}

void launch_update(gks_mesh* m, const double* W, const double* F, double* Wn) {
    const int nt = m->d.nt;
    PROFB(KC_UPDATE, (double)nt * (12.0 + 8.0 + 64.0 + 3 * 32.0), hipLaunchKernelGGL(k_update, dim3(nblocks(nt)), dim3(TPB), 0, m->stream, nt, m->d.nf,
                                       m->d.cface, m->d.area, W, F, Wn, m->prm.gamma, m->w.counters + 1));
}

static LimArgs limit_args(gks_mesh* m, const double* W, const double* X, double* Xcopy, double* dst,
                          double threshold, int variables, int32_t* count, int32_t* list, double* lbuf, int cap,
                          int lstride) {
    LimArgs a;
    a.nt = m->d.nt;
    a.nf = m->d.nf;
    a.own = m->d.own;
    a.nbr = m->d.nbr;
    a.cface = m->d.cface;
    a.nbc = m->d.nbc;
    a.a0c = m->d.a0c;
    a.gpd = m->d.gpd;
    a.cgeo = m->d.cgeo;
    a.W = W;
    a.X = X;
    a.Xcopy = Xcopy;
    a.gamma = m->prm.gamma;
    a.threshold = threshold;
    a.all_quadratic = m->prm.all_quadratic;
    a.charvars = variables == GKS_LIMIT_CHARACTERISTIC;
    a.count = count;
    a.list = list;
    a.lbuf = lbuf;
    a.dst = dst;
    a.cap = cap;
    a.lstride = lstride;
    return a;
}

void launch_limit(gks_mesh* m, const double* W, const double* X, double* Xcopy, double* dst, double threshold,
                  int variables, int32_t* count) {
    const LimArgs a = limit_args(m, W, X, Xcopy, dst, threshold, variables, count, m->w.lim_list, m->w.lim_buf,
                                 m->d.nt, m->d.nt);
    // unique bytes per cell (a neighbour's data is the same array element as
    // that cell's own): density average and its five coefficients, h and the
    // moments, neighbour slots and offsets; plus the copy of X if asked
    const double by = (double)a.nt * (8.0 + 40.0 + 32.0 + 12.0 + 48.0 + (Xcopy ? 320.0 : 0.0));
    PROFB(KC_LIMIT, by, hipLaunchKernelGGL(k_limit_mark, dim3(nblocks(a.nt)), dim3(TPB), 0, m->stream, a));
    // the limited cells are few and their work is arithmetic: a fixed grid
    // of one-wave blocks strides over the list
    const int nb = std::max(1, std::min(2048, nblocks(a.nt, 64)));
    PROF(KC_LIMIT_APPLY, hipLaunchKernelGGL(k_limit_apply, dim3(nb), dim3(64), 0, m->stream, a));
    PROF(KC_LIMIT_APPLY, hipLaunchKernelGGL(k_limit_scatter, dim3(std::min(256, nblocks(a.nt))), dim3(TPB), 0,
                                            m->stream, a));
}

__global__ void k_zero_i32(int count, int32_t* p) {
    if ((int)threadIdx.x < count) p[threadIdx.x] = 0;
}

// ------------------------------------------------------------------ static limiter scratch
// Work space of gks_limit_noalloc: the count of limited cells, their list and
// their limited coefficients, for at most GKS_LIMIT_NOALLOC_MAX_CELLS limited
// cells, in one array of the code object.  Each device holds its own copy
// from module load until the process ends; in host code the array's name is
// only a stand-in, so kernels receive the device address that
// hipGetSymbolAddress returns for the current device (scratch_device_ptr).
constexpr size_t SCR_COUNT = 0;                                                   // int32 count
constexpr size_t SCR_LIST = 256;                                                  // int32 [MAX]
constexpr size_t SCR_LBUF = SCR_LIST + ((size_t)GKS_LIMIT_NOALLOC_MAX_CELLS * 4 + 255) / 256 * 256;  // double [20][MAX]
constexpr size_t SCR_BYTES = SCR_LBUF + (size_t)20 * GKS_LIMIT_NOALLOC_MAX_CELLS * sizeof(double);
static_assert(SCR_BYTES == 10748160, "size of the static limiter scratch");

static __device__ __align__(256) unsigned char scratch[SCR_BYTES];

// Device address of `scratch` on the current device, looked up once per
// device (hipGetSymbolAddress with that device current) and kept; null when
// the lookup fails (err receives the reason).
void* scratch_device_ptr(std::string* err) {
    static std::mutex mu;
    static void* ptrs[64] = {nullptr};
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess || dev < 0 || dev >= 64) {
        if (err) *err = std::string("hipGetDevice: ") + hipGetErrorString(e);
        return nullptr;
    }
    std::lock_guard<std::mutex> lk(mu);
    if (!ptrs[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            if (err) *err = std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e);
            return nullptr;
        }
        ptrs[dev] = p;
    }
    return ptrs[dev];
}

// The limiter of launch_limit with its list, buffer and count in the static
// scratch at scr (the device address of `scratch`).  Phase 1 copies X to
// Xout, clears the count and marks the cells (entries past the scratch's
// limit are counted but not stored); phase 2, run only when the host has
// read a count within the limit, limits the listed cells and scatters them
// into Xout.  No profiling events (nothing is created or allocated).
void launch_limit_noalloc(gks_mesh* m, void* scr, int phase, const double* W, const double* X, double* Xout,
                          double threshold, int variables) {
    char* base = (char*)scr;
    int32_t* count = (int32_t*)(base + SCR_COUNT);
    const LimArgs a = limit_args(m, W, X, phase == 1 ? Xout : nullptr, Xout, threshold, variables, count,
                                 (int32_t*)(base + SCR_LIST), (double*)(base + SCR_LBUF),
                                 GKS_LIMIT_NOALLOC_MAX_CELLS, GKS_LIMIT_NOALLOC_MAX_CELLS);
    if (phase == 1) {
        hipLaunchKernelGGL(k_zero_i32, dim3(1), dim3(64), 0, m->stream, 1, count);
        check_launch(KC_MISC);
        hipLaunchKernelGGL(k_limit_mark, dim3(nblocks(a.nt)), dim3(TPB), 0, m->stream, a);
        check_launch(KC_LIMIT);
        return;
    }
    const int nb = std::max(1, std::min(2048, nblocks(std::min(a.nt, a.cap), 64)));
    hipLaunchKernelGGL(k_limit_apply, dim3(nb), dim3(64), 0, m->stream, a);
    check_launch(KC_LIMIT_APPLY);
    hipLaunchKernelGGL(k_limit_scatter, dim3(std::min(256, nblocks(std::min(a.nt, a.cap)))), dim3(TPB), 0,
                       m->stream, a);
    check_launch(KC_LIMIT_APPLY);
}

int32_t* scratch_count(void* scr) { return (int32_t*)((char*)scr + SCR_COUNT); }

void launch_cfl(gks_mesh* m, const double* W, double* dt_out) {
    const int nt = m->d.nt;
    const int nb = std::min(1024, nblocks(nt));
    PROF(KC_CFL, hipLaunchKernelGGL(k_cfl, dim3(nb), dim3(TPB), 0, m->stream, nt, m->d.nf, m->d.cface, m->d.area,
                                    m->d.fgeo, W, m->prm.gamma, m->w.dtpart));
    PROF(KC_CFL, hipLaunchKernelGGL(k_cfl_final, dim3(1), dim3(64), 0, m->stream, nb, m->w.dtpart, m->prm.cfl,
                                    dt_out));
}

void launch_set_scalar(gks_mesh* m, double* p, double v) {
    hipLaunchKernelGGL(k_set, dim3(1), dim3(1), 0, m->stream, p, v);
    check_launch(KC_MISC);
}

void launch_zero(gks_mesh* m, double* p, int64_t count) {
    if (count <= 0) return;
    hipLaunchKernelGGL(k_zero, dim3(nblocks(count)), dim3(TPB), 0, m->stream, count, p);
    check_launch(KC_MISC);
}

void launch_zero_i32(gks_mesh* m, int32_t* p, int count) {
    hipLaunchKernelGGL(k_zero_i32, dim3(1), dim3(64), 0, m->stream, count, p);
    check_launch(KC_MISC);
}

void launch_copy(gks_mesh* m, double* dst, const double* src, int64_t count) {
    if (count <= 0) return;
    hipLaunchKernelGGL(k_copy, dim3(nblocks(count)), dim3(TPB), 0, m->stream, count, dst, src);
    check_launch(KC_MISC);
}


// ================================================================== grouped launches
// The same kernels for several handles at once (gks_batch_step): one launch
// per kernel and level covers every handle of the group, each with the
// arguments and grid of its own launch (Group, GridV), so each handle's
// arithmetic is exactly that of its own launches.  Handles whose grid is
// empty for a launch are left out of it.

// Launch `kernel` over the items (arguments, own grid in blocks) in groups
// of at most MAXB, each item's first block on a multiple of NXCD.
template <class A, class K>
static void glaunch(hipStream_t st, K kernel, int tpb, const std::vector<std::pair<A, int>>& items, int kc,
                    dim3 extra = dim3(1, 1, 1)) {
    static_assert(sizeof(Group<A>) <= 4000, "grouped kernel arguments");
    size_t q = 0;
    while (q < items.size()) {
        Group<A> g;
        g.n = 0;
        int tot = 0;
        for (; q < items.size() && g.n < MAXB; ++q) {
            if (items[q].second <= 0) continue;
            g.start[g.n] = tot;
            g.nblk[g.n] = items[q].second;
            g.a[g.n] = items[q].first;
            tot += (items[q].second + NXCD - 1) / NXCD * NXCD;
            ++g.n;
        }
        if (g.n == 0) continue;
        g.start[g.n] = tot;
        hipLaunchKernelGGL(kernel, dim3(tot, extra.y, extra.z), dim3(tpb), 0, st, g);
        check_launch(kc);
    }
}

// Status words of the group's solves and the step counters, copied by the
// device into one pinned host array (read after one synchronisation).
struct StatArgs {
    const Status* st;
    const int32_t* counters;
    const double* dt;
    BatchSlot* out;
};
__global__ void __launch_bounds__(64) kg_gather(Group<StatArgs> g) {
    GridV v;
    const int r = group_locate(g, v);
    if (r < 0) return;
    const StatArgs& a = g.a[r];
    const int t = threadIdx.x;
    constexpr int NW = (int)(sizeof(Status) / sizeof(int32_t));
    static_assert(sizeof(Status) % sizeof(int32_t) == 0, "Status words");
    const int32_t* src = reinterpret_cast<const int32_t*>(a.st);
    int32_t* dst = reinterpret_cast<int32_t*>(&a.out->st);
    for (int k = t; k < NW; k += 64) dst[k] = src[k];
    if (a.counters && t < 4) a.out->counters[t] = a.counters[t];
    if (a.dt && t == 0) a.out->dt = *a.dt;
}

struct ZeroArgs {
    int32_t* p;
    int count;
    double* dt;      // when set, receives dtv
    double dtv;
};
__global__ void __launch_bounds__(64) kg_zero_set(Group<ZeroArgs> g) {
    GridV v;
    const int r = group_locate(g, v);
    if (r < 0) return;
    const ZeroArgs& a = g.a[r];
    if ((int)threadIdx.x < a.count) a.p[threadIdx.x] = 0;
    if (a.dt && threadIdx.x == 0) *a.dt = a.dtv;
}

void glaunch_gather(hipStream_t st, const std::vector<gks_mesh*>& ms, const std::vector<BatchSlot*>& out,
                    bool counters) {
    std::vector<std::pair<StatArgs, int>> it;
    for (size_t r = 0; r < ms.size(); ++r)
        it.push_back({StatArgs{&ms[r]->w.ks->st, counters ? ms[r]->w.counters : nullptr,
                               counters ? ms[r]->w.dt_dev : nullptr, out[r]}, 1});
    glaunch(st, kg_gather, 64, it, KC_MISC);
}

void glaunch_zero_counters(hipStream_t st, const std::vector<gks_mesh*>& ms, const std::vector<double>& dt) {
    std::vector<std::pair<ZeroArgs, int>> it;
    for (size_t r = 0; r < ms.size(); ++r)
        it.push_back({ZeroArgs{ms[r]->w.counters, 4, dt[r] > 0.0 ? ms[r]->w.dt_dev : nullptr, dt[r]}, 1});
    glaunch(st, kg_zero_set, 64, it, KC_MISC);
}

void glaunch_cfl(hipStream_t st, const std::vector<gks_mesh*>& ms, const std::vector<const double*>& W) {
    std::vector<std::pair<CflArgs, int>> a;
    std::vector<std::pair<CflFinalArgs, int>> b;
    for (size_t r = 0; r < ms.size(); ++r) {
        gks_mesh* m = ms[r];
        const int nt = m->d.nt;
        const int nb = std::min(1024, nblocks(nt));
        a.push_back({CflArgs{nt, m->d.nf, m->d.cface, m->d.area, m->d.fgeo, W[r], m->prm.gamma, m->w.dtpart}, nb});
        b.push_back({CflFinalArgs{nb, m->w.dtpart, m->prm.cfl, m->w.dt_dev}, 1});
    }
    glaunch(st, kg_cfl, TPB, a, KC_CFL);
    glaunch(st, kg_cfl_final, 64, b, KC_CFL);
}

void glaunch_extrap(hipStream_t st, const std::vector<gks_mesh*>& ms, const std::vector<int>& npts) {
    std::vector<std::pair<ExtrapArgs, int>> it;
    for (size_t r = 0; r < ms.size(); ++r) {
        const ExtrapArgs a = extrap_args(ms[r], npts[r]);
        it.push_back({a, nblocks(a.len)});
    }
    glaunch(st, kg_extrap, TPB, it, KC_EXTRAP);
}

// sum partials of nval values per handle (partial, nblk per handle) into out
static void gsum(hipStream_t st, const std::vector<SumArgs>& sa) {
    std::vector<std::pair<SumArgs, int>> it;
    for (const auto& a : sa) it.push_back({a, a.nval});
    glaunch(st, kg_sum_partials, TPB, it, KC_FINAL);
}

void glaunch_rhs(hipStream_t st, const std::vector<gks_mesh*>& ms, const std::vector<const double*>& W) {
    std::vector<std::pair<RhsArgs, int>> it;
    std::vector<SumArgs> sa;
    for (size_t r = 0; r < ms.size(); ++r) {
        gks_mesh* m = ms[r];
        const int nt = m->d.nt, nb = nblocks(nt);
        it.push_back({RhsArgs{nt, m->d.iperm, m->d.nbc, m->d.a0c, W[r], m->w.R, m->w.npart}, nb});
        sa.push_back(SumArgs{NC, nb, m->w.npart, nullptr, m->w.ks->sq, nullptr});
    }
    glaunch(st, kg_rhs, TPB, it, KC_RHS);
    gsum(st, sa);
}

void glaunch_ctl(hipStream_t st, const std::vector<gks_mesh*>& ms, int mode) {
    std::vector<std::pair<CtlArgs, int>> it;
    for (gks_mesh* m : ms) it.push_back({CtlArgs{mode, m->w.ks, m->prm.restart, 0}, 1});
    glaunch(st, kg_gmres_ctl, 64, it, KC_MISC);
}

void glaunch_mask_cols(hipStream_t st, const std::vector<gks_mesh*>& ms) {
    std::vector<std::pair<MaskArgs, int>> it;
    for (gks_mesh* m : ms) it.push_back({MaskArgs{m->d.n, m->w.X, m->w.ks}, nblocks(m->d.n)});
    glaunch(st, kg_mask_cols, TPB, it, KC_MISC);
}

// r = R - K X with its norms, then the start of a cycle (as cycle_start)
void glaunch_cycle_start(hipStream_t st, const std::vector<gks_mesh*>& ms) {
    std::vector<std::pair<SpmvArgs<double, double>, int>> it;
    std::vector<SumArgs> sa;
    for (gks_mesh* m : ms) {
        const int n = m->d.n, nb = nblocks(n);
        it.push_back({SpmvArgs<double, double>{n, m->d.np, m->d.Kval, m->d.Kcol, m->d.worder, m->w.X, nullptr, m->w.R,
                                               m->w.V, nullptr, m->w.npart},
                      nb});
        sa.push_back(SumArgs{NC, nb, m->w.npart, nullptr, m->w.ks->sq, nullptr});
    }
    glaunch(st, kg_spmv<double, double, true>, TPB, it, KC_SPMV_RES);
    gsum(st, sa);
    glaunch_ctl(st, ms, 1);
}

// FP64 BILU(0) solve out = M^-1 (s .* in) for every handle (as launch_ilu):
// level l of each handle in one launch per kernel variant
static void gilu(hipStream_t st, const std::vector<gks_mesh*>& ms, const std::vector<const double*>& in,
                 const std::vector<const double*>& in_scale, const std::vector<double*>& tmp,
                 const std::vector<double*>& out) {
    int maxl = 0;
    for (gks_mesh* m : ms) maxl = std::max(maxl, (int)m->d.lev_ptr.size() - 1);
    auto tpb_of = [&](const std::vector<int>& rows) {
        int tb = TPB;
        for (int r : rows) tb = std::min(tb, sweep_tpb(r));
        return tb;
    };
    for (int l = 0; l < maxl; ++l) {
        std::vector<std::pair<IluFwdArgs, int>> f[2];
        std::vector<int> rows[2];
        for (size_t r = 0; r < ms.size(); ++r) {
            const DevMesh& D = ms[r]->d;
            const auto& lp = D.lev_ptr;
            const int nl = (int)lp.size() - 1;
            const int l0 = nl >= 2 ? 1 : 0;
            if (l < l0 || l >= nl || lp[l + 1] <= lp[l]) continue;
            const int zrows = l0 ? lp[1] : 0;
            const int last = l == nl - 1;
            f[last].push_back({IluFwdArgs{D.np, lp[l], lp[l + 1], D.Lsbase[l], zrows, D.Li, D.Lval, D.Dinv, in[r],
                                          in_scale[r], tmp[r], out[r], nullptr},
                               lp[l + 1] - lp[l]});
            rows[last].push_back(lp[l + 1] - lp[l]);
        }
        for (int last = 0; last < 2; ++last) {
            if (f[last].empty()) continue;
            const int tb = tpb_of(rows[last]);
            for (auto& e : f[last]) e.second = nblocks(e.second, tb);
            if (last)
                glaunch(st, kg_ilu_fwd<true>, tb, f[last], KC_ILU_FWD);
            else
                glaunch(st, kg_ilu_fwd<false>, tb, f[last], KC_ILU_FWD);
        }
    }
    for (int l = maxl - 2; l >= 0; --l) {
        std::vector<std::pair<IluBwdArgs, int>> b;
        std::vector<int> rows;
        for (size_t r = 0; r < ms.size(); ++r) {
            const DevMesh& D = ms[r]->d;
            const auto& lp = D.lev_ptr;
            const int nl = (int)lp.size() - 1;
            if (l > nl - 2 || lp[l + 1] <= lp[l]) continue;
            const int l0 = nl >= 2 ? 1 : 0;
            const bool from_v = l == 0 && l0 == 1;
            b.push_back({IluBwdArgs{D.np, lp[l], lp[l + 1], D.Usbase[l], D.Ui, D.Uval, D.Dinv, from_v ? in[r] : tmp[r],
                                    from_v ? in_scale[r] : nullptr, out[r], nullptr},
                         lp[l + 1] - lp[l]});
            rows.push_back(lp[l + 1] - lp[l]);
        }
        if (b.empty()) continue;
        const int tb = tpb_of(rows);
        for (auto& e : b) e.second = nblocks(e.second, tb);
        glaunch(st, kg_ilu_bwd, tb, b, KC_ILU_BWD);
    }
}

// The mixed form's inner sweeps in the split form for every handle (as
// mx_sweeps_split): sweep sw and level l of each handle in one launch per
// kernel variant.
static void gmx_split(hipStream_t st, const std::vector<gks_mesh*>& ms, const std::vector<const double*>& v,
                      const std::vector<const double*>& vscale, const std::vector<float*>& z, int k) {
    using ACC = double;
    int maxl = 0, maxq = 0;
    std::vector<int> qh(ms.size());   // sweeps of each handle at Arnoldi step k
    for (size_t r = 0; r < ms.size(); ++r) {
        maxl = std::max(maxl, (int)ms[r]->d.lev_ptr.size() - 1);
        qh[r] = outer_step_sweeps(ms[r], k);
        maxq = std::max(maxq, qh[r]);
    }
    for (int sw = 0; sw < maxq; ++sw) {
        const bool first = sw == 0;
        for (int l = 0; l < maxl; ++l) {
            std::vector<std::pair<EsFwdArgs, int>> f[2];
            std::vector<int> rows[2];
            for (size_t r = 0; r < ms.size(); ++r) {
                gks_mesh* m = ms[r];
                const DevMesh& D = m->d;
                const auto& lp = D.lev_ptr;
                const int nl = (int)lp.size() - 1;
                if (sw >= qh[r] || l >= nl || lp[l + 1] <= lp[l]) continue;
                if (!(first || nl < 2) && l == 0) continue;   // no level-0 forward pass after the first sweep
                const int last = l == nl - 1;
                f[last].push_back({EsFwdArgs{D.np, lp[l], lp[l + 1], D.Lsbase[l], lp[1], D.Li, D.Lval32, D.E32,
                                             D.Dinv32, v[r], vscale[r], m->w.bf, m->w.df, m->w.yf, z[r], nullptr},
                                   lp[l + 1] - lp[l]});
                rows[last].push_back(lp[l + 1] - lp[l]);
            }
            for (int last = 0; last < 2; ++last) {
                if (f[last].empty()) continue;
                int tb = TPB;
                for (int rr : rows[last]) tb = std::min(tb, sweep_tpb(rr));
                for (auto& e : f[last]) e.second = nblocks(e.second, tb);
                if (first && last)
                    glaunch(st, kg_es_fwd<true, true, ACC>, tb, f[last], KC_ILU_FWD32);
                else if (first)
                    glaunch(st, kg_es_fwd<true, false, ACC>, tb, f[last], KC_ILU_FWD32);
                else if (last)
                    glaunch(st, kg_es_fwd<false, true, ACC>, tb, f[last], KC_ILU_FWD32);
                else
                    glaunch(st, kg_es_fwd<false, false, ACC>, tb, f[last], KC_ILU_FWD32);
            }
        }
        for (int l = maxl - 2; l >= 0; --l) {
            std::vector<std::pair<EsBwdArgs, int>> b;
            std::vector<int> rows;
            for (size_t r = 0; r < ms.size(); ++r) {
                gks_mesh* m = ms[r];
                const DevMesh& D = m->d;
                const auto& lp = D.lev_ptr;
                const int nl = (int)lp.size() - 1;
                if (sw >= qh[r] || l > nl - 2 || lp[l + 1] <= lp[l]) continue;
                b.push_back({EsBwdArgs{lp[l], lp[l + 1], D.Usbase[l], D.Ui, D.Uval32, l == 0 ? m->w.bf : m->w.yf, z[r],
                                       nullptr},
                             lp[l + 1] - lp[l]});
                rows.push_back(lp[l + 1] - lp[l]);
            }
            if (b.empty()) continue;
            int tb = TPB;
            for (int rr : rows) tb = std::min(tb, sweep_tpb(rr));
            for (auto& e : b) e.second = nblocks(e.second, tb);
            glaunch(st, kg_es_bwd<ACC>, tb, b, KC_ILU_BWD32);
        }
    }
}

// Arnoldi step k for every handle (as arnoldi_step without a gate)
void glaunch_arnoldi(hipStream_t st, const std::vector<gks_mesh*>& ms, int k) {
    const bool fused = k + 1 <= FUSED_DOTS_MAX;
    const bool mixed = ms[0]->prm.precision == GKS_MIXED;
    std::vector<const double*> vk, sk;
    std::vector<double*> t1, t2;
    std::vector<float*> zk;
    for (gks_mesh* m : ms) {
        const int64_t vs = (int64_t)(m->d.n + 1) * CB;
        vk.push_back(m->w.V + (int64_t)k * vs);
        sk.push_back(&m->w.ks->scale[k][0]);
        t1.push_back(m->w.t1);
        t2.push_back(m->w.t2);
        zk.push_back(mixed ? m->w.Z + (int64_t)k * vs : nullptr);
    }
    if (mixed)
        gmx_split(st, ms, vk, sk, zk, k);
    else
        gilu(st, ms, vk, sk, t1, t2);
    std::vector<SumArgs> sa;
    if (fused) {
        if (mixed) {
            std::vector<std::pair<SpmvDotsArgs<float>, int>> it;
            for (size_t r = 0; r < ms.size(); ++r) {
                gks_mesh* m = ms[r];
                const int n = m->d.n, nb = nblocks(n);
                const int64_t vs = (int64_t)(n + 1) * CB;
                it.push_back({SpmvDotsArgs<float>{n, m->d.np, m->d.Kval, m->d.Kcol, m->d.worder, zk[r], m->w.w, m->w.V,
                                                  vs, k + 1, m->w.dpart, nullptr},
                              nb});
                sa.push_back(SumArgs{(k + 1) * NC, nb, m->w.dpart, &m->w.ks->scale[0][0], &m->w.ks->h1[0][0], nullptr});
            }
            glaunch(st, kg_spmv_dots<float>, TPB, it, KC_SPMV);
        } else {
            std::vector<std::pair<SpmvDotsArgs<double>, int>> it;
            for (size_t r = 0; r < ms.size(); ++r) {
                gks_mesh* m = ms[r];
                const int n = m->d.n, nb = nblocks(n);
                const int64_t vs = (int64_t)(n + 1) * CB;
                it.push_back({SpmvDotsArgs<double>{n, m->d.np, m->d.Kval, m->d.Kcol, m->d.worder, m->w.t2, m->w.w,
                                                   m->w.V, vs, k + 1, m->w.dpart, nullptr},
                              nb});
                sa.push_back(SumArgs{(k + 1) * NC, nb, m->w.dpart, &m->w.ks->scale[0][0], &m->w.ks->h1[0][0], nullptr});
            }
            glaunch(st, kg_spmv_dots<double>, TPB, it, KC_SPMV);
        }
        gsum(st, sa);
        // w1 = w - V h1 into the basis slot k + 1, with the second products
        // and the norms of w1, then whether the second pass runs
        std::vector<std::pair<AxpyDotsArgs, int>> ad;
        sa.clear();
        for (gks_mesh* m : ms) {
            const int n = m->d.n;
            const int64_t vs = (int64_t)(n + 1) * CB;
            const int nb = axpy_dots_blocks(n);
            ad.push_back({AxpyDotsArgs{n, m->w.V, vs, k + 1, &m->w.ks->h1[0][0], &m->w.ks->scale[0][0], m->w.w,
                                       m->w.V + (int64_t)(k + 1) * vs, m->w.dpart, nullptr, m->w.npart},
                          nb});
            sa.push_back(SumArgs{(k + 1) * NC, nb, m->w.dpart, &m->w.ks->scale[0][0], &m->w.ks->h2[0][0], nullptr});
            sa.push_back(SumArgs{NC, nb, m->w.npart, nullptr, m->w.ks->sq, nullptr});
        }
        glaunch(st, kg_axpy_dots, TPB, ad, KC_AXPY_DOTS);
        gsum(st, sa);
    } else {
        // y = K M^-1 v_k
        if (mixed) {
            std::vector<std::pair<SpmvArgs<double, float>, int>> it;
            for (size_t r = 0; r < ms.size(); ++r) {
                gks_mesh* m = ms[r];
                it.push_back({SpmvArgs<double, float>{m->d.n, m->d.np, m->d.Kval, m->d.Kcol, m->d.worder, zk[r], nullptr,
                                                      nullptr, m->w.w, nullptr, nullptr},
                              nblocks(m->d.n)});
            }
            glaunch(st, kg_spmv<double, float, false>, TPB, it, KC_SPMV);
        } else {
            std::vector<std::pair<SpmvArgs<double, double>, int>> it;
            for (gks_mesh* m : ms)
                it.push_back({SpmvArgs<double, double>{m->d.n, m->d.np, m->d.Kval, m->d.Kcol, m->d.worder, m->w.t2,
                                                       nullptr, nullptr, m->w.w, nullptr, nullptr},
                              nblocks(m->d.n)});
            glaunch(st, kg_spmv<double, double, false>, TPB, it, KC_SPMV);
        }
        // h1 = V^T w, w1 = w - V h1 into slot k + 1 with its norms, h2 = V^T w1
        // (unfused passes, as launch_dots_reduce / launch_axpy)
        const int nch = (k + 1 + RED_CHUNK - 1) / RED_CHUNK;
        for (int pass = 0; pass < 2; ++pass) {
            std::vector<std::pair<DotsArgs, int>> dt;
            sa.clear();
            for (gks_mesh* m : ms) {
                const int64_t vs = (int64_t)(m->d.n + 1) * CB;
                const double* x = pass == 0 ? m->w.w : m->w.V + (int64_t)(k + 1) * vs;
                dt.push_back({DotsArgs{m->d.n, m->w.V, vs, k + 1, x, m->w.partial, nullptr}, m->w.nblk_red});
                sa.push_back(SumArgs{(k + 1) * NC, m->w.nblk_red, m->w.partial, &m->w.ks->scale[0][0],
                                     pass == 0 ? &m->w.ks->h1[0][0] : &m->w.ks->h2[0][0], nullptr});
            }
            glaunch(st, kg_dots, TPB, dt, KC_DOTS, dim3(1, nch, 1));
            gsum(st, sa);
            if (pass == 0) {
                std::vector<std::pair<AxpyArgs, int>> ax;
                sa.clear();
                for (gks_mesh* m : ms) {
                    const int n = m->d.n;
                    const int64_t vs = (int64_t)(n + 1) * CB;
                    const int nb = std::min(AXPY_BLOCKS, nblocks((int64_t)n * 10));
                    ax.push_back({AxpyArgs{n, m->w.V, vs, k + 1, &m->w.ks->h1[0][0], &m->w.ks->scale[0][0], m->w.w,
                                           m->w.V + (int64_t)(k + 1) * vs, nullptr, m->w.npart},
                                  nb});
                    sa.push_back(SumArgs{NC, nb, m->w.npart, nullptr, m->w.ks->sq, nullptr});
                }
                glaunch(st, kg_axpy, TPB, ax, KC_AXPY_DOTS);
                gsum(st, sa);
            }
        }
    }
    glaunch_ctl(st, ms, 4);
    // the second pass where ks->reorth asks for it: v_{k+1} = w1 - V h2
    // in place in slot k + 1 with its norm, then the control step
    std::vector<std::pair<AxpyArgs, int>> ax;
    sa.clear();
    for (gks_mesh* m : ms) {
        const int n = m->d.n;
        const int64_t vs = (int64_t)(n + 1) * CB;
        const int nb = std::min(AXPY_BLOCKS, nblocks((int64_t)n * 10));
        double* vk1 = m->w.V + (int64_t)(k + 1) * vs;
        ax.push_back({AxpyArgs{n, m->w.V, vs, k + 1, &m->w.ks->h2[0][0], &m->w.ks->scale[0][0], vk1,
                               vk1, &m->w.ks->reorth, m->w.npart},
                      nb});
        sa.push_back(SumArgs{NC, nb, m->w.npart, nullptr, m->w.ks->sq, &m->w.ks->reorth});
    }
    glaunch(st, kg_axpy, TPB, ax, KC_REORTH);
    gsum(st, sa);
    glaunch_ctl(st, ms, 2);
}

// End of a cycle of nvec[r] steps for every handle (as end_cycle without a
// graph): y from the triangular system, then X += Z y (mixed) or
// X += M^-1 (V y) (FP64).
void glaunch_end_cycle(hipStream_t st, const std::vector<gks_mesh*>& ms, const std::vector<int>& nvec) {
    glaunch_ctl(st, ms, 3);
    const bool mixed = ms[0]->prm.precision == GKS_MIXED;
    if (mixed) {
        std::vector<std::pair<CombineArgs<float>, int>> it;
        for (size_t r = 0; r < ms.size(); ++r) {
            gks_mesh* m = ms[r];
            const int n = m->d.n;
            const int64_t vs = (int64_t)(n + 1) * CB;
            it.push_back({CombineArgs<float>{n, m->w.Z, vs, nvec[r], &m->w.ks->y[0][0], m->w.ones, m->w.X, nullptr,
                                             nullptr},
                          nblocks((int64_t)n * Grp<float>::T)});
        }
        glaunch(st, kg_combine<float, true>, TPB, it, KC_COMBINE);
        return;
    }
    std::vector<std::pair<CombineArgs<double>, int>> it;
    std::vector<const double*> in, sc;
    std::vector<double*> tmp, out;
    for (size_t r = 0; r < ms.size(); ++r) {
        gks_mesh* m = ms[r];
        const int n = m->d.n;
        const int64_t vs = (int64_t)(n + 1) * CB;
        it.push_back({CombineArgs<double>{n, m->w.V, vs, nvec[r], &m->w.ks->y[0][0], &m->w.ks->scale[0][0], m->w.t1,
                                          nullptr, nullptr},
                      nblocks((int64_t)n * Grp<double>::T)});
        in.push_back(m->w.t1);
        sc.push_back(nullptr);
        tmp.push_back(m->w.t2);
        out.push_back(m->w.t3);
    }
    glaunch(st, kg_combine<double, false>, TPB, it, KC_COMBINE);
    gilu(st, ms, in, sc, tmp, out);
    std::vector<std::pair<AccArgs, int>> ac;
    for (gks_mesh* m : ms) {
        const int64_t len = (int64_t)m->d.n * CB;
        ac.push_back({AccArgs{len, m->w.X, m->w.t3, nullptr}, nblocks(len)});
    }
    glaunch(st, kg_acc, TPB, ac, KC_AXPY);
}

// Copy-out of X, fluxes and update for every handle (as the eager step)
void glaunch_flux_update(hipStream_t st, const std::vector<gks_mesh*>& ms, const std::vector<const double*>& W) {
    std::vector<std::pair<CopyoutArgs<double>, int>> co;
    std::vector<std::pair<FluxArgs, int>> fl;
    std::vector<std::pair<UpdateArgs, int>> up;
    for (size_t r = 0; r < ms.size(); ++r) {
        gks_mesh* m = ms[r];
        const int nt = m->d.nt;
        co.push_back({CopyoutArgs<double>{nt, m->d.iperm, m->w.X, m->w.Xcell}, nblocks(nt)});
        FluxArgs a;
        a.nf = m->d.nf;
        a.nt = nt;
        a.own = m->d.own;
        a.nbr = m->d.nbr;
        a.fgeo = m->d.fgeo;
        a.gpd = m->d.gpd;
        a.cgeo = m->d.cgeo;
        a.bc_kind = m->d.bc_kind;
        a.bc_state = m->d.bc_state;
        a.W = W[r];
        a.X = m->w.Xcell;
        a.dt = m->w.dt_dev;
        a.F = m->w.F;
        a.nonphys = m->w.counters;
        a.fp.gamma = m->prm.gamma;
        a.fp.K = 2.0 / (m->prm.gamma - 1.0) - 2.0;
        a.fp.mu = m->prm.mu;
        a.fp.eps = m->prm.tau_eps;
        a.fp.exact_time = m->prm.exact_time;
        a.fallback = m->prm.nonphys_fallback;
        fl.push_back({a, nblocks(2 * (int64_t)a.nf, 128)});
        up.push_back({UpdateArgs{nt, m->d.nf, m->d.cface, m->d.area, W[r], m->w.F, m->w.Wn, m->prm.gamma,
                                 m->w.counters + 1},
                      nblocks(nt)});
    }
    glaunch(st, kg_copyout<double>, TPB, co, KC_COPYOUT);
    glaunch(st, kg_flux, 128, fl, KC_FLUX);
    glaunch(st, kg_update, TPB, up, KC_UPDATE);
}

// W <- Wn for every handle
void glaunch_commit(hipStream_t st, const std::vector<gks_mesh*>& ms, const std::vector<double*>& W) {
    std::vector<std::pair<CopyArgs, int>> it;
    for (size_t r = 0; r < ms.size(); ++r) {
        const int64_t len = (int64_t)4 * ms[r]->d.nt;
        it.push_back({CopyArgs{len, W[r], ms[r]->w.Wn}, nblocks(len)});
    }
    glaunch(st, kg_copy, TPB, it, KC_MISC);
}

}  // namespace gks
