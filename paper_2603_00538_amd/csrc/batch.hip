// Many transfers at once: target/source pairs of mixed dimension and size,
// each with its own samples per element, run as one sequence of launches
// (sec. 4.1 steps 1-7 for every pair; the pairs are independent work units,
// sec. 4.1 last paragraph).  Built-in P1 sources in the binary64 or the
// binary32 form of the fused route.  A transfer of F fields runs as F
// systems, one per field, that share the transfer's target (mass matrix,
// incidence, samples) and write their own slice of its field buffers; the
// kernels below work on systems.
//
// Work lists built once at creation:
//   node tiles     (transfer, 256 / 128 target nodes) step 1, the control g
//   element tiles  (transfer, 64/G target elements)  steps 3-5, fused
//   row tiles      (transfer, 256 rows)              steps 2, 6, 7 and the report
// The node and element stages are persistent kernels: a grid sized to the
// device walks its list with a fixed stride.  Each element tile is one
// wavefront; its (dimension, form, lanes per element G, samples per lane P)
// variant is chosen per transfer (by default as the single-transfer route
// chooses G and P from N; ft_batch_autotune times the candidates), and
// every variant runs as a launch of its own (each with its own register
// budget, hence occupancy), the dearest variants (largest N, 3D) first.
//
// The solve is a batched Jacobi-PCG: all systems share the launches, every
// system keeps its own scalars, and a converged system's tiles return at once.
// Reductions have no atomics: each row tile writes its partial sums, and one
// wavefront per system adds its tiles' partials in tile order.  The number of
// iterations launched is fixed (max_iter), so the whole run contains no host
// synchronization and no memset and can be captured as one graph, replayed
// on every later call.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <numeric>
#include <set>
#include <string>
#include <vector>

#include "fused.h"

struct ft_batch;

namespace ft {

ft_status check_sample_cfg(const ft_target* T, const ft_sample_cfg* cfg);
ft_status ensure_field_buffers(ft_target* T, int F, hipStream_t stream);
SrcView source_view(const ft_source* S);

constexpr int BT = 256;   // threads per block; rows per row tile

struct BatchXfer {
    SrcView src;
    const double* coords;
    const int32_t* conn;
    const double* vol;
    const int64_t* inc_ptr;
    const int32_t* inc;
    const int64_t* rowptr;
    const int32_t* col;
    const double* val;
    const double* diag;
    const double* lumped;
    double* g;
    double* beta;
    double* bres;
    unsigned long long* ood;       // this transfer's out-of-domain counter (batch-owned)
    int64_t n, E;
    int64_t row0;                  // first row in the concatenated solver vectors
    int32_t tile0, ntiles;         // this system's row tiles
    int32_t dim;
    int32_t f32;                   // binary32 form of the fused route
    uint32_t N;
    double alpha;
    SampleKey key;
};

struct Tile {
    int32_t k;         // transfer
    int32_t variant;   // element tiles: (dimension, G, P); node tiles: dimension
    int64_t start;     // first element / node / row
};

// partial slots per row tile, scalar slots per system
enum { BP_BB = 0, BP_SB, BP_RZ, BP_RR, BP_PQ, BP_TRR, BP_MX, BP_COUNT };
enum { BS_RHO = 0, BS_ALPHA, BS_BETA, BS_TOL2, BS_DONE, BS_ITERS, BS_BB, BS_SUMB, BS_INTX, BS_TRR, BS_COUNT };

// ---------------------------------------------------------------- variants
// G lanes per element and P samples per lane per round: by default as the
// single-transfer fused route picks them (N <= 8 uses G = 16 here).
constexpr int kVariants = 5;
static int variant_of(int N) {
    if (N >= 256) return 0;   // G 64, P 4
    if (N >= 128) return 1;   // G 64, P 2
    if (N >= 64) return 2;    // G 64, P 1
    if (N > 16) return 3;     // G 32
    return 4;                 // G 16
}
static int lanes_of(int v) { return v <= 2 ? 64 : (v == 3 ? 32 : 16); }
static int per_lane_of(int v) { return v == 0 ? 4 : (v == 1 ? 2 : 1); }
// launch code of (variant, dimension, form)
static int code_of(int v, int dim, bool f32) { return v + (dim == 3 ? kVariants : 0) + (f32 ? 2 * kVariants : 0); }

template <int D, int G, int P, bool F32>
__device__ __forceinline__ void batch_elements(const BatchXfer& x, int64_t start, int lane, unsigned& nf,
                                               unsigned& nood, double* c_af) {
    const uint32_t t = uint32_t(start) + uint32_t(lane / G);
    fused_elements<D, G, P, 1, F32>(x.src, x.coords, x.n, x.conn, x.vol, uint32_t(x.E), x.N, x.alpha, x.key, x.g,
                                    x.beta, t, lane % G, nf, nood, c_af);
}

// One launch per (dimension, G, P) variant over that variant's tiles
// [first, last), so that each variant gets its own register budget.
template <int D, int G, int P, bool F32>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(D == 2 ? 3 : 2))) void k_batch_fused(
    const BatchXfer* __restrict__ X, const Tile* __restrict__ tiles, int64_t first, int64_t last,
    unsigned long long* __restrict__ nonfinite) {
    constexpr int WS = kWaveSlots<D> + kLamSlots<D, P>;
    __shared__ double lds[4 * WS];
    const int lane = threadIdx.x & 63;
    const int64_t stride = int64_t(gridDim.x) * 4;
    // the wave index, uniform by construction: the tile and its descriptor load into scalar registers
    const int wv = __builtin_amdgcn_readfirstlane(int(threadIdx.x >> 6));
    double* c_af = lds + wv * WS;
    for (int64_t w = first + int64_t(blockIdx.x) * 4 + wv; w < last; w += stride) {
        const Tile tl = tiles[w];
        const BatchXfer& x = X[tl.k];
        unsigned nf = 0, nood = 0;
        batch_elements<D, G, P, F32>(x, tl.start, lane, nf, nood, c_af);
        if (nf) atomicAdd(nonfinite + tl.k, (unsigned long long)nf);
        if (nood) atomicAdd(x.ood, (unsigned long long)nood);
    }
}

constexpr int kCodes = 4 * kVariants;   // variant, + kVariants for 3D, + 2 kVariants for binary32

template <int D, int G, int P, bool F32>
static void launch_fused_v(unsigned grid, hipStream_t s, const BatchXfer* X, const Tile* tiles, int64_t first,
                           int64_t last, unsigned long long* nf) {
    k_batch_fused<D, G, P, F32><<<grid, 256, 0, s>>>(X, tiles, first, last, nf);
}

template <int D, int G, int P, bool F32>
static int fused_blocks_per_cu() {
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_batch_fused<D, G, P, F32>, 256, 0) != hipSuccess ||
        per_cu < 1)
        per_cu = 1;
    return per_cu;
}

// launch (op 0) or resident blocks per CU (op 1) of element-stage code c
template <int D, bool F32>
static int fused_code_dv(int v, int op, unsigned grid, hipStream_t s, const BatchXfer* X, const Tile* tiles,
                         int64_t first, int64_t last, unsigned long long* nf) {
    switch (v) {
        case 0: return op ? fused_blocks_per_cu<D, 64, 4, F32>() : (launch_fused_v<D, 64, 4, F32>(grid, s, X, tiles, first, last, nf), 0);
        case 1: return op ? fused_blocks_per_cu<D, 64, 2, F32>() : (launch_fused_v<D, 64, 2, F32>(grid, s, X, tiles, first, last, nf), 0);
        case 2: return op ? fused_blocks_per_cu<D, 64, 1, F32>() : (launch_fused_v<D, 64, 1, F32>(grid, s, X, tiles, first, last, nf), 0);
        case 3: return op ? fused_blocks_per_cu<D, 32, 1, F32>() : (launch_fused_v<D, 32, 1, F32>(grid, s, X, tiles, first, last, nf), 0);
        default: return op ? fused_blocks_per_cu<D, 16, 1, F32>() : (launch_fused_v<D, 16, 1, F32>(grid, s, X, tiles, first, last, nf), 0);
    }
}

static int fused_code(int c, int op, unsigned grid, hipStream_t s, const BatchXfer* X, const Tile* tiles,
                      int64_t first, int64_t last, unsigned long long* nf) {
    const int v = c % kVariants;
    const bool d3 = ((c / kVariants) & 1) != 0;
    const bool f32 = c >= 2 * kVariants;
    if (!d3) return f32 ? fused_code_dv<2, true>(v, op, grid, s, X, tiles, first, last, nf)
                        : fused_code_dv<2, false>(v, op, grid, s, X, tiles, first, last, nf);
    return f32 ? fused_code_dv<3, true>(v, op, grid, s, X, tiles, first, last, nf)
               : fused_code_dv<3, false>(v, op, grid, s, X, tiles, first, last, nf);
}

static void launch_fused(int c, unsigned grid, hipStream_t s, const BatchXfer* X, const Tile* tiles, int64_t first,
                         int64_t last, unsigned long long* nf) {
    (void)fused_code(c, 0, grid, s, X, tiles, first, last, nf);
}

static int fused_per_cu(int c) { return fused_code(c, 1, 0, nullptr, nullptr, nullptr, 0, 0, nullptr); }

// step 1: g = f^s at the target nodes, 256 (2D) or 128 (3D) nodes per wavefront
__global__ __launch_bounds__(256) void k_batch_nodes(const BatchXfer* __restrict__ X, const Tile* __restrict__ tiles,
                                                     int64_t n_tiles) {
    __shared__ double lds[4 * kWaveSlots<3>];   // sized for the larger (3D) slots
    const int64_t stride = int64_t(gridDim.x) * 4;
    const int wv = __builtin_amdgcn_readfirstlane(int(threadIdx.x >> 6));
    double* c_af = lds + wv * kWaveSlots<3>;
    for (int64_t w = int64_t(blockIdx.x) * 4 + wv; w < n_tiles; w += stride) {
        const Tile tl = tiles[w];
        const BatchXfer& x = X[tl.k];
        unsigned nood;
        if (tl.variant == 2)
            nood = x.f32 ? eval_wave<2, 4, false, false, true>(x.src, tl.start, x.n, x.coords, x.n, x.g, x.n, nullptr, c_af)
                         : eval_wave<2, 4, false, false>(x.src, tl.start, x.n, x.coords, x.n, x.g, x.n, nullptr, c_af);
        else
            nood = x.f32 ? eval_wave<3, 2, false, false, true>(x.src, tl.start, x.n, x.coords, x.n, x.g, x.n, nullptr, c_af)
                         : eval_wave<3, 2, false, false>(x.src, tl.start, x.n, x.coords, x.n, x.g, x.n, nullptr, c_af);
        if (nood) atomicAdd(x.ood, (unsigned long long)nood);
    }
}

__global__ void k_fill_u64(unsigned long long* __restrict__ p, int64_t n) {
    for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x)
        p[i] = 0ull;
}

// ---------------------------------------------------------------- row-tile kernels
__device__ __forceinline__ double tile_total(double v) {
    __shared__ double sm[BT / 64];
    v = wave_sum_xor(v, 64);
    if ((threadIdx.x & 63) == 0) sm[threadIdx.x >> 6] = v;
    __syncthreads();
    double s = sm[0];
    for (int k = 1; k < BT / 64; ++k) s += sm[k];
    __syncthreads();
    return s;
}

__device__ __forceinline__ void tile_partial(double* __restrict__ part, int slot, double v) {
    const double t = tile_total(v);
    if (threadIdx.x == 0) part[int64_t(blockIdx.x) * BP_COUNT + slot] = t;
}

__device__ __forceinline__ double row_dot(const BatchXfer& x, int64_t i, const double* __restrict__ v) {
    double s = 0.0;
    for (int64_t k = x.rowptr[i]; k < x.rowptr[i + 1]; ++k) s = fma(x.val[k], v[x.col[k]], s);
    return s;
}

// step 6: b_res = sum over the incidence list of beta (ascending (t, k))
__global__ __launch_bounds__(BT) void k_batch_assemble(const BatchXfer* __restrict__ X, const Tile* __restrict__ rt) {
    const Tile tl = rt[blockIdx.x];
    const BatchXfer& x = X[tl.k];
    const int64_t v = tl.start + threadIdx.x;
    if (v >= x.n) return;
    double s = 0.0;
    for (int64_t i = x.inc_ptr[v]; i < x.inc_ptr[v + 1]; ++i) s += x.beta[x.inc[i]];
    x.bres[v] = s;
}

// step 2 and the right-hand side: b = alpha M g + b_res; partials of ||b||^2, sum b
__global__ __launch_bounds__(BT) void k_batch_rhs(const BatchXfer* __restrict__ X, const Tile* __restrict__ rt,
                                                  double* __restrict__ B, double* __restrict__ part) {
    const Tile tl = rt[blockIdx.x];
    const BatchXfer& x = X[tl.k];
    const int64_t i = tl.start + threadIdx.x;
    double bb = 0.0, sb = 0.0;
    if (i < x.n) {
        const double bi = x.alpha * row_dot(x, i, x.g) + x.bres[i];
        B[x.row0 + i] = bi;
        bb = bi * bi;
        sb = bi;
    }
    tile_partial(part, BP_BB, bb);
    tile_partial(part, BP_SB, sb);
}

// y = 0, r = b_res, z = D^-1 r, p_old = 0; partials of r.z and r.r
__global__ __launch_bounds__(BT) void k_batch_cg_init(const BatchXfer* __restrict__ X, const Tile* __restrict__ rt,
                                                      double* __restrict__ Y, double* __restrict__ R,
                                                      double* __restrict__ Z, double* __restrict__ Pold,
                                                      double* __restrict__ part) {
    const Tile tl = rt[blockIdx.x];
    const BatchXfer& x = X[tl.k];
    const int64_t i = tl.start + threadIdx.x;
    double rz = 0.0, rr = 0.0;
    if (i < x.n) {
        const int64_t o = x.row0 + i;
        const double ri = x.bres[i];
        const double zi = ri / x.diag[i];
        Y[o] = 0.0;
        R[o] = ri;
        Z[o] = zi;
        Pold[o] = 0.0;
        rz = ri * zi;
        rr = ri * ri;
    }
    tile_partial(part, BP_RZ, rz);
    tile_partial(part, BP_RR, rr);
}

// p_new = z + beta p_old (own rows), q = M p; partial p.q.  Eight lanes per
// row walk its entries together (consecutive entries, so each load of the
// matrix is a contiguous run per row) and add their parts with a butterfly;
// the tile's 256 rows take eight passes of 32 rows.
constexpr int kRowLanes = 8;

__global__ __launch_bounds__(BT) void k_batch_cg_spmv(const BatchXfer* __restrict__ X, const Tile* __restrict__ rt,
                                                      const double* __restrict__ Z, const double* __restrict__ Pold,
                                                      double* __restrict__ Pnew, double* __restrict__ Qv,
                                                      const double* __restrict__ sc, double* __restrict__ part) {
    const Tile tl = rt[blockIdx.x];
    if (sc[int64_t(tl.k) * BS_COUNT + BS_DONE] != 0.0) return;   // block-uniform
    const BatchXfer& x = X[tl.k];
    const double bt = sc[int64_t(tl.k) * BS_COUNT + BS_BETA];
    const double* z = Z + x.row0;
    const double* po = Pold + x.row0;
    const int sub = int(threadIdx.x) & (kRowLanes - 1);
    double pq = 0.0;
    for (int r0 = 0; r0 < BT; r0 += BT / kRowLanes) {
        const int64_t i = tl.start + r0 + int(threadIdx.x) / kRowLanes;
        double qi = 0.0;
        if (i < x.n) {
            const int64_t k1 = x.rowptr[i + 1];
            for (int64_t k = x.rowptr[i] + sub; k < k1; k += kRowLanes) {
                const int32_t j = x.col[k];
                qi = fma(x.val[k], fma(bt, po[j], z[j]), qi);
            }
        }
        qi += __shfl_xor(qi, 1, kRowLanes);
        qi += __shfl_xor(qi, 2, kRowLanes);
        qi += __shfl_xor(qi, 4, kRowLanes);
        if (i < x.n && sub == 0) {
            const double pi = fma(bt, po[i], z[i]);
            Pnew[x.row0 + i] = pi;
            Qv[x.row0 + i] = qi;
            pq = fma(pi, qi, pq);
        }
    }
    tile_partial(part, BP_PQ, pq);
}

// y += alpha p, r -= alpha q, z = D^-1 r; partials of r.z and r.r
__global__ __launch_bounds__(BT) void k_batch_cg_update(const BatchXfer* __restrict__ X, const Tile* __restrict__ rt,
                                                        const double* __restrict__ Pv, const double* __restrict__ Qv,
                                                        double* __restrict__ Y, double* __restrict__ R,
                                                        double* __restrict__ Z, const double* __restrict__ sc,
                                                        double* __restrict__ part) {
    const Tile tl = rt[blockIdx.x];
    if (sc[int64_t(tl.k) * BS_COUNT + BS_DONE] != 0.0) return;
    const BatchXfer& x = X[tl.k];
    const double a = sc[int64_t(tl.k) * BS_COUNT + BS_ALPHA];
    const int64_t i = tl.start + threadIdx.x;
    double rz = 0.0, rr = 0.0;
    if (i < x.n) {
        const int64_t o = x.row0 + i;
        Y[o] = fma(a, Pv[o], Y[o]);
        const double ri = fma(-a, Qv[o], R[o]);
        const double zi = ri / x.diag[i];
        R[o] = ri;
        Z[o] = zi;
        rz = ri * zi;
        rr = ri * ri;
    }
    tile_partial(part, BP_RZ, rz);
    tile_partial(part, BP_RR, rr);
}

// x = alpha g + y into the caller's arrays (pointer table); b copied if asked
__global__ __launch_bounds__(BT) void k_batch_solution(const BatchXfer* __restrict__ X, const Tile* __restrict__ rt,
                                                       const double* __restrict__ Y, const double* __restrict__ B,
                                                       double* const* __restrict__ xs, double* const* __restrict__ bs) {
    const Tile tl = rt[blockIdx.x];
    const BatchXfer& x = X[tl.k];
    const int64_t i = tl.start + threadIdx.x;
    if (i >= x.n) return;
    xs[tl.k][i] = fma(x.alpha, x.g[i], Y[x.row0 + i]);
    if (bs[tl.k]) bs[tl.k][i] = B[x.row0 + i];
}

// partials of ||b - M x||^2 and m^T x
__global__ __launch_bounds__(BT) void k_batch_report(const BatchXfer* __restrict__ X, const Tile* __restrict__ rt,
                                                     const double* __restrict__ B, double* const* __restrict__ xs,
                                                     double* __restrict__ part) {
    const Tile tl = rt[blockIdx.x];
    const BatchXfer& x = X[tl.k];
    const int64_t i = tl.start + threadIdx.x;
    double trr = 0.0, mx = 0.0;
    if (i < x.n) {
        const double* xv = xs[tl.k];
        const double ri = B[x.row0 + i] - row_dot(x, i, xv);
        trr = ri * ri;
        mx = x.lumped[i] * xv[i];
    }
    tile_partial(part, BP_TRR, trr);
    tile_partial(part, BP_MX, mx);
}

// Per-system scalars from the tile partials: one wavefront per system adds its
// tiles' partials (lane-strided, fixed butterfly) and lane 0 updates.
//   mode 0: after the rhs           ||b||^2, sum b, threshold, reset
//   mode 1: after r.z and r.r       stopping test; beta = rz / rho (0 at it = 0); rho = rz
//   mode 2: after p.q               alpha = rho / p.q
//   mode 3: after the report        ||b - M x||^2, m^T x
__device__ __forceinline__ double system_total(const BatchXfer& x, const double* __restrict__ part, int slot) {
    double s = 0.0;
    for (int t = threadIdx.x; t < x.ntiles; t += 64) s += part[int64_t(x.tile0 + t) * BP_COUNT + slot];
    return wave_sum_xor(s, 64);
}

__global__ __launch_bounds__(64) void k_batch_scalars(const BatchXfer* __restrict__ X, int mode, int it, double rtol2,
                                                      const double* __restrict__ part, double* __restrict__ sc) {
    const BatchXfer& x = X[blockIdx.x];
    double* s = sc + int64_t(blockIdx.x) * BS_COUNT;
    if (mode == 0) {
        const double bb = system_total(x, part, BP_BB);
        const double sb = system_total(x, part, BP_SB);
        if (threadIdx.x == 0) {
            s[BS_BB] = bb;
            s[BS_SUMB] = sb;
            s[BS_TOL2] = rtol2 * bb;
            s[BS_DONE] = 0.0;
            s[BS_ITERS] = 0.0;
            s[BS_BETA] = 0.0;
            s[BS_ALPHA] = 0.0;
            s[BS_RHO] = 0.0;
        }
    } else if (mode == 1) {
        if (s[BS_DONE] != 0.0) return;
        const double rz = system_total(x, part, BP_RZ);
        const double rr = system_total(x, part, BP_RR);
        if (threadIdx.x == 0) {
            s[BS_ITERS] = double(it);
            if (rr <= s[BS_TOL2] || !isfinite(rr)) {
                s[BS_DONE] = 1.0;
            } else {
                s[BS_BETA] = it == 0 ? 0.0 : rz / s[BS_RHO];
                s[BS_RHO] = rz;
            }
        }
    } else if (mode == 2) {
        if (s[BS_DONE] != 0.0) return;
        const double pq = system_total(x, part, BP_PQ);
        if (threadIdx.x == 0) s[BS_ALPHA] = s[BS_RHO] / pq;
    } else {
        const double trr = system_total(x, part, BP_TRR);
        const double mx = system_total(x, part, BP_MX);
        if (threadIdx.x == 0) {
            s[BS_TRR] = trr;
            s[BS_INTX] = mx;
        }
    }
}

}  // namespace ft

// ---------------------------------------------------------------- host side
struct ft_batch {
    int count = 0;                      // systems: one per field of each transfer
    int n_xfer = 0;                     // transfers
    std::vector<ft_target*> T;          // per system
    std::vector<ft_source*> S;
    std::vector<ft_sample_cfg> cfg;     // per system (one field)
    std::vector<int> xfer, field;       // per system: its transfer and field
    std::vector<int> first;             // per transfer: its first system
    std::vector<ft_sample_cfg> xcfg;    // per transfer, as given
    std::vector<int> var;         // element-stage variant (G, P) of each transfer
    int64_t rows = 0;
    size_t elem_cap = 0;          // element tiles d_elem can hold
    int64_t n_elem_tiles = 0, n_node_tiles = 0, n_row_tiles = 0;
    ft::BatchXfer* d_x = nullptr;
    ft::Tile* d_elem = nullptr;
    ft::Tile* d_node = nullptr;
    ft::Tile* d_row = nullptr;
    double *B = nullptr, *Y = nullptr, *R = nullptr, *Z = nullptr, *P = nullptr, *Q = nullptr;
    double* part = nullptr;
    double* sc = nullptr;
    unsigned long long* nonfinite = nullptr;   // [2][count]: non-finite values, out-of-domain queries
    std::vector<ft::BatchXfer> h_x;   // the descriptor table as last uploaded to d_x
    double** d_xs = nullptr;      // [2][count] pointer tables: x, then b
    double** h_xs = nullptr;      // pinned mirror
    double* h_sc = nullptr;       // pinned [count][BS_COUNT]
    unsigned long long* h_nf = nullptr;
    // element launch i runs code code_order[i] over tiles [code_first[i], code_first[i + 1]),
    // dearest tiles first
    int code_order[ft::kCodes] = {};
    int64_t code_first[ft::kCodes + 1] = {};
    unsigned code_grid[ft::kCodes] = {};
    unsigned grid_node = 1;
    bool use_graph = false;
    hipStream_t cap_stream = nullptr;
    hipGraphExec_t exec = nullptr;
    double cap_rtol = -1.0;
    int cap_iters = -1;
};

namespace ft {

ft_batch* batch_new(int count, ft_target* const* targets, ft_source* const* sources, const ft_sample_cfg* cfgs,
                    bool graph) {
    auto* b = new ft_batch();
    b->n_xfer = count;
    b->xcfg.assign(cfgs, cfgs + count);
    for (int k = 0; k < count; ++k) {
        b->first.push_back(int(b->T.size()));
        for (int f = 0; f < cfgs[k].n_fields; ++f) {
            ft_sample_cfg c = cfgs[k];
            c.n_fields = 1;
            b->T.push_back(targets[k]);
            b->S.push_back(sources[k]);
            b->cfg.push_back(c);
            b->xfer.push_back(k);
            b->field.push_back(f);
            b->var.push_back(variant_of(c.samples_per_elem));
        }
    }
    b->count = int(b->T.size());
    b->use_graph = graph;
    return b;
}

void batch_delete(ft_batch* b) { delete b; }

// after a run every target holds g, beta and b_res of its transfer, as after
// ft_transfer_p1: ft_project may re-solve it on its own
void batch_mark_consumed(ft_batch* b) {
    for (int k = 0; k < b->n_xfer; ++k) {
        ft_target* T = b->T[b->first[k]];
        T->consumed = true;
        T->consumed_cfg = b->xcfg[k];
    }
}

void batch_release(ft_batch* b) {
    if (!b) return;
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->cap_stream) (void)hipStreamDestroy(b->cap_stream);
    void* ps[] = {b->d_x, b->d_elem, b->d_node, b->d_row, b->B, b->Y, b->R, b->Z, b->P, b->Q, b->part, b->sc,
                  b->nonfinite, b->d_xs};
    for (void* p : ps) dev_free(p);
    if (b->h_xs) (void)hipHostFree(b->h_xs);
    if (b->h_sc) (void)hipHostFree(b->h_sc);
    if (b->h_nf) (void)hipHostFree(b->h_nf);
}

// The parts of a transfer's descriptor that point into its target and source.
// They are read again before every run: a source's bins are rebuilt by
// ft_source_autotune, and a target's field buffers are reallocated when a
// transfer of more fields grows them.
static void fill_live(ft_batch* b, int k, BatchXfer& x) {
    ft_target* T = b->T[k];
    ft_source* S = b->S[k];
    const int f = b->field[k];
    if (!S) {   // caller-values batch: no built-in source
        std::memset(&x.src, 0, sizeof(x.src));
    } else {
        x.src = source_view(S);
    }
    if (S && S->F > 1) {   // this system's field: the source seen as one field in its values array
        x.src.values += int64_t(f) * S->n;
        x.src.F = 1;
        x.src.rec_values = 0;
    }
    x.coords = T->coords;
    x.conn = T->conn;
    x.vol = T->vol;
    x.inc_ptr = T->inc_ptr;
    x.inc = T->inc;
    x.rowptr = T->rowptr;
    x.col = T->col;
    x.val = T->val;
    x.diag = T->diag;
    x.lumped = T->lumped;
    x.g = T->g + int64_t(f) * T->n;
    x.beta = T->beta + int64_t(f) * T->E * (T->dim + 1);
    x.bres = T->bres + int64_t(f) * T->n;
    x.ood = b->nonfinite + b->count + k;
}

static unsigned persistent_grid(int per_cu, int64_t waves) {
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) !=
                                                 hipSuccess)
        cus = 256;
    const int64_t want = (waves + 3) / 4;
    return unsigned(std::max<int64_t>(1, std::min<int64_t>(want, int64_t(cus) * std::max(1, per_cu))));
}

// Element tiles of every transfer with its variant, grouped by launch code;
// codes in the order of their dearest transfer (samples a tile draws, 3D
// about 1.5x dearer).  Uploads the list and sizes each code's persistent grid.
static ft_status build_element_tiles(ft_batch* b, hipStream_t s) {
    const int K = b->count;
    struct Group {
        double cost;
        int k;
    };
    std::vector<Group> order;
    for (int k = 0; k < K; ++k) {
        const int epw = 64 / lanes_of(b->var[k]);   // elements per wavefront
        order.push_back(Group{double(epw) * b->cfg[k].samples_per_elem * (b->T[k]->dim == 3 ? 1.5 : 1.0), k});
    }
    std::stable_sort(order.begin(), order.end(), [](const Group& a, const Group& c) { return a.cost > c.cost; });
    std::vector<std::vector<Tile>> by_code(kCodes);
    bool seen[kCodes] = {};
    int n_order = 0;
    for (const Group& gp : order) {
        const int k = gp.k;
        const int epw = 64 / lanes_of(b->var[k]);
        const int code = code_of(b->var[k], b->T[k]->dim, b->cfg[k].precision == FT_F32);
        if (!seen[code]) b->code_order[n_order++] = code;
        seen[code] = true;
        for (int64_t t = 0; t < b->T[k]->E; t += epw) by_code[code].push_back(Tile{k, code, t});
    }
    for (int c = 0; c < kCodes; ++c)
        if (!seen[c]) b->code_order[n_order++] = c;
    std::vector<Tile> elem;
    for (int i = 0; i < kCodes; ++i) {
        const int c = b->code_order[i];
        b->code_first[i] = int64_t(elem.size());
        elem.insert(elem.end(), by_code[c].begin(), by_code[c].end());
    }
    b->code_first[kCodes] = int64_t(elem.size());
    b->n_elem_tiles = int64_t(elem.size());
    if (elem.size() > b->elem_cap) {
        FT_TRY_HIP(hipStreamSynchronize(s));
        dev_free(b->d_elem);
        b->d_elem = nullptr;
        b->elem_cap = 0;
        FT_TRY(dev_alloc_n(&b->d_elem, elem.size()));
        b->elem_cap = elem.size();
    }
    FT_TRY_HIP(hipMemcpyAsync(b->d_elem, elem.data(), sizeof(Tile) * elem.size(), hipMemcpyHostToDevice, s));
    FT_TRY_HIP(hipStreamSynchronize(s));   // the host list goes out of scope
    for (int i = 0; i < kCodes; ++i)
        b->code_grid[i] = persistent_grid(fused_per_cu(b->code_order[i]), b->code_first[i + 1] - b->code_first[i]);
    return FT_OK;
}

ft_status batch_setup(ft_batch* b, hipStream_t s) {
    const int K = b->count;
    std::vector<BatchXfer> xs(K);
    std::vector<Tile> node, row;
    int64_t row0 = 0;
    for (int k = 0; k < K; ++k) {
        ft_target* T = b->T[k];
        const ft_sample_cfg& c = b->cfg[k];
        FT_TRY(ensure_field_buffers(T, b->xcfg[b->xfer[k]].n_fields, s));
        BatchXfer& x = xs[k];
        x.n = T->n;
        x.E = T->E;
        x.row0 = row0;
        x.tile0 = int32_t(row.size());
        x.dim = T->dim;
        x.f32 = c.precision == FT_F32 ? 1 : 0;
        x.N = uint32_t(c.samples_per_elem);
        x.alpha = c.alpha;
        x.key = make_sample_key(c, T->dim);
        for (int64_t v = 0; v < T->n; v += BT) row.push_back(Tile{k, T->dim, v});
        const int node_tile = T->dim == 2 ? 256 : 128;   // points per wavefront of the node stage
        for (int64_t v = 0; v < T->n; v += node_tile) node.push_back(Tile{k, T->dim, v});
        x.ntiles = int32_t(row.size()) - x.tile0;
        row0 += T->n;
    }
    if (row.size() >= (size_t(1) << 31)) {
        set_error("batch too large (%zu row tiles)", row.size());
        return FT_E_UNSUPPORTED;
    }
    b->rows = row0;
    b->n_node_tiles = int64_t(node.size());
    b->n_row_tiles = int64_t(row.size());
    FT_TRY(dev_alloc_n(&b->d_x, size_t(K)));
    FT_TRY(dev_alloc_n(&b->d_node, node.size()));
    FT_TRY(dev_alloc_n(&b->d_row, row.size()));
    for (double** p : {&b->B, &b->Y, &b->R, &b->Z, &b->Q}) FT_TRY(dev_alloc_n(p, size_t(row0)));
    FT_TRY(dev_alloc_n(&b->P, size_t(2 * row0)));
    FT_TRY(dev_alloc_n(&b->part, size_t(row.size()) * BP_COUNT));
    FT_TRY(dev_alloc_n(&b->sc, size_t(K) * BS_COUNT));
    FT_TRY(dev_alloc_n(&b->nonfinite, size_t(2 * K)));
    for (int k = 0; k < K; ++k) fill_live(b, k, xs[k]);
    FT_TRY(dev_alloc_n(&b->d_xs, size_t(2 * K)));
    FT_TRY_HIP(hipHostMalloc((void**)&b->h_xs, sizeof(double*) * 2 * K, hipHostMallocDefault));
    FT_TRY_HIP(hipHostMalloc((void**)&b->h_sc, sizeof(double) * BS_COUNT * K, hipHostMallocDefault));
    FT_TRY_HIP(hipHostMalloc((void**)&b->h_nf, sizeof(unsigned long long) * 2 * K, hipHostMallocDefault));
    FT_TRY_HIP(hipMemcpyAsync(b->d_x, xs.data(), sizeof(BatchXfer) * K, hipMemcpyHostToDevice, s));
    FT_TRY_HIP(hipMemcpyAsync(b->d_node, node.data(), sizeof(Tile) * node.size(), hipMemcpyHostToDevice, s));
    FT_TRY_HIP(hipMemcpyAsync(b->d_row, row.data(), sizeof(Tile) * row.size(), hipMemcpyHostToDevice, s));
    FT_TRY_HIP(hipStreamSynchronize(s));   // the host vectors go out of scope
    b->h_x = xs;
    FT_TRY(build_element_tiles(b, s));
    int node_per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&node_per_cu, k_batch_nodes, 256, 0) != hipSuccess)
        node_per_cu = 1;
    b->grid_node = persistent_grid(node_per_cu, b->n_node_tiles);
    if (b->use_graph) FT_TRY_HIP(hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking));
    return FT_OK;
}

// Every launch of one run, in order; no host synchronization, no memset.
// Without the element stage (the caller-values route) the runs starts from
// g and the element loads the consumption left in the targets.
static ft_status enqueue_run(ft_batch* b, const ft_solve_cfg* cfg, hipStream_t s, bool elements = true) {
    const int K = b->count;
    const unsigned nrt = unsigned(b->n_row_tiles);
    const int64_t rows = b->rows;
    k_fill_u64<<<grid_for(2 * K, 256), 256, 0, s>>>(b->nonfinite, 2 * K);
    if (elements && b->n_node_tiles) k_batch_nodes<<<b->grid_node, 256, 0, s>>>(b->d_x, b->d_node, b->n_node_tiles);
    for (int i = 0; elements && i < kCodes; ++i)
        if (b->code_first[i + 1] > b->code_first[i])
            launch_fused(b->code_order[i], b->code_grid[i], s, b->d_x, b->d_elem, b->code_first[i],
                         b->code_first[i + 1], b->nonfinite);
    k_batch_assemble<<<nrt, BT, 0, s>>>(b->d_x, b->d_row);
    k_batch_rhs<<<nrt, BT, 0, s>>>(b->d_x, b->d_row, b->B, b->part);
    k_batch_scalars<<<K, 64, 0, s>>>(b->d_x, 0, 0, cfg->rtol * cfg->rtol, b->part, b->sc);
    k_batch_cg_init<<<nrt, BT, 0, s>>>(b->d_x, b->d_row, b->Y, b->R, b->Z, b->P, b->part);
    k_batch_scalars<<<K, 64, 0, s>>>(b->d_x, 1, 0, 0.0, b->part, b->sc);
    for (int it = 0; it < cfg->max_iter; ++it) {
        double* Pold = b->P + ((it & 1) ? rows : 0);
        double* Pnew = b->P + ((it & 1) ? 0 : rows);
        k_batch_cg_spmv<<<nrt, BT, 0, s>>>(b->d_x, b->d_row, b->Z, Pold, Pnew, b->Q, b->sc, b->part);
        k_batch_scalars<<<K, 64, 0, s>>>(b->d_x, 2, it, 0.0, b->part, b->sc);
        k_batch_cg_update<<<nrt, BT, 0, s>>>(b->d_x, b->d_row, Pnew, b->Q, b->Y, b->R, b->Z, b->sc, b->part);
        k_batch_scalars<<<K, 64, 0, s>>>(b->d_x, 1, it + 1, 0.0, b->part, b->sc);
    }
    k_batch_solution<<<nrt, BT, 0, s>>>(b->d_x, b->d_row, b->Y, b->B, b->d_xs, b->d_xs + K);
    k_batch_report<<<nrt, BT, 0, s>>>(b->d_x, b->d_row, b->B, b->d_xs, b->part);
    k_batch_scalars<<<K, 64, 0, s>>>(b->d_x, 3, 0, 0.0, b->part, b->sc);
    FT_TRY_HIP(hipGetLastError());
    return FT_OK;
}

// Descriptors that point at memory a target or source has since replaced are
// refreshed (the kernels, and a captured graph, read the table at run time).
static ft_status refresh_descriptors(ft_batch* b, hipStream_t s) {
    const int K = b->count;
    std::vector<BatchXfer> xs = b->h_x;
    for (int k = 0; k < K; ++k) {
        fill_live(b, k, xs[k]);
        b->T[k]->fields_inner = false;   // the batch writes one field, [F][n] layout
    }
    if (std::memcmp(xs.data(), b->h_x.data(), sizeof(BatchXfer) * K) != 0) {
        b->h_x = xs;
        FT_TRY_HIP(hipMemcpyAsync(b->d_x, b->h_x.data(), sizeof(BatchXfer) * K, hipMemcpyHostToDevice, s));
    }
    return FT_OK;
}

// ---------------------------------------------------------------- autotuning
ft_status emit_points(ft_target* T, const ft_sample_cfg* cfg, void* points, hipStream_t s);
ft_status source_autotune(ft_source* S, int64_t head, int64_t npts, const void* pts, int64_t ld, int prec, int ncand,
                          const int32_t* cand, hipStream_t s);
ft_status source_rebin(ft_source* S, int32_t per_axis, hipStream_t s);
int32_t source_cells_longest(const ft_source* S);
int32_t source_default_cells(const ft_source* S);

// Tuned choice for one kind of transfer: its element variant and its bin
// grid as a factor on the source's default cells along the longest axis.
struct TuneEntry {
    int var = 2;
    double bins_scale = 1.0;
    double ms = 0.0;
};

// Cache file: JSON, one entry per line,
//   "<key>": {"G": 64, "P": 2, "bins_scale": 1.25, "ms": 0.4321}
// keyed by architecture, dimension, form, N, fields and the power-of-two
// buckets of the target and source element counts.
static std::map<std::string, TuneEntry> read_tune_cache(const char* path) {
    std::map<std::string, TuneEntry> out;
    if (!path) return out;
    FILE* f = std::fopen(path, "r");
    if (!f) return out;
    char line[1024];
    while (std::fgets(line, sizeof(line), f)) {
        char key[512];
        int G = 0, P = 0;
        double sc = 0.0, ms = 0.0;
        if (std::sscanf(line, " \"%511[^\"]\": {\"G\": %d, \"P\": %d, \"bins_scale\": %lf, \"ms\": %lf", key, &G, &P,
                        &sc, &ms) == 5) {
            int v = -1;
            for (int c = 0; c < kVariants; ++c)
                if (lanes_of(c) == G && per_lane_of(c) == P) v = c;
            if (v >= 0 && sc > 0.0 && sc < 100.0) out[key] = TuneEntry{v, sc, ms};
        }
    }
    std::fclose(f);
    return out;
}

static bool write_tune_cache(const char* path, const std::map<std::string, TuneEntry>& c) {
    if (!path) return true;
    FILE* f = std::fopen(path, "w");
    if (!f) return false;
    std::fprintf(f, "{\n  \"format\": \"ft batch autotune cache, one entry per line\",\n  \"entries\": {\n");
    size_t i = 0;
    for (const auto& kv : c) {
        std::fprintf(f, "    \"%s\": {\"G\": %d, \"P\": %d, \"bins_scale\": %.6g, \"ms\": %.6g}%s\n", kv.first.c_str(),
                     lanes_of(kv.second.var), per_lane_of(kv.second.var), kv.second.bins_scale, kv.second.ms,
                     ++i < c.size() ? "," : "");
    }
    std::fprintf(f, "  }\n}\n");
    return std::fclose(f) == 0;
}

static int ilog2(int64_t x) {
    int l = 0;
    while ((int64_t(1) << (l + 1)) <= x) ++l;
    return l;
}

static std::string tune_key(const char* arch, const ft_batch* b, int k) {
    char buf[256];
    std::snprintf(buf, sizeof(buf), "%s|d=%d|%s|N=%d|F=%d|E=2^%d|Es=2^%d", arch, b->T[k]->dim,
                  b->cfg[k].precision == FT_F32 ? "f32" : "f64", b->cfg[k].samples_per_elem, b->cfg[k].n_fields,
                  ilog2(b->T[k]->E), ilog2(b->S[k]->E));
    return buf;
}

// Element-stage time of transfer k alone with variant v (a warm-up launch,
// then two timed ones).
static ft_status time_variant(ft_batch* b, int k, int v, Tile* d_tiles, hipEvent_t e0, hipEvent_t e1, hipStream_t s,
                              float* ms) {
    const int epw = 64 / lanes_of(v);
    const int code = code_of(v, b->T[k]->dim, b->cfg[k].precision == FT_F32);
    std::vector<Tile> tiles;
    for (int64_t t = 0; t < b->T[k]->E; t += epw) tiles.push_back(Tile{k, code, t});
    const int64_t nt = int64_t(tiles.size());   // <= E, what d_tiles holds
    FT_TRY_HIP(hipMemcpyAsync(d_tiles, tiles.data(), sizeof(Tile) * tiles.size(), hipMemcpyHostToDevice, s));
    const unsigned grid = persistent_grid(fused_per_cu(code), nt);
    launch_fused(code, grid, s, b->d_x, d_tiles, 0, nt, b->nonfinite);
    FT_TRY_HIP(hipEventRecord(e0, s));
    for (int r = 0; r < 2; ++r) launch_fused(code, grid, s, b->d_x, d_tiles, 0, nt, b->nonfinite);
    FT_TRY_HIP(hipEventRecord(e1, s));
    FT_TRY_HIP(hipEventSynchronize(e1));
    FT_TRY_HIP(hipEventElapsedTime(ms, e0, e1));
    *ms *= 0.5f;
    return FT_OK;
}

ft_status batch_autotune(ft_batch* b, const char* cache_path, int32_t* n_tuned, hipStream_t s) {
    const int K = b->count;
    int dev = 0;
    hipDeviceProp_t prop{};
    FT_TRY_HIP(hipGetDevice(&dev));
    FT_TRY_HIP(hipGetDeviceProperties(&prop, dev));
    char arch[64];
    std::snprintf(arch, sizeof(arch), "%s", prop.gcnArchName);
    for (char* c = arch; *c; ++c)
        if (*c == ':') *c = 0;
    std::map<std::string, TuneEntry> cache = read_tune_cache(cache_path);
    std::map<std::string, std::vector<int>> groups;
    for (int k = 0; k < K; ++k) groups[tune_key(arch, b, k)].push_back(k);
    int tuned = 0;
    std::set<const ft_source*> rebinned;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    void* pts = nullptr;
    Tile* d_tiles = nullptr;
    ScratchGuard guard;
    guard.add(&pts);
    guard.add((void**)&d_tiles);
    ft_status st = FT_OK;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        set_error("event creation failed while tuning the batch");
        st = FT_E_DEVICE;
    }
    for (auto& g : groups) {
        if (st != FT_OK) break;
        auto it = cache.find(g.first);
        TuneEntry e;
        if (it != cache.end()) {
            e = it->second;
        } else {
            int rep = g.second[0];
            for (int k : g.second)
                if (b->T[k]->E > b->T[rep]->E) rep = k;
            ft_target* T = b->T[rep];
            ft_source* S = b->S[rep];
            const ft_sample_cfg& c = b->cfg[rep];
            // bins: the source autotuner on a run of this transfer's own samples
            const int64_t N = c.samples_per_elem;
            const int64_t Q = T->n + T->E * N;
            const size_t psz = c.precision == FT_F32 ? 4 : 8;
            dev_free(pts);
            pts = nullptr;
            if ((st = dev_alloc(&pts, size_t(T->dim) * size_t(Q) * psz)) != FT_OK) break;
            if ((st = emit_points(T, &c, pts, s)) != FT_OK) break;
            const int64_t m = std::max<int64_t>(1, std::min<int64_t>(T->E, (int64_t(1) << 21) / N));
            const int64_t t0 = (T->E - m) / 2;
            const int32_t base = source_default_cells(S);
            std::vector<int32_t> cand;
            for (double f : {0.6, 0.8, 1.0, 1.25, 1.6}) {
                const int32_t v = std::max<int32_t>(2, int32_t(std::lround(base * f)));
                if (std::find(cand.begin(), cand.end(), v) == cand.end()) cand.push_back(v);
            }
            const char* sample = static_cast<const char*>(pts) + (T->n + t0 * N) * psz;
            if ((st = source_autotune(S, 0, m * N, sample, Q, c.precision == FT_F32 ? FT_F32 : FT_F64,
                                      int(cand.size()), cand.data(), s)) != FT_OK)
                break;
            e.bins_scale = double(source_cells_longest(S)) / double(base);
            rebinned.insert(S);
            // element variant: the batch kernel of each candidate on this transfer's tiles
            if ((st = refresh_descriptors(b, s)) != FT_OK) break;
            dev_free(d_tiles);
            d_tiles = nullptr;
            // one tile per wavefront: E tiles for one element per wave, fewer otherwise
            if ((st = dev_alloc_n(&d_tiles, size_t(T->E))) != FT_OK) break;
            float best = INFINITY;
            for (int v = 0; v < kVariants && st == FT_OK; ++v) {
                float ms = 0.0f;
                st = time_variant(b, rep, v, d_tiles, e0, e1, s, &ms);
                if (st == FT_OK && ms < best) {
                    best = ms;
                    e.var = v;
                }
            }
            e.ms = best;
            cache[g.first] = e;
            ++tuned;
        }
        // the group's choices for all its transfers
        for (int k : g.second) {
            b->var[k] = e.var;
            ft_source* S = b->S[k];
            if (rebinned.count(S)) continue;
            const int32_t cells = std::max<int32_t>(2, int32_t(std::lround(source_default_cells(S) * e.bins_scale)));
            if (cells != source_cells_longest(S) && (st = source_rebin(S, cells, s)) != FT_OK) break;
            rebinned.insert(S);
        }
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (st != FT_OK) return st;
    FT_TRY(build_element_tiles(b, s));
    FT_TRY(refresh_descriptors(b, s));
    if (b->exec) {   // the launches changed: the next run captures again
        FT_TRY_HIP(hipGraphExecDestroy(b->exec));
        b->exec = nullptr;
    }
    FT_TRY_HIP(hipStreamSynchronize(s));
    if (!write_tune_cache(cache_path, cache)) {
        set_error("cannot write the autotuning cache %s", cache_path);
        return FT_E_ARG;
    }
    if (n_tuned) *n_tuned = tuned;
    return FT_OK;
}

int batch_count(const ft_batch* b) { return b->n_xfer; }
int batch_systems(const ft_batch* b) { return b->count; }

// The element-stage variant of transfer k as (G, P) (that of its first field).
void batch_variant(const ft_batch* b, int k, int32_t* G, int32_t* P) {
    *G = lanes_of(b->var[b->first[k]]);
    *P = per_lane_of(b->var[b->first[k]]);
}

ft_status batch_run(ft_batch* b, const ft_solve_cfg* cfg, double* const* x, double* const* bvec, ft_report* rep,
                    int32_t* status, hipStream_t s) {
    const int K = b->count;
    FT_TRY(refresh_descriptors(b, s));
    for (int k = 0; k < K; ++k) {   // system k: field f of transfer xfer[k], rows [f n, (f + 1) n)
        const int64_t off = int64_t(b->field[k]) * b->T[k]->n;
        b->h_xs[k] = x[b->xfer[k]] + off;
        b->h_xs[K + k] = bvec ? bvec[b->xfer[k]] + off : nullptr;
    }
    FT_TRY_HIP(hipMemcpyAsync(b->d_xs, b->h_xs, sizeof(double*) * 2 * K, hipMemcpyHostToDevice, s));
    if (b->use_graph) {
        if (!b->exec || b->cap_rtol != cfg->rtol || b->cap_iters != cfg->max_iter) {
            if (b->exec) {
                FT_TRY_HIP(hipGraphExecDestroy(b->exec));
                b->exec = nullptr;
            }
            hipGraph_t graph = nullptr;
            FT_TRY_HIP(hipStreamBeginCapture(b->cap_stream, hipStreamCaptureModeThreadLocal));
            const ft_status st = enqueue_run(b, cfg, b->cap_stream);
            const hipError_t e = hipStreamEndCapture(b->cap_stream, &graph);
            if (st != FT_OK) {
                if (graph) (void)hipGraphDestroy(graph);
                return st;
            }
            FT_TRY_HIP(e);
            const hipError_t ie = hipGraphInstantiate(&b->exec, graph, nullptr, nullptr, 0);
            (void)hipGraphDestroy(graph);
            FT_TRY_HIP(ie);
            b->cap_rtol = cfg->rtol;
            b->cap_iters = cfg->max_iter;
        }
        FT_TRY_HIP(hipGraphLaunch(b->exec, s));
    } else {
        FT_TRY(enqueue_run(b, cfg, s));
    }
    FT_TRY_HIP(hipMemcpyAsync(b->h_sc, b->sc, sizeof(double) * BS_COUNT * K, hipMemcpyDeviceToHost, s));
    FT_TRY_HIP(hipMemcpyAsync(b->h_nf, b->nonfinite, sizeof(unsigned long long) * 2 * K, hipMemcpyDeviceToHost, s));
    FT_TRY_HIP(hipStreamSynchronize(s));
    ft_status worst = FT_OK;
    for (int k = 0; k < K; ++k) {
        const double* h = b->h_sc + int64_t(k) * BS_COUNT;
        ft_report& R = rep[k];
        R.sum_b = h[BS_SUMB];
        R.int_x = h[BS_INTX];
        R.cons_defect = h[BS_SUMB] != 0.0 ? std::fabs(h[BS_INTX] - h[BS_SUMB]) / std::fabs(h[BS_SUMB])
                                          : std::fabs(h[BS_INTX]);
        R.rel_resid = h[BS_BB] > 0.0 ? std::sqrt(h[BS_TRR] / h[BS_BB]) : std::sqrt(h[BS_TRR]);
        R.iters = int32_t(h[BS_ITERS]);
        R.n_nonfinite = int64_t(b->h_nf[k]);
        R.n_out_of_domain = int64_t(b->h_nf[K + k]);
        b->T[k]->ood_mode = 2;   // a later ft_project of this target reports the same count
        b->T[k]->var_mode = VAR_NONE;
        R.sum_b_stderr = -1.0;
        if (b->field[k] == 0) b->T[k]->ood_host = R.n_out_of_domain;
        R.status = b->h_nf[k] ? FT_E_NONFINITE : (h[BS_DONE] != 0.0 ? FT_OK : FT_E_NOCONV);
        if (status) status[k] = R.status;
        if (R.status != FT_OK && (worst == FT_OK || R.status == FT_E_NONFINITE)) worst = ft_status(R.status);
    }
    if (worst == FT_E_NONFINITE) set_error("non-finite source values in at least one transfer of the batch");
    else if (worst == FT_E_NOCONV) set_error("CG did not reach rtol=%g within %d iterations for at least one transfer",
                                             cfg->rtol, cfg->max_iter);
    return worst;
}

ft_status consume_values(ft_target* T, const ft_sample_cfg* cfg, const void* values, double* beta, hipStream_t s);
ft_status stderr_launch(ft_target* T, int F, hipStream_t s);

ft_target* batch_target(const ft_batch* b, int k) { return b->T[b->first[k]]; }
const ft_sample_cfg* batch_cfg(const ft_batch* b, int k) { return &b->xcfg[k]; }
bool batch_has_sources(const ft_batch* b) {
    for (const ft_source* S : b->S)
        if (!S) return false;
    return true;
}

// Steps 4-7 of every transfer from caller values (the black-box route of
// each target, ft_consume_queries, then the batched solve): each transfer's
// consumption writes its element loads, g and b_res for all its fields; the
// batch then assembles, solves and reports every field, with no graph.
ft_status batch_run_values(ft_batch* b, const ft_solve_cfg* cfg, const void* const* values, double* const* x,
                           double* const* bvec, ft_report* rep, int32_t* status, hipStream_t s) {
    const int K = b->count;
    FT_TRY(refresh_descriptors(b, s));
    std::vector<unsigned long long> nonfinite(b->n_xfer, 0ull);
    for (int k = 0; k < b->n_xfer; ++k) {
        ft_target* T = b->T[b->first[k]];
        FT_TRY(consume_values(T, &b->xcfg[k], values[k], T->beta, s));
        FT_TRY_HIP(hipMemcpyAsync(&nonfinite[k], T->counters, sizeof(unsigned long long), hipMemcpyDeviceToHost, s));
        FT_TRY(stderr_launch(T, b->xcfg[k].n_fields, s));
    }
    for (int k = 0; k < K; ++k) {
        const int64_t off = int64_t(b->field[k]) * b->T[k]->n;
        b->h_xs[k] = x[b->xfer[k]] + off;
        b->h_xs[K + k] = bvec ? bvec[b->xfer[k]] + off : nullptr;
    }
    FT_TRY_HIP(hipMemcpyAsync(b->d_xs, b->h_xs, sizeof(double*) * 2 * K, hipMemcpyHostToDevice, s));
    FT_TRY(enqueue_run(b, cfg, s, false));
    FT_TRY_HIP(hipMemcpyAsync(b->h_sc, b->sc, sizeof(double) * BS_COUNT * K, hipMemcpyDeviceToHost, s));
    FT_TRY_HIP(hipStreamSynchronize(s));
    ft_status worst = FT_OK;
    for (int k = 0; k < K; ++k) {
        const double* h = b->h_sc + int64_t(k) * BS_COUNT;
        ft_report& R = rep[k];
        R.sum_b = h[BS_SUMB];
        R.int_x = h[BS_INTX];
        R.cons_defect = h[BS_SUMB] != 0.0 ? std::fabs(h[BS_INTX] - h[BS_SUMB]) / std::fabs(h[BS_SUMB])
                                          : std::fabs(h[BS_INTX]);
        R.rel_resid = h[BS_BB] > 0.0 ? std::sqrt(h[BS_TRR] / h[BS_BB]) : std::sqrt(h[BS_TRR]);
        R.iters = int32_t(h[BS_ITERS]);
        R.n_nonfinite = int64_t(nonfinite[b->xfer[k]]);
        R.n_out_of_domain = -1;   // the caller's black box evaluated the points
        R.sum_b_stderr = b->T[k]->var_mode == VAR_ESTIMATED ? std::sqrt(b->T[k]->h_var[b->field[k]]) : -1.0;
        R.status = R.n_nonfinite ? FT_E_NONFINITE : (h[BS_DONE] != 0.0 ? FT_OK : FT_E_NOCONV);
        if (status) status[k] = R.status;
        if (R.status != FT_OK && (worst == FT_OK || R.status == FT_E_NONFINITE)) worst = ft_status(R.status);
    }
    if (worst == FT_E_NONFINITE) set_error("non-finite query values in at least one transfer of the batch");
    else if (worst == FT_E_NOCONV) set_error("CG did not reach rtol=%g within %d iterations for at least one transfer",
                                             cfg->rtol, cfg->max_iter);
    return worst;
}

}  // namespace ft
