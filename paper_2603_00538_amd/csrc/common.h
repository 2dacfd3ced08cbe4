// Internal helpers shared by the HIP translation units of libft.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <string>

#include "../../include/ft.h"

namespace ft {

// ---------------------------------------------------------------- errors
void set_error(const char* fmt, ...);
void clear_error();

#define FT_TRY_HIP(expr)                                                          \
    do {                                                                          \
        hipError_t e_ = (expr);                                                   \
        if (e_ != hipSuccess) {                                                   \
            ::ft::set_error("%s failed: %s (%s:%d)", #expr, hipGetErrorString(e_), \
                            __FILE__, __LINE__);                                  \
            return FT_E_DEVICE;                                                   \
        }                                                                         \
    } while (0)

#define FT_TRY(expr)                     \
    do {                                 \
        ft_status s_ = (expr);           \
        if (s_ != FT_OK) return s_;      \
    } while (0)

#define FT_ARG_CHECK(cond, ...)                 \
    do {                                        \
        if (!(cond)) {                          \
            ::ft::set_error(__VA_ARGS__);       \
            return FT_E_ARG;                    \
        }                                       \
    } while (0)

// Device allocation that reports FT_E_OOM (and honours an optional byte cap
// from the FT_MAX_BYTES environment variable, for failure-path tests).
ft_status dev_alloc(void** p, size_t bytes);
template <class T>
ft_status dev_alloc_n(T** p, size_t n) { return dev_alloc(reinterpret_cast<void**>(p), n * sizeof(T) + 8); }
void dev_free(void* p);

// Frees registered scratch allocations when a setup routine returns.
struct ScratchGuard {
    void** ps[16];
    int count = 0;
    void add(void** p) { ps[count++] = p; }
    ~ScratchGuard() {
        for (int i = 0; i < count; ++i) {
            dev_free(*ps[i]);
            *ps[i] = nullptr;
        }
    }
};

inline unsigned int grid_for(int64_t n, int block) {
    int64_t g = (n + block - 1) / block;
    return (unsigned int)(g < 1 ? 1 : g);
}

// ---------------------------------------------------------------- sparse rows
// sum over the entries kk in [k0, k1) of a row, in order, of val[kk] * x(col[kk]):
// the column indices, values and x of four entries are loaded together (the last
// one to three entries reread entry k0 for the slots past the row, unused).
template <class T, class X>
__device__ __forceinline__ T row_dot4(const int32_t* __restrict__ col, const T* __restrict__ val, int64_t k0,
                                      int64_t k1, X&& x) {
    T s = T(0);
    int64_t kk = k0;
    for (; kk < k1; kk += 4) {
        int32_t j[4];
        T a[4], xj[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int64_t ku = kk + u < k1 ? kk + u : k0;
            j[u] = col[ku];
            a[u] = val[ku];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) xj[u] = x(j[u]);
#pragma unroll
        for (int u = 0; u < 4; ++u)
            if (kk + u < k1) s = fma(a[u], xj[u], s);
    }
    return s;
}

// Iterative solvers: CG iterations launched before the first host check, one
// more than the previous solve of the same kind needed (launches after
// convergence return at once), else 8.
inline int first_chunk(int hint) { return hint > 0 ? (hint + 1 < 64 ? hint + 1 : 64) : 8; }

// Exclusive scan of n int32 counts into n+1 int64 offsets (device arrays,
// work enqueued on stream; `tmp` must hold scan_tmp_elems(n) int64).
int64_t scan_tmp_elems(int64_t n);
ft_status exclusive_scan(const int32_t* counts, int64_t* offsets, int64_t n, int64_t* tmp, hipStream_t s);

// ---------------------------------------------------------------- Philox4x32-10
// Salmon, Moraes, Dror, Shaw (SC'11): ten rounds of two 32x32->64-bit
// multiplications per 4-word counter block, key bumped by the Weyl constants
// between rounds.
struct u32x4 {
    uint32_t x, y, z, w;
};

__device__ __forceinline__ u32x4 philox4x32_10(u32x4 c, uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        // one 32x32->64 product per multiplier gives both halves (a single v_mad_u64_u32)
        const uint64_t p0 = uint64_t(0xD2511F53u) * c.x;
        const uint64_t p1 = uint64_t(0xCD9E8D57u) * c.z;
        const uint32_t lo0 = uint32_t(p0), hi0 = uint32_t(p0 >> 32);
        const uint32_t lo1 = uint32_t(p1), hi1 = uint32_t(p1 >> 32);
        c = u32x4{hi1 ^ c.y ^ k0, lo1, hi0 ^ c.w ^ k1, lo0};
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return c;
}

// (2m+1) 2^-53 with m = ((a<<32)|b) >> 12, built exactly from the bit pattern
// 1.m (a double in [1,2)): (1 + m 2^-52) - 1 + 2^-53, all three steps exact.
__device__ __forceinline__ double uniform53(uint32_t a, uint32_t b) {
    const uint64_t m = ((uint64_t(a) << 32) | b) >> 12;
    const double one_m = __longlong_as_double((long long)(0x3FF0000000000000ull | m));
    return (one_m - 1.0) + 0x1p-53;
}

// (2k+1) 2^-24 with k the top 23 bits of the same m, i.e. a >> 9.
__device__ __forceinline__ float uniform24(uint32_t a) {
    const float one_k = __uint_as_float(0x3F800000u | (a >> 9));
    return (one_k - 1.0f) + 0x1p-24f;
}

// ---------------------------------------------------------------- division by an invariant
// Unsigned 32-bit division by a runtime-invariant d >= 1 with one multiply-high
// (Granlund & Montgomery, "Division by invariant integers using multiplication",
// PLDI 1994): l = ceil(log2 d), m' = floor(2^32 (2^l - d) / d) + 1,
// q = (t + ((n - t) >> min(l,1))) >> max(l-1, 0) with t = mulhi(m', n).
struct FastDiv {
    uint32_t d, mul, sh1, sh2;
};

inline FastDiv make_fastdiv(uint32_t d) {
    uint32_t l = 0;
    while ((uint64_t(1) << l) < d) ++l;
    const uint64_t m = ((uint64_t(1) << 32) * ((uint64_t(1) << l) - d)) / d + 1;
    return FastDiv{d, uint32_t(m), l < 1 ? l : 1u, l > 1 ? l - 1 : 0u};
}

__device__ __forceinline__ uint32_t fast_div(uint32_t n, const FastDiv& f) {
    const uint32_t t = __umulhi(f.mul, n);
    return (t + ((n - t) >> f.sh1)) >> f.sh2;
}

// ---------------------------------------------------------------- query value layouts
// Where the value of field f at a query lives.  Node v: values[f * node_ld + v].
// Sample j of element t: values[samp0 + t * samp_elem + f * samp_fld + j].
//   field-major [F][Q]:       node_ld = samp_fld = Q, samp0 = n, samp_elem = N
//   element tiles (F x N per  node_ld = n, samp0 = F n, samp_fld = N, samp_elem = F N
//   element, after [F][n]):
// A run of points without elements (plain evaluation) is field-major with
// N = 1 (each point its own "element").
struct ValueLayout {
    int64_t node_ld, samp0, samp_fld, samp_elem;
    FastDiv ndiv;   // division by N (samples per element)
};

inline ValueLayout field_major_layout(int64_t Q, int64_t n, int64_t N) {
    return ValueLayout{Q, n, Q, N, make_fastdiv(uint32_t(N))};
}

inline ValueLayout element_tile_layout(int64_t n, int64_t N, int F) {
    return ValueLayout{n, int64_t(F) * n, N, int64_t(F) * N, make_fastdiv(uint32_t(N))};
}

// ---------------------------------------------------------------- element basis
// Local edges of a P2 element: vertex pairs a < b in lexicographic order,
// d = 2: (0,1) (0,2) (1,2); d = 3: (0,1) (0,2) (0,3) (1,2) (1,3) (2,3).
__host__ __device__ constexpr int p2_edge(int d, int e, int end) {
    return d == 2 ? (end == 0 ? (e < 2 ? 0 : 1) : (e == 0 ? 1 : 2))
                  : (end == 0 ? (e < 3 ? 0 : (e < 5 ? 1 : 2)) : (e < 3 ? e + 1 : (e == 3 ? 2 : 3)));
}

// Lagrange basis of degree P on a straight-sided simplex, from the barycentric
// coordinates of the point: P1 psi_k = l_k; P2 vertex k: l_k (2 l_k - 1),
// edge e = (a, b): 4 l_a l_b.  Both sets add up to 1.
template <int D, int P>
struct Basis {
    static constexpr int n = P == 1 ? D + 1 : (D + 1) * (D + 2) / 2;
};

template <int D, int P>
__device__ __forceinline__ void basis_at(const double (&lam)[D + 1], double (&psi)[Basis<D, P>::n]) {
    if constexpr (P == 1) {
#pragma unroll
        for (int k = 0; k <= D; ++k) psi[k] = lam[k];
    } else {
#pragma unroll
        for (int k = 0; k <= D; ++k) psi[k] = lam[k] * (2.0 * lam[k] - 1.0);
#pragma unroll
        for (int e = 0; e < Basis<D, P>::n - D - 1; ++e)
            psi[D + 1 + e] = 4.0 * lam[p2_edge(D, e, 0)] * lam[p2_edge(D, e, 1)];
    }
}

// ---------------------------------------------------------------- wave helpers (wave64)
__device__ __forceinline__ double wave_sum_xor(double v, int width) {
    for (int o = width >> 1; o > 0; o >>= 1) v += __shfl_xor(v, o, width);
    return v;
}

// ---- totals of K binary64 values over the 64 lanes, returned wave-uniform.
// First the values are folded into rows of 16 lanes with the gfx950 lane-swap
// instructions: v_permlane32_swap exchanges the upper 32 lanes of one value
// with the lower 32 lanes of another, so one add leaves value i's partial sums
// in lanes 0-31 and value i+A's in lanes 32-63; v_permlane16_swap does the
// same between 16-lane rows, after which each row holds partial sums of a
// different value.  Each row is then summed on the DPP crossbar (quad
// permutations for lanes i^1 and i^2, the half-row and row mirrors; every lane
// of a row ends with the same total, since binary64 addition commutes), and
// the totals are read from lanes 0, 16, 32, 48.  No LDS traffic, and a fixed
// order of additions: the same totals every run.
__device__ __forceinline__ void swap_halves32(double& x, double& y) {
    const unsigned long long xb = __builtin_bit_cast(unsigned long long, x);
    const unsigned long long yb = __builtin_bit_cast(unsigned long long, y);
    const auto lo = __builtin_amdgcn_permlane32_swap(unsigned(xb), unsigned(yb), false, false);
    const auto hi = __builtin_amdgcn_permlane32_swap(unsigned(xb >> 32), unsigned(yb >> 32), false, false);
    x = __builtin_bit_cast(double, (static_cast<unsigned long long>(hi[0]) << 32) | lo[0]);
    y = __builtin_bit_cast(double, (static_cast<unsigned long long>(hi[1]) << 32) | lo[1]);
}

__device__ __forceinline__ void swap_rows16(double& x, double& y) {
    const unsigned long long xb = __builtin_bit_cast(unsigned long long, x);
    const unsigned long long yb = __builtin_bit_cast(unsigned long long, y);
    const auto lo = __builtin_amdgcn_permlane16_swap(unsigned(xb), unsigned(yb), false, false);
    const auto hi = __builtin_amdgcn_permlane16_swap(unsigned(xb >> 32), unsigned(yb >> 32), false, false);
    x = __builtin_bit_cast(double, (static_cast<unsigned long long>(hi[0]) << 32) | lo[0]);
    y = __builtin_bit_cast(double, (static_cast<unsigned long long>(hi[1]) << 32) | lo[1]);
}

template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v) {
    const unsigned long long u = __builtin_bit_cast(unsigned long long, v);
    const int lo = __builtin_amdgcn_update_dpp(int(unsigned(u)), int(unsigned(u)), CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(int(unsigned(u >> 32)), int(unsigned(u >> 32)), CTRL, 0xF, 0xF, false);
    return __builtin_bit_cast(double, (static_cast<unsigned long long>(unsigned(hi)) << 32) | unsigned(lo));
}

__device__ __forceinline__ double row_sum_f64(double v) {
    v += dpp_f64<0xB1>(v);    // quad_perm [1,0,3,2]
    v += dpp_f64<0x4E>(v);    // quad_perm [2,3,0,1]
    v += dpp_f64<0x141>(v);   // row_half_mirror: the two quads of each half-row
    v += dpp_f64<0x140>(v);   // row_mirror: the two halves of the row
    return v;
}

__device__ __forceinline__ double lane_f64(double v, int lane) {
    const unsigned long long u = __builtin_bit_cast(unsigned long long, v);
    const unsigned lo = __builtin_amdgcn_readlane(unsigned(u), lane);
    const unsigned hi = __builtin_amdgcn_readlane(unsigned(u >> 32), lane);
    return __builtin_bit_cast(double, (static_cast<unsigned long long>(hi) << 32) | lo);
}

// All 64 lanes must be active.  v[i] becomes the wave-uniform total of v[i].
template <int K>
__device__ __forceinline__ void wave_totals(double (&v)[K]) {
    constexpr int A = (K + 1) / 2;   // values after the 32-lane fold
    constexpr int B = (A + 1) / 2;   // after the 16-lane fold: one per row
    double a[A];
#pragma unroll
    for (int i = 0; i < A; ++i) {
        double x = v[i], y = i + A < K ? v[i + A] : 0.0;
        swap_halves32(x, y);
        a[i] = x + y;   // lanes 0-31: value i, lanes 32-63: value i + A
    }
    double b[B];
#pragma unroll
    for (int i = 0; i < B; ++i) {
        double x = a[i], y = i + B < A ? a[i + B] : 0.0;
        swap_rows16(x, y);
        b[i] = row_sum_f64(x + y);   // rows 0..3: values i, i + B, i + A, i + A + B
    }
#pragma unroll
    for (int i = 0; i < B; ++i) {
        v[i] = lane_f64(b[i], 0);
        if (i + B < A) v[i + B] = lane_f64(b[i], 16);
        if (i + A < K) v[i + A] = lane_f64(b[i], 32);
        if (i + A + B < K && i + B < A) v[i + A + B] = lane_f64(b[i], 48);
    }
}

// Binary32 minimum / maximum over the 64 lanes, returned wave-uniform (in
// scalar registers): butterflies inside each row of 16 lanes on the DPP
// crossbar (quad permutations for lanes i^1 and i^2, row rotations by 4 and 8),
// then the four row results.  No LDS traffic.
template <int CTRL>
__device__ __forceinline__ float dpp_f32(float v) {
    const int b = __builtin_bit_cast(int, v);
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(b, b, CTRL, 0xF, 0xF, false));
}

__device__ __forceinline__ float lane_f32(float v, int lane) {
    return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), lane));
}

__device__ __forceinline__ float wave_min_f32(float v) {
    v = fminf(v, dpp_f32<0xB1>(v));    // quad_perm [1,0,3,2]
    v = fminf(v, dpp_f32<0x4E>(v));    // quad_perm [2,3,0,1]
    v = fminf(v, dpp_f32<0x124>(v));   // row_ror:4
    v = fminf(v, dpp_f32<0x128>(v));   // row_ror:8
    return fminf(fminf(lane_f32(v, 0), lane_f32(v, 16)), fminf(lane_f32(v, 32), lane_f32(v, 48)));
}

__device__ __forceinline__ float wave_max_f32(float v) {
    v = fmaxf(v, dpp_f32<0xB1>(v));
    v = fmaxf(v, dpp_f32<0x4E>(v));
    v = fmaxf(v, dpp_f32<0x124>(v));
    v = fmaxf(v, dpp_f32<0x128>(v));
    return fmaxf(fmaxf(lane_f32(v, 0), lane_f32(v, 16)), fmaxf(lane_f32(v, 32), lane_f32(v, 48)));
}

__device__ __forceinline__ int read_lane(int v, int lane) {
    return __builtin_amdgcn_readlane(v, lane);
}

__device__ __forceinline__ int uniform_int(int v) {
    return __builtin_amdgcn_readfirstlane(v);
}

// The variance of an element's Monte Carlo total |Omega|/N sum_j r_j from the
// sum s1 and the sum of squares s2 of its N residuals (shifted by any
// constant): |Omega|^2 s^2 / N, s^2 the unbiased sample variance.  inv_n =
// 1/N, inv_var = 1/(N (N - 1)) (0 for N < 2, which gives 0).
__device__ __forceinline__ double element_variance(double vol, double s1, double s2, double inv_n, double inv_var) {
    const double ss = fmax(s2 - s1 * (s1 * inv_n), 0.0);   // sum of squared deviations
    return vol * vol * ss * inv_var;
}

// A value known to be equal in every lane, moved to scalar registers.
__device__ __forceinline__ double uniform_double(double v) {
    const unsigned long long u = __builtin_bit_cast(unsigned long long, v);
    const unsigned lo = __builtin_amdgcn_readfirstlane(unsigned(u));
    const unsigned hi = __builtin_amdgcn_readfirstlane(unsigned(u >> 32));
    return __builtin_bit_cast(double, (static_cast<unsigned long long>(hi) << 32) | lo);
}

}  // namespace ft

// ---------------------------------------------------------------- handles
// blocks of the per-field reduction of the element variances
constexpr int kVarBlocks = 64;
// what the last transfer says about the standard error of sum b
enum { VAR_NONE = 0, VAR_ESTIMATED = 1, VAR_EXACT = 2 };

struct ft_target {
    int dim = 0;
    int order = 1;              // 1: P1 (nodes = vertices); 2: P2 (vertices, then edge nodes)
    int nb = 0;                 // basis functions per element: dim+1, or (dim+1)(dim+2)/2 for P2
    int64_t n = 0, E = 0, nnz = 0, n_inverted = 0;
    // mesh copies
    double* coords = nullptr;   // [dim][n] every node (the vertices among them)
    int32_t* conn = nullptr;    // [E][dim+1] vertices: the element geometry and its samples
    int32_t* dofs = nullptr;    // [E][nb] the element's nodes (== conn for P1)
    double* vol = nullptr;      // [E]
    // mass matrix (CSR) and derived vectors
    int64_t* rowptr = nullptr;  // [n+1]
    int32_t* col = nullptr;     // [nnz]
    double* val = nullptr;      // [nnz]
    double* diag = nullptr;     // [n]
    double* lumped = nullptr;   // [n] m = M 1
    // node -> (element, local node) incidence, entries t*nb+k ascending
    int64_t* inc_ptr = nullptr; // [n+1]
    int32_t* inc = nullptr;     // [E*nb]
    // per-transfer state
    int F_cap = 0;
    double* beta = nullptr;     // [F][E][nb], or [E][nb][F] when fields_inner
    double* g = nullptr;        // [F][n], or [n][F] when fields_inner
    double* bres = nullptr;     // [F][n], or [n][F] when fields_inner
    bool fields_inner = false;  // layout of the last transfer (many-field matrix-core route)
    // the variance of each element's Monte Carlo total, [F][E] (written by the
    // black-box consumption, the fused route and plans: VAR_ESTIMATED after
    // them), its per-field sums [F] and their block partials [F][kVarBlocks][2]
    double* var_el = nullptr;
    double* var_tot = nullptr;
    double* var_part = nullptr;
    double* h_var = nullptr;    // pinned host copy of var_tot
    int var_mode = 0;           // VAR_NONE, VAR_ESTIMATED or VAR_EXACT (no sampling error)
    // solver work vectors and reduction scratch
    double *r = nullptr, *z = nullptr, *p = nullptr, *q = nullptr, *y = nullptr, *b = nullptr;
    double* scal = nullptr;               // device scalars
    double* partials = nullptr;           // per-block partial sums
    // [0] non-finite values seen by the last consume; [1] out-of-domain queries of
    // the last transfer from a built-in source, counted by its kernels
    unsigned long long* counters = nullptr;
    // where the report's out-of-domain count comes from: 0 unknown (black-box
    // route), 1 counters[1], 2 the host value ood_host (a plan's fixed count)
    int ood_mode = 0;
    int64_t ood_host = 0;
    double* h_scal = nullptr;             // pinned host mirror
    // mixed-precision solve (binary32 inner PCG), allocated on first use
    float* val32 = nullptr;               // [nnz] binary32 copy of M
    float* diag32 = nullptr;              // [n]
    float* w32 = nullptr;                 // [6n] r, z, p (2n), q, d in binary32
    double* scal32 = nullptr;             // inner-solve scalars
    // batched many-field solve, allocated on first use and grown with the field count
    int mf_Fp = 0;                        // field capacity (a power of two) of mf_vec
    double* mf_vec = nullptr;             // 8 vectors [n][mf_Fp]: G, B, Y, R, Z, Q, P (two)
    double* mf_sc = nullptr;              // per-field CG scalars
    double* mf_part = nullptr;            // per-field block partials
    int reduce_blocks = 0;
    // iterations the last solve of each kind needed (binary64, binary32 inner,
    // many-field): the first launch chunk of the next one, so that a repeated
    // transfer waits on the host once
    int cg_hint[3] = {0, 0, 0};
    // call-order state
    bool consumed = false;
    ft_sample_cfg consumed_cfg{};
};

struct ft_source {
    int dim = 0;
    int64_t n = 0, E = 0;
    int F = 0;
    double* coords = nullptr;   // [dim][n]
    int32_t* conn = nullptr;    // [E][dim+1]
    double* values = nullptr;   // [F][n]
    double* values_nm = nullptr;   // [n][F] node-major copy when F > 1 (a node's fields in one row)
    double* rec = nullptr;      // [E][RS]: origin + inverse Jacobian (barycentric map)
    float* box = nullptr;       // [E][8 | 6] outward-rounded boxes (2D also x+y, x-y ranges)
    int32_t nb[3] = {1, 1, 1};  // bins per axis
    double hx[3] = {0, 0, 0};   // largest half-extent of an element box per axis (enlarged)
    double dom_lo[3] = {0, 0, 0}, dom_hi[3] = {0, 0, 0};   // bounding box of the source nodes
    double lo[3] = {0, 0, 0};   // grid origin
    double inv_h[3] = {1, 1, 1};// bins per unit length
    int64_t* bin_ptr = nullptr; // [nbins+1]
    int32_t* bin_elems = nullptr;
    int64_t n_reg = 0;
    double fast_tau = 1e-9;     // margin of the localization's fast selection test
    unsigned long long* counters = nullptr;  // [0] out-of-domain points of ft_source_eval*
    unsigned long long* h_counters = nullptr;
};

namespace ft {
// Out-of-domain queries of the target's last transfer for its report, from
// its counters copied to the host: -1 when a caller's black box evaluated them.
inline int64_t report_ood(const ft_target* T, const unsigned long long* cnt) {
    return T->ood_mode == 1 ? int64_t(cnt[1]) : (T->ood_mode == 2 ? T->ood_host : int64_t(-1));
}
}  // namespace ft
