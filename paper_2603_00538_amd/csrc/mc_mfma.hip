// Many-field element sums on the matrix cores (sec. 4.1 step 5 for F fields).
//
// For one target element t with N samples and F fields the residual element
// loads form a small matrix product,
//   beta_t (F x (d+1)) = R_t^T (F x N) * Lambda_t (N x (d+1)) * |Omega_t| / N,
//   R_t[j][f] = y_f(X_tj) - alpha sum_l lambda_jl g_f(v_l),
// i.e. the residual of Eq. cv_element_load_residual_operator for every field
// at once.  It runs on v_mfma_f32_16x16x32_{f16,bf16}: M = 16 fields per tile,
// K = 32 samples per step, N = 16 columns of which the first d+1 are the
// barycentric weights.  Matrix-core products are split into hi + lo parts,
//   r lambda ~ r_hi lambda_hi + r_hi lambda_lo + r_lo lambda_hi
// (three MFMAs, FP32 accumulation), which keeps about 22 bits (f16) or 16 bits
// (bf16) of each product.  For f16 every field row of a K step is first
// scaled by a power of two so that its largest residual sits in [2^13, 2^14)
// (exact, undone when the step's products are added to binary64 running
// sums); bf16 shares the binary32 exponent range and needs no scaling.
//
// One wavefront per element stages its lambda (recomputed from the same
// Philox counters as the emission, binary32 form), the control values and a
// chunk of query values in LDS.  The element loads are written fields-inner,
// beta[t][k][f], for the node assembly that follows.  Every element sum
// is a fixed sequence of MFMAs and binary64 adds, so results are reproducible
// run to run.
#include "sampling.h"

namespace ft {

typedef float v4f __attribute__((ext_vector_type(4)));
typedef _Float16 v8h __attribute__((ext_vector_type(8)));
typedef __bf16 v8b __attribute__((ext_vector_type(8)));

constexpr int MF_NMAX = 256;   // samples per element handled by this kernel

template <bool BF16>
struct Split;

template <>
struct Split<false> {
    using vec = v8h;
    static __device__ __forceinline__ void set(vec& hi, vec& lo, int i, float v) {
        const _Float16 h = (_Float16)v;
        hi[i] = h;
        lo[i] = (_Float16)(v - (float)h);
    }
    static __device__ __forceinline__ v4f mma(const vec& a, const vec& b, v4f c) {
        return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
    }
};

template <>
struct Split<true> {
    using vec = v8b;
    static __device__ __forceinline__ void set(vec& hi, vec& lo, int i, float v) {
        const __bf16 h = (__bf16)v;
        hi[i] = h;
        lo[i] = (__bf16)(v - (float)h);
    }
    static __device__ __forceinline__ v4f mma(const vec& a, const vec& b, v4f c) {
        return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
    }
};

// One wavefront (and workgroup) per element.  The values are staged 16 field
// rows x 128 samples at a time (one chunk): 32 coalesced loads per lane, each
// reading 64 consecutive samples of one row, all in flight together, and the
// next chunk's loads are issued before this chunk's matrix-core work so that
// memory and compute overlap.  Every K step of 32 samples gets its own
// power-of-two row scaling (f16), and its products are unscaled into binary64
// running sums, so memory is read once.
constexpr int MF_CHUNK = 128;                   // samples per staged chunk (four K steps)
constexpr int MF_LPL = 16 * MF_CHUNK / 64;      // staged floats per lane

// FULL: every field tile and every chunk is whole (F a multiple of 16, N of
// MF_CHUNK), so no load, residual or weight needs a bounds test: the same
// sums with a quarter fewer vector instructions (measured at 64 fields x 128
// samples: 11.0 -> 8.7 ms in f16, 9.9 -> 8.4 ms in bf16).

template <int D, bool BF16, bool FULL>
__global__ __launch_bounds__(64) void k_consume_mfma(const float* __restrict__ values, ValueLayout L, int F,
                                                     const int32_t* __restrict__ conn, const double* __restrict__ vol,
                                                     int64_t n, uint32_t E, uint32_t N, float alpha, SampleKey key,
                                                     double* __restrict__ beta,
                                                     unsigned long long* __restrict__ nonfinite) {
    using S = Split<BF16>;
    __shared__ float lam_s[MF_NMAX][4];
    __shared__ float g_s[4][64];
    __shared__ float r_s[16][MF_CHUNK + 1];   // +1: row stride off the bank period
    const int lane = threadIdx.x & 63;
    const uint32_t t = blockIdx.x;            // grid = E: every block has an element
    int v[4] = {0, 0, 0, 0};
#pragma unroll
    for (int k = 0; k <= D; ++k) v[k] = conn[int64_t(t) * (D + 1) + k];
    // stage lambda (binary32 sampling form) and the control values
    for (uint32_t j = lane; j < MF_NMAX; j += 64) {
        float lf[D + 1];
        if (j < N) {
            sample_lambda_f32<D>(t, j, key, lf);
        } else {
#pragma unroll
            for (int k = 0; k <= D; ++k) lf[k] = 0.0f;
        }
#pragma unroll
        for (int k = 0; k < 4; ++k) lam_s[j][k] = k <= D ? lf[k < D + 1 ? k : 0] : 0.0f;
    }
    for (int idx = lane; idx < 4 * 64; idx += 64) {
        const int k = idx >> 6, f = idx & 63;
        g_s[k][f] = (k <= D && f < F) ? values[int64_t(f) * L.node_ld + v[k]] : 0.0f;
    }
    __syncthreads();

    const int sg = lane >> 4;            // sample group within a K step (8 samples)
    const int col = lane & 15;           // A row (field in the tile) / B, C column
    const int64_t qbase = L.samp0 + int64_t(t) * L.samp_elem;
    const int nchunk = int((N + MF_CHUNK - 1) / MF_CHUNK);
    const int nstep = ((F + 15) / 16) * nchunk;   // (field tile, sample chunk) pairs
    unsigned int nf = 0;
    const double scale_out = vol[t] / double(N);
    // load m of chunk s: row m/2 of its field tile, samples (m%2)*64 + lane of its chunk
    float pre[MF_LPL];
    auto load_chunk = [&](int s_) {
        const int f0 = (s_ / nchunk) * 16;
        const uint32_t c0 = uint32_t(s_ % nchunk) * MF_CHUNK;
#pragma unroll
        for (int m = 0; m < MF_LPL; ++m) {
            const int f = f0 + (m >> 1);
            const uint32_t j = c0 + uint32_t((m & 1) * 64 + lane);
            pre[m] = (FULL || (f < F && j < N)) ? values[int64_t(f) * L.samp_fld + qbase + j] : 0.0f;
        }
    };
    load_chunk(0);
    double run[4] = {0.0, 0.0, 0.0, 0.0};   // C[4 sg + i][col] of the current field tile, unscaled
    for (int s_ = 0; s_ < nstep; ++s_) {
        const int f0 = (s_ / nchunk) * 16;
        const uint32_t c0 = uint32_t(s_ % nchunk) * MF_CHUNK;
#pragma unroll
        for (int m = 0; m < MF_LPL; ++m) {
            nf += !isfinite(pre[m]);
            r_s[m >> 1][(m & 1) * 64 + lane] = pre[m];
        }
        __builtin_amdgcn_wave_barrier();
        if (s_ + 1 < nstep) load_chunk(s_ + 1);   // in flight during this chunk's products
        for (int ks = 0; ks < MF_CHUNK / 32; ++ks) {
            if (!FULL && c0 + uint32_t(ks * 32) >= N) break;   // wave-uniform: no samples left in this chunk
            const uint32_t jb = c0 + uint32_t(ks * 32 + sg * 8);
            const int f = f0 + col;
            float rv[8];
            float mx = 0.0f;
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                const uint32_t j = jb + uint32_t(i);
                float r = 0.0f;
                if (FULL || (f < F && j < N)) {
                    float gx = 0.0f;
#pragma unroll
                    for (int k = 0; k <= D; ++k) gx = fmaf(lam_s[j][k], g_s[k][f & 63], gx);
                    r = r_s[col][ks * 32 + sg * 8 + i] - alpha * gx;
                }
                rv[i] = r;
                mx = fmaxf(mx, fabsf(r));
            }
            int e = 0;
            if (!BF16) {   // row maximum over this K step's 32 samples -> [2^13, 2^14)
                mx = fmaxf(mx, __shfl_xor(mx, 16, 64));
                mx = fmaxf(mx, __shfl_xor(mx, 32, 64));
                if (mx > 0.0f && isfinite(mx)) e = 13 - ilogbf(mx);
            }
            const float sc = ldexpf(1.0f, e);
            typename S::vec ahi, alo, bhi, blo;
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                const uint32_t j = jb + uint32_t(i);
                S::set(ahi, alo, i, rv[i] * sc);
                const float lv = FULL ? (col <= D ? lam_s[j][col & 3] : 0.0f)
                                      : ((col <= D && j < MF_NMAX) ? lam_s[j < MF_NMAX ? j : 0][col & 3] : 0.0f);
                S::set(bhi, blo, i, lv);
            }
            v4f acc = {0.0f, 0.0f, 0.0f, 0.0f};
            acc = S::mma(ahi, bhi, acc);
            acc = S::mma(ahi, blo, acc);
            acc = S::mma(alo, bhi, acc);
#pragma unroll
            for (int i = 0; i < 4; ++i) run[i] += ldexp(double(acc[i]), -__shfl(e, 4 * sg + i, 64));
        }
        __builtin_amdgcn_wave_barrier();
        if (s_ % nchunk == nchunk - 1) {
            // C[row][col]: row = 4*sg + i (field f0 + row), col = barycentric index;
            // beta[t][col][f], the fields of one (element, vertex) contiguous
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int fo = f0 + 4 * sg + i;
                if (col <= D && fo < F) beta[(int64_t(t) * (D + 1) + col) * F + fo] = run[i] * scale_out;
                run[i] = 0.0;
            }
        }
    }
    if (nf) atomicAdd(nonfinite, (unsigned long long)nf);
}

template <int D, bool BF16>
static void launch_mfma(ft_target* T, const ft_sample_cfg* cfg, const float* vals, const ValueLayout& L, float a,
                        const SampleKey& key, double* beta, hipStream_t s) {
    const uint32_t N = uint32_t(cfg->samples_per_elem);
    const bool full = cfg->n_fields % 16 == 0 && N % MF_CHUNK == 0;
    auto kern = full ? k_consume_mfma<D, BF16, true> : k_consume_mfma<D, BF16, false>;
    kern<<<unsigned(T->E), 64, 0, s>>>(vals, L, cfg->n_fields, T->conn, T->vol, T->n, uint32_t(T->E), N, a, key, beta,
                                       T->counters);   // one element per workgroup
}

ft_status consume_mfma(ft_target* T, const ft_sample_cfg* cfg, const void* values, const ValueLayout& L,
                       double* beta, hipStream_t s) {
    const SampleKey key = make_sample_key(*cfg, T->dim);
    if (T->E == 0) return FT_OK;
    const bool bf = cfg->precision == FT_SPLIT_BF16;
    const float* vals = static_cast<const float*>(values);
    const float a = float(cfg->alpha);
    if (T->dim == 2) {
        if (bf) launch_mfma<2, true>(T, cfg, vals, L, a, key, beta, s);
        else launch_mfma<2, false>(T, cfg, vals, L, a, key, beta, s);
    } else {
        if (bf) launch_mfma<3, true>(T, cfg, vals, L, a, key, beta, s);
        else launch_mfma<3, false>(T, cfg, vals, L, a, key, beta, s);
    }
    FT_TRY_HIP(hipGetLastError());
    return FT_OK;
}

}  // namespace ft
