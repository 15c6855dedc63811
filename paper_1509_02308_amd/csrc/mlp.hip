// mlp.hip -- learned candidate proposer: features of the fixed probe grid,
// Philox-noised training samples, canonical labels, a 768-256-256-n MLP
// trained with bf16 MFMA GEMMs (fp32 accumulate) and Adam, and the top-k
// proposal that the exact replay then confirms.
//
// The grid is the Section 4.2 procedure fixed once: array sizes swept
// across the candidate capacities, strides around the line sizes, two
// passes; a feature is the steady-pass miss ratio r of Section 4.1.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <unordered_map>

#include "plan.h"

namespace pc {

constexpr uint32_t kIn = PCHASE_MLP_IN, kHid = PCHASE_MLP_HIDDEN;
constexpr uint32_t kGridSizes = 256, kGridStrides = 3;
constexpr uint32_t kMaxBase4 = 32;   // base offsets 4 * [0, 32): below the largest line
constexpr uint32_t kMaxTopK = 64;

static void grid_probe(uint32_t p, uint64_t base, pchase_probe* out) {
    static const uint32_t strides[kGridStrides] = {32, 64, 128};
    out->n_bytes = 4096 + 512ull * (p % kGridSizes);
    out->s_bytes = strides[p / kGridSizes];
    out->base_offset = base;
    out->j0 = 0;
    out->elem_bytes = 4;
    out->passes = 2;
}

// ------------------------------------------------------------- philox ---
// Philox4x32-10 (Salmon et al., SC'11), all four output words.
__host__ __device__ inline void philox4(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint32_t k0,
                                        uint32_t k1, uint32_t out[4]) {
    for (int r = 0; r < 10; ++r) {
        const uint64_t p0 = (uint64_t)0xD2511F53u * c0, p1 = (uint64_t)0xCD9E8D57u * c2;
        const uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
        const uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
        c1 = (uint32_t)p1;
        c3 = (uint32_t)p0;
        c0 = n0;
        c2 = n2;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    out[0] = c0;
    out[1] = c1;
    out[2] = c2;
    out[3] = c3;
}

__device__ __forceinline__ uint16_t f2bf(float v) {
    uint32_t u = __float_as_uint(v);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

// ------------------------------------------------------ feature kernel ---
// One wave per (row, probe): x = (L - steady hits after optional flips) / L.
struct FeatArgs {
    const uint32_t* bits;
    const uint64_t* row_bit0;    // per row: bit offset of the row's bits
    const uint64_t* probe_bit;   // per probe: bit offset of its first access
    const uint32_t* probe_L;     // per probe: cycle length; steady bits are [L, 2L)
    const uint32_t* row_thr;     // per row flip threshold (16-bit), or NULL
    const uint64_t* row_sample;  // per row sample index (noise counter)
    const uint32_t* row_out;     // output row, or NULL for identity
    uint32_t rows, n_probes;
    uint32_t key0, key1;
    float* x;
};

__global__ void __launch_bounds__(256) feature_kernel(FeatArgs a, uint32_t row_first) {
    const uint32_t lane = threadIdx.x & 63;
    const uint32_t p = blockIdx.x * 4 + (threadIdx.x >> 6);
    const uint32_t r = row_first + blockIdx.y;
    if (p >= a.n_probes || r >= a.rows) return;
    const uint32_t L = a.probe_L[p];
    const uint64_t q0 = (a.row_bit0 ? a.row_bit0[r] : 0) + a.probe_bit[p] + L;
    const uint32_t thr = a.row_thr ? a.row_thr[r] : 0u;
    const uint64_t sample = a.row_sample ? a.row_sample[r] : 0;
    const uint32_t s_lo = (uint32_t)sample, s_hi = 0x80000000u | (uint32_t)(sample >> 32);
    uint32_t hits = 0;
    const uint32_t chunks = (L + 31) / 32;
    for (uint32_t c = lane; c < chunks; c += 64) {
        const uint32_t nb = min(32u, L - 32 * c);
        const uint64_t q = q0 + 32ull * c;
        const uint64_t w0 = q >> 5;
        const uint32_t sh = (uint32_t)(q & 31);
        uint32_t v = a.bits[w0] >> sh;
        if (sh && sh + nb > 32) v |= a.bits[w0 + 1] << (32 - sh);
        const uint32_t valid = nb == 32 ? 0xFFFFFFFFu : ((1u << nb) - 1u);
        uint32_t flip = 0;
        if (thr) {
            for (uint32_t blk = 0; blk < 4; ++blk) {
                if (8 * blk >= nb) break;
                uint32_t o[4];
                philox4(4 * c + blk, p, s_lo, s_hi, a.key0, a.key1, o);
                for (uint32_t t = 0; t < 8; ++t) {
                    const uint32_t u16 = (o[t >> 1] >> (16 * (t & 1))) & 0xFFFFu;
                    flip |= (u16 < thr ? 1u : 0u) << (8 * blk + t);
                }
            }
        }
        hits += __popc((v ^ flip) & valid);
    }
    for (int o = 32; o > 0; o >>= 1) hits += __shfl_xor(hits, o);
    if (lane == 0) {
        const uint32_t out = a.row_out ? a.row_out[r] : r;
        a.x[(uint64_t)out * a.n_probes + p] = (float)((double)(L - hits) / (double)L);
    }
}

// ------------------------------------------------------ label kernels ---
// Position-mixed 64-bit sum of the steady bits of one slot (grouping key).
__device__ __forceinline__ uint64_t mix64(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

__device__ __forceinline__ uint32_t steady_chunk(const uint32_t* bits, uint64_t q, uint32_t nb) {
    const uint64_t w0 = q >> 5;
    const uint32_t sh = (uint32_t)(q & 31);
    uint32_t v = bits[w0] >> sh;
    if (sh && sh + nb > 32) v |= bits[w0 + 1] << (32 - sh);
    return nb == 32 ? v : (v & ((1u << nb) - 1u));
}

__global__ void __launch_bounds__(256) signature_kernel(const uint32_t* bits, uint64_t slot_bits,
                                                        const uint64_t* probe_bit, const uint32_t* probe_L,
                                                        uint32_t n_probes, uint64_t* sig) {
    __shared__ uint64_t part[256];
    const uint32_t slot = blockIdx.x;
    uint64_t h = 0;
    for (uint32_t p = 0; p < n_probes; ++p) {
        const uint32_t L = probe_L[p];
        const uint64_t q0 = slot * slot_bits + probe_bit[p] + L;
        for (uint32_t c = threadIdx.x; c < (L + 31) / 32; c += 256) {
            const uint32_t v = steady_chunk(bits, q0 + 32ull * c, min(32u, L - 32 * c));
            h += mix64(((uint64_t)p << 48) ^ ((uint64_t)c << 32) ^ v);
        }
    }
    part[threadIdx.x] = h;
    __syncthreads();
    for (uint32_t s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s) part[threadIdx.x] += part[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) sig[slot] = part[0];
}

// differ[k] = 1 when slots pair[2k] and pair[2k+1] have different steady bits
__global__ void __launch_bounds__(256) pair_differ_kernel(const uint32_t* bits, uint64_t slot_bits,
                                                          const uint64_t* probe_bit, const uint32_t* probe_L,
                                                          uint32_t n_probes, const uint32_t* pair,
                                                          uint32_t* differ) {
    __shared__ uint32_t any;
    if (threadIdx.x == 0) any = 0;
    __syncthreads();
    const uint32_t i = pair[2 * blockIdx.x], j = pair[2 * blockIdx.x + 1];
    uint32_t d = 0;
    for (uint32_t p = 0; p < n_probes && !d; ++p) {
        const uint32_t L = probe_L[p];
        const uint64_t qi = i * slot_bits + probe_bit[p] + L, qj = j * slot_bits + probe_bit[p] + L;
        for (uint32_t c = threadIdx.x; c < (L + 31) / 32; c += 256) {
            const uint32_t nb = min(32u, L - 32 * c);
            d |= steady_chunk(bits, qi + 32ull * c, nb) ^ steady_chunk(bits, qj + 32ull * c, nb);
        }
    }
    if (d) any = 1;   // benign same-value race
    __syncthreads();
    if (threadIdx.x == 0) differ[blockIdx.x] = any;
}

// ------------------------------------------------------------- GEMM ---
// C(m, n) = alpha * sum_k A(m, k) B(k, n) with fp32 accumulation on gfx950's
// v_mfma_f32_32x32x16_bf16: a 256-thread block computes a 64 x 64 tile as
// 2 x 2 waves of 32 x 32, K staged through LDS 32 at a time.
// An operand is either bf16 (the weights and the input features, whose
// values are exactly bf16) or fp32 (hidden activations and back-propagated
// errors).  An fp32 operand is split while it is staged into v = hi + lo,
// hi = bf16(v), lo = bf16(v - hi), which holds v to about 2^-17 relative;
// the product then takes hi*hi + lo*hi + hi*lo (lo*lo is below fp32
// rounding of the sum).  Operands are addressed through element strides, so
// transposed products need no copies.  Epilogue: + bias[n], ReLU, keep only
// where mask(m, n) > 0 (ReLU backward on the fp32 activation), fp32 store.
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

struct GemmArgs {
    const uint16_t* A;    // bf16 operand, or NULL when Af is given
    const float* Af;      // fp32 operand, split into hi + lo
    const uint16_t* B;
    const float* Bf;
    int64_t a_m, a_k, b_k, b_n;
    uint32_t M, N, K;
    float alpha;
    const float* bias;
    const float* mask;
    int64_t ld;
    float* out_f;
    int relu;
};

constexpr int kTM = 64, kTN = 64, kTK = 32, kPitch = 40;

__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

__global__ void __launch_bounds__(256) gemm_bf16_kernel(GemmArgs g) {
    __shared__ __align__(16) uint16_t As[2][kTM * kPitch];   // [hi|lo][m][k]
    __shared__ __align__(16) uint16_t Bs[2][kTN * kPitch];   // [hi|lo][n][k]
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int wm = w >> 1, wn = w & 1;
    const uint32_t m0 = blockIdx.y * kTM, n0 = blockIdx.x * kTN;
    const bool a_kfast = g.a_k == 1, b_kfast = g.b_k == 1;
    const bool a_split = g.Af != nullptr, b_split = g.Bf != nullptr;
    f32x16 acc = {};
    for (uint32_t k0 = 0; k0 < g.K; k0 += kTK) {
#pragma unroll
        for (int r = 0; r < 8; ++r) {
            const int e = tid + 256 * r;
            int mm, kk;
            if (a_kfast) { kk = e & 31; mm = e >> 5; } else { mm = e & 63; kk = e >> 6; }
            uint32_t gm = m0 + mm, gk = k0 + kk;
            const bool a_in = gm < g.M && gk < g.K;
            const int64_t ai = (int64_t)gm * g.a_m + (int64_t)gk * g.a_k;
            if (a_split) {
                const float v = a_in ? g.Af[ai] : 0.f;
                const uint16_t hi = f2bf(v);
                As[0][mm * kPitch + kk] = hi;
                As[1][mm * kPitch + kk] = f2bf(v - bf2f(hi));
            } else {
                As[0][mm * kPitch + kk] = a_in ? g.A[ai] : 0;
            }
            int nn;
            if (b_kfast) { kk = e & 31; nn = e >> 5; } else { nn = e & 63; kk = e >> 6; }
            const uint32_t gn = n0 + nn;
            gk = k0 + kk;
            const bool b_in = gn < g.N && gk < g.K;
            const int64_t bi = (int64_t)gk * g.b_k + (int64_t)gn * g.b_n;
            if (b_split) {
                const float v = b_in ? g.Bf[bi] : 0.f;
                const uint16_t hi = f2bf(v);
                Bs[0][nn * kPitch + kk] = hi;
                Bs[1][nn * kPitch + kk] = f2bf(v - bf2f(hi));
            } else {
                Bs[0][nn * kPitch + kk] = b_in ? g.B[bi] : 0;
            }
        }
        __syncthreads();
        // lane l feeds row (l mod 32) with 8 consecutive k at 8 (l div 32);
        // A and B use the same k positions, so the sum is over all 16
#pragma unroll
        for (int ks = 0; ks < kTK; ks += 16) {
            const int row = lane & 31, kq = ks + (lane >> 5) * 8;
            const int ao = (wm * 32 + row) * kPitch + kq, bo = (wn * 32 + row) * kPitch + kq;
            const bf16x8 ah = *reinterpret_cast<const bf16x8*>(&As[0][ao]);
            const bf16x8 bh = *reinterpret_cast<const bf16x8*>(&Bs[0][bo]);
            acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, bh, acc, 0, 0, 0);
            if (a_split) {
                const bf16x8 al = *reinterpret_cast<const bf16x8*>(&As[1][ao]);
                acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al, bh, acc, 0, 0, 0);
            }
            if (b_split) {
                const bf16x8 bl = *reinterpret_cast<const bf16x8*>(&Bs[1][bo]);
                acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, bl, acc, 0, 0, 0);
            }
        }
        __syncthreads();
    }
    const uint32_t col = n0 + wn * 32 + (lane & 31);
    if (col >= g.N) return;
#pragma unroll
    for (int j = 0; j < 16; ++j) {
        const uint32_t row = m0 + wm * 32 + (j >> 2) * 8 + (lane >> 5) * 4 + (j & 3);
        if (row >= g.M) continue;
        float v = acc[j] * g.alpha;
        if (g.bias) v += g.bias[col];
        if (g.relu) v = v > 0.f ? v : 0.f;
        const int64_t at = (int64_t)row * g.ld + col;
        if (g.mask && !(g.mask[at] > 0.f)) v = 0.f;
        g.out_f[at] = v;
    }
}

static hipError_t gemm(const GemmArgs& g, hipStream_t s) {
    if (g.M == 0 || g.N == 0) return hipSuccess;
    dim3 grid((g.N + kTN - 1) / kTN, (g.M + kTM - 1) / kTM);
    hipLaunchKernelGGL(gemm_bf16_kernel, grid, dim3(256), 0, s, g);
    return hipGetLastError();
}

// ------------------------------------------------ small MLP kernels ---
// Training state on the device, so that one captured step serves every
// batch of a pass: the step reads batch `batch` of the sample arrays, and
// the loss kernel advances the batch and the Adam step count t (with the
// bias corrections c1 = 1 / (1 - 0.9^t), c2 = 1 / (1 - 0.999^t)).
struct TrainState {
    uint64_t step;
    uint32_t batch, n_batches;
    float c1, c2;
    uint32_t pad[2];
};

__global__ void set_state_kernel(TrainState* st, uint64_t step, uint32_t n_batches) {
    st->step = step;
    st->batch = 0;
    st->n_batches = n_batches;
    st->c1 = st->c2 = 0.f;
}

// y = bf16(x) for the n elements of batch st->batch (stride n), or of x
// itself when st is NULL
__global__ void cvt_bf16_kernel(const float* x, uint16_t* y, uint64_t n, const TrainState* st) {
    if (st) x += (uint64_t)st->batch * n;
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
        y[i] = f2bf(x[i]);
}

// softmax cross-entropy, one wave per row; dz = (softmax - onehot) / B;
// labels of batch st->batch
__global__ void __launch_bounds__(256) xent_kernel(const float* z, const int32_t* y, uint32_t rows, uint32_t C,
                                                   float inv_b, float* dz_f, float* loss_row, const TrainState* st) {
    const uint32_t r = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
    if (r >= rows) return;
    y += (uint64_t)st->batch * rows;
    const float* zr = z + (uint64_t)r * C;
    float mx = -INFINITY;
    for (uint32_t c = lane; c < C; c += 64) mx = fmaxf(mx, zr[c]);
    for (int o = 32; o > 0; o >>= 1) mx = fmaxf(mx, __shfl_xor(mx, o));
    float sum = 0.f;
    for (uint32_t c = lane; c < C; c += 64) sum += expf(zr[c] - mx);
    for (int o = 32; o > 0; o >>= 1) sum += __shfl_xor(sum, o);
    const int32_t lab = y[r];
    const bool ok = lab >= 0 && (uint32_t)lab < C;   // an out-of-range label yields a NaN loss
    const float inv = 1.f / sum;
    for (uint32_t c = lane; c < C; c += 64) {
        float d = expf(zr[c] - mx) * inv - ((int32_t)c == lab ? 1.f : 0.f);
        d *= inv_b;
        dz_f[(uint64_t)r * C + c] = d;
    }
    if (lane == 0) loss_row[r] = ok ? logf(sum) + mx - zr[lab] : NAN;
}

// out[c] = sum over rows of G[r][c]; 64 columns per block, 4 row phases
__global__ void __launch_bounds__(256) colsum_kernel(const float* G, uint32_t rows, uint32_t cols, float* out) {
    __shared__ float part[256];
    const uint32_t c = blockIdx.x * 64 + (threadIdx.x & 63), ph = threadIdx.x >> 6;
    float s = 0.f;
    if (c < cols)
        for (uint32_t r = ph; r < rows; r += 4) s += G[(uint64_t)r * cols + c];
    part[threadIdx.x] = s;
    __syncthreads();
    if (ph == 0 && c < cols) out[c] = (part[threadIdx.x] + part[threadIdx.x + 64]) + (part[threadIdx.x + 128] + part[threadIdx.x + 192]);
}

// mean loss of the batch; then (every read of the batch's samples is done)
// the next batch and the next Adam step
__global__ void __launch_bounds__(256) mean_kernel(const float* v, uint32_t n, float* out, TrainState* st) {
    __shared__ float part[256];
    float s = 0.f;
    for (uint32_t i = threadIdx.x; i < n; i += 256) s += v[i];
    part[threadIdx.x] = s;
    __syncthreads();
    for (uint32_t k = 128; k > 0; k >>= 1) {
        if (threadIdx.x < k) part[threadIdx.x] += part[threadIdx.x + k];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        out[0] = part[0] / (float)n;
        const uint32_t nb = st->batch + 1;
        st->batch = nb >= st->n_batches ? 0u : nb;
        const uint64_t t = st->step + 1;
        st->step = t;
        st->c1 = (float)(1.0 / (1.0 - pow(0.9, (double)t)));
        st->c2 = (float)(1.0 / (1.0 - pow(0.999, (double)t)));
    }
}

struct AdamSeg {
    float* p;
    float* m;
    float* v;
    const float* g;
    uint16_t* wb;   // bf16 copy of the weights, or NULL (biases)
    uint64_t n;
};
struct AdamArgs {
    AdamSeg seg[6];
    float lr, b1, b2, eps;
    const TrainState* st;   // bias corrections of the step
};

__global__ void __launch_bounds__(256) adam_kernel(AdamArgs a) {
    const AdamSeg s = a.seg[blockIdx.y];
    const float c1 = a.st->c1, c2 = a.st->c2;
    for (uint64_t i = blockIdx.x * 256ull + threadIdx.x; i < s.n; i += (uint64_t)gridDim.x * 256) {
        const float g = s.g[i];
        const float m = a.b1 * s.m[i] + (1.f - a.b1) * g;
        const float v = a.b2 * s.v[i] + (1.f - a.b2) * g * g;
        s.m[i] = m;
        s.v[i] = v;
        const float p = s.p[i] - a.lr * (m * c1) / (sqrtf(v * c2) + a.eps);
        s.p[i] = p;
        if (s.wb) s.wb[i] = f2bf(p);
    }
}

// weights uniform in [-1/sqrt(fan_in), 1/sqrt(fan_in)) from Philox
// (counter = (i, tensor, 0, 0x494E4954)), biases zero
__global__ void init_kernel(float* p, uint16_t* wb, uint64_t n, uint32_t which, float bound, uint32_t k0,
                            uint32_t k1) {
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x) {
        float v = 0.f;
        if (wb) {
            uint32_t o[4];
            philox4((uint32_t)i, which, 0, 0x494E4954u, k0, k1, o);
            const float u = (float)(o[0] >> 8) * (1.f / 16777216.f);
            v = (2.f * u - 1.f) * bound;
            wb[i] = f2bf(v);
        }
        p[i] = v;
    }
}

__global__ void refresh_bf16_kernel(const float* p, uint16_t* wb, uint64_t n) {
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
        wb[i] = f2bf(p[i]);
}

// top-k columns of each row (largest first, ties to the lower index)
__global__ void __launch_bounds__(64) topk_kernel(const float* z, uint32_t C, uint32_t k, int32_t* idx) {
    const uint32_t r = blockIdx.x, lane = threadIdx.x;
    const float* zr = z + (uint64_t)r * C;
    uint64_t taken = 0;   // bit t: column lane + 64 t already chosen
    for (uint32_t j = 0; j < k; ++j) {
        float bv = -INFINITY;
        int32_t bi = 0x7FFFFFFF;
        for (uint32_t c = lane, t = 0; c < C; c += 64, ++t) {
            if ((taken >> t) & 1) continue;
            const float v = zr[c];
            if (v > bv || (v == bv && (int32_t)c < bi)) {
                bv = v;
                bi = (int32_t)c;
            }
        }
        for (int o = 32; o > 0; o >>= 1) {
            const float ov = __shfl_xor(bv, o);
            const int32_t oi = __shfl_xor(bi, o);
            if (ov > bv || (ov == bv && oi < bi)) {
                bv = ov;
                bi = oi;
            }
        }
        if (lane == 0) idx[(uint64_t)r * k + j] = bi;
        if (bi != 0x7FFFFFFF && (uint32_t)bi % 64 == lane) taken |= 1ull << ((uint32_t)bi / 64);
    }
}

static uint32_t blocks_for(uint64_t n, uint32_t per = 256, uint32_t cap = 4096) {
    return (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>(cap, (n + per - 1) / per));
}

// ---------------------------------------------------- grid replay bank ---
// Steady bits of the grid probes for "slots" (model, base offset), replayed
// into one bitmap; slot s's probe p starts at bit s * slot_bits + pbit[p].
struct GridTable {
    std::vector<DevProbe> dp;      // kMaxBase4 copies of the grid: base 4 * (index / 768)
    std::vector<uint64_t> len;
    std::vector<uint64_t> pbit;    // per grid probe, word aligned
    std::vector<uint32_t> L;
    uint64_t slot_bits = 0;
};

static int grid_table(GridTable* t) {
    if (!t->dp.empty()) return PCHASE_OK;
    t->dp.resize((size_t)kMaxBase4 * kIn);
    t->len.resize(t->dp.size());
    for (uint32_t b4 = 0; b4 < kMaxBase4; ++b4)
        for (uint32_t p = 0; p < kIn; ++p) {
            pchase_probe pr;
            grid_probe(p, 4ull * b4, &pr);
            int rc = check_probe(pr, &t->dp[b4 * kIn + p], &t->len[b4 * kIn + p], p);
            if (rc) return rc;
        }
    t->pbit.resize(kIn);
    t->L.resize(kIn);
    uint64_t off = 0;
    for (uint32_t p = 0; p < kIn; ++p) {
        t->pbit[p] = off;
        t->L[p] = t->dp[p].L;
        off += (t->len[p] + 31) / 32 * 32;
    }
    t->slot_bits = off;
    return PCHASE_OK;
}

struct Slot {
    uint32_t model, base4;
};

// Replays the grid for `slots` into bank (cleared first).
static int replay_slots(Workspace* ws, const GridTable& gt, const std::vector<DevModel>& dm,
                        const std::vector<Slot>& slots, uint32_t* bank, hipStream_t stream) {
    std::vector<uint32_t> order(slots.size());
    for (uint32_t i = 0; i < slots.size(); ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](uint32_t x, uint32_t y) { return slots[x].model < slots[y].model; });
    std::vector<SweepJob> jobs;
    jobs.reserve(slots.size() * kIn);
    for (uint32_t oi : order) {
        for (uint32_t p = 0; p < kIn; ++p) {
            SweepJob j{};
            j.model = slots[oi].model;
            j.probe = slots[oi].base4 * kIn + p;
            j.out = (uint32_t)(jobs.size());
            j.trace_id = p;
            j.count_from = gt.L[p];
            j.bitoff = (oi * gt.slot_bits + gt.pbit[p]) / 32;   // word offset (both terms are word aligned)
            jobs.push_back(j);
        }
    }
    return replay_jobs(ws, dm, gt.dp, gt.len, jobs, bank, (slots.size() * gt.slot_bits) / 32, stream);
}

// bank + per-slot/row device arrays in the workspace's mlp buffer
struct BankLayout {
    uint32_t* bank;
    uint64_t* pbit;
    uint32_t* L;
    uint8_t* rows;   // row arrays follow
};

static int bank_alloc(Workspace* ws, const GridTable& gt, uint64_t n_slots, size_t row_bytes, BankLayout* bl,
                      hipStream_t stream) {
    const size_t bank_bytes = ((n_slots * gt.slot_bits / 32 + 1) * 4 + 255) / 256 * 256;
    const size_t tab_bytes = (kIn * 12 + 255) / 256 * 256;
    hipError_t e = ws->mlp.ensure(bank_bytes + tab_bytes + row_bytes);
    if (e != hipSuccess) return set_error(PCHASE_ENOMEM, "grid bank of %llu bytes: %s",
                                          (unsigned long long)bank_bytes, hipGetErrorString(e));
    uint8_t* b = ws->mlp.as<uint8_t>();
    bl->bank = reinterpret_cast<uint32_t*>(b);
    bl->pbit = reinterpret_cast<uint64_t*>(b + bank_bytes);
    bl->L = reinterpret_cast<uint32_t*>(bl->pbit + kIn);
    bl->rows = b + bank_bytes + tab_bytes;
    PC_HIP(hipMemcpyAsync(bl->pbit, gt.pbit.data(), kIn * 8, hipMemcpyHostToDevice, stream));
    PC_HIP(hipMemcpyAsync(bl->L, gt.L.data(), kIn * 4, hipMemcpyHostToDevice, stream));
    return PCHASE_OK;
}

static hipError_t launch_features(const FeatArgs& fa, hipStream_t s) {
    for (uint32_t r0 = 0; r0 < fa.rows; r0 += 65535) {
        dim3 grid((fa.n_probes + 3) / 4, std::min<uint32_t>(65535, fa.rows - r0));
        hipLaunchKernelGGL(feature_kernel, grid, dim3(256), 0, s, fa, r0);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

constexpr uint64_t kBankBytesMax = 2ull << 30;

}  // namespace pc

using namespace pc;

// ---------------------------------------------------------------- net ---
struct pchase_mlp {
    int device = -1;
    uint32_t n_out = 0;
    uint64_t steps = 0;
    uint64_t count[6] = {};
    DevBuf params;
    float* p[6] = {};
    float* m[6] = {};
    float* v[6] = {};
    float* g[6] = {};
    uint16_t* wb[3] = {};
    pc::TrainState* st = nullptr;
    DevBuf act;
    uint32_t act_batch = 0;
    uint16_t* xb = nullptr;
    float *h1 = nullptr, *h2 = nullptr, *z = nullptr, *dz_f = nullptr, *dh2_f = nullptr, *dh1_f = nullptr;
    float *loss_row = nullptr, *loss = nullptr;
    int32_t* idx = nullptr;
    // captured training step (replayed once per batch by pchase_mlp_train)
    hipGraphExec_t gexec = nullptr;
    std::string gkey;
    ~pchase_mlp() {
        if (gexec) (void)hipGraphExecDestroy(gexec);
        params.release();
        act.release();
    }
};

namespace pc {

static int ensure_act(pchase_mlp* net, uint32_t batch) {
    if (batch <= net->act_batch) return PCHASE_OK;
    const uint64_t B = batch, C = net->n_out;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off += (bytes + 255) / 256 * 256;
        return o;
    };
    const size_t o_xb = take(B * kIn * 2), o_h1 = take(B * kHid * 4), o_h2 = take(B * kHid * 4);
    const size_t o_z = take(B * C * 4), o_dzf = take(B * C * 4);
    const size_t o_dh2f = take(B * kHid * 4), o_dh1f = take(B * kHid * 4);
    const size_t o_lr = take(B * 4), o_l = take(256), o_idx = take(B * kMaxTopK * 4);
    hipError_t e = net->act.ensure(off);
    if (e != hipSuccess) return set_error(PCHASE_ENOMEM, "activations for batch %u: %s", batch, hipGetErrorString(e));
    uint8_t* b = net->act.as<uint8_t>();
    net->xb = reinterpret_cast<uint16_t*>(b + o_xb);
    net->h1 = reinterpret_cast<float*>(b + o_h1);
    net->h2 = reinterpret_cast<float*>(b + o_h2);
    net->z = reinterpret_cast<float*>(b + o_z);
    net->dz_f = reinterpret_cast<float*>(b + o_dzf);
    net->dh2_f = reinterpret_cast<float*>(b + o_dh2f);
    net->dh1_f = reinterpret_cast<float*>(b + o_dh1f);
    net->loss_row = reinterpret_cast<float*>(b + o_lr);
    net->loss = reinterpret_cast<float*>(b + o_l);
    net->idx = reinterpret_cast<int32_t*>(b + o_idx);
    net->act_batch = batch;
    return PCHASE_OK;
}

// A(m, k) at element a_m * m + a_k * k, B(k, n) at b_k * k + b_n * n; the
// operand given as fp32 (Af / Bf) is split, the bf16 one is taken as is
static GemmArgs gargs(const uint16_t* A, const float* Af, int64_t a_m, int64_t a_k, const uint16_t* B,
                      const float* Bf, int64_t b_k, int64_t b_n, uint32_t M, uint32_t N, uint32_t K, int64_t ld,
                      float* out) {
    GemmArgs g{};
    g.A = A;
    g.Af = Af;
    g.B = B;
    g.Bf = Bf;
    g.a_m = a_m;
    g.a_k = a_k;
    g.b_k = b_k;
    g.b_n = b_n;
    g.M = M;
    g.N = N;
    g.K = K;
    g.alpha = 1.f;
    g.ld = ld;
    g.out_f = out;
    return g;
}

// forward of xb (already bf16 in net->xb) into net->z; the hidden
// activations stay fp32 and enter the next product split
static hipError_t forward_net(const pchase_mlp* net, uint32_t B, hipStream_t s) {
    const uint32_t C = net->n_out;
    GemmArgs g = gargs(net->xb, nullptr, kIn, 1, net->wb[0], nullptr, 1, kIn, B, kHid, kIn, kHid, net->h1);
    g.bias = net->p[1];
    g.relu = 1;
    hipError_t e = gemm(g, s);
    if (e != hipSuccess) return e;
    g = gargs(nullptr, net->h1, kHid, 1, net->wb[1], nullptr, 1, kHid, B, kHid, kHid, kHid, net->h2);
    g.bias = net->p[3];
    g.relu = 1;
    if ((e = gemm(g, s)) != hipSuccess) return e;
    g = gargs(nullptr, net->h2, kHid, 1, net->wb[2], nullptr, 1, kHid, B, C, kHid, C, net->z);
    g.bias = net->p[5];
    return gemm(g, s);
}

static hipError_t to_bf16(const float* x, uint16_t* y, uint64_t n, const TrainState* st, hipStream_t s) {
    hipLaunchKernelGGL(cvt_bf16_kernel, dim3(blocks_for(n)), dim3(256), 0, s, x, y, n, st);
    return hipGetLastError();
}

// One training step on batch net->st->batch of (x, y), B rows per batch;
// launches only (capturable): nothing on the host depends on the step.
static int enqueue_step(pchase_mlp* net, const float* x, const int32_t* y, uint32_t B, float lr, hipStream_t s) {
    const uint32_t C = net->n_out;
    PC_HIP(to_bf16(x, net->xb, (uint64_t)B * kIn, net->st, s));
    PC_HIP(forward_net(net, B, s));
    hipLaunchKernelGGL(xent_kernel, dim3((B + 3) / 4), dim3(256), 0, s, net->z, y, B, C, 1.f / (float)B, net->dz_f,
                       net->loss_row, net->st);
    PC_HIP(hipGetLastError());
    hipLaunchKernelGGL(mean_kernel, dim3(1), dim3(256), 0, s, net->loss_row, B, net->loss, net->st);
    PC_HIP(hipGetLastError());
    // layer 3: dW3 = dz^T h2, db3 = colsum dz, dh2 = (dz W3) * [h2 > 0]
    GemmArgs g = gargs(nullptr, net->dz_f, 1, C, nullptr, net->h2, kHid, 1, C, kHid, B, kHid, net->g[4]);
    PC_HIP(gemm(g, s));
    hipLaunchKernelGGL(colsum_kernel, dim3((C + 63) / 64), dim3(256), 0, s, net->dz_f, B, C, net->g[5]);
    PC_HIP(hipGetLastError());
    g = gargs(nullptr, net->dz_f, C, 1, net->wb[2], nullptr, kHid, 1, B, kHid, C, kHid, net->dh2_f);
    g.mask = net->h2;
    PC_HIP(gemm(g, s));
    // layer 2
    g = gargs(nullptr, net->dh2_f, 1, kHid, nullptr, net->h1, kHid, 1, kHid, kHid, B, kHid, net->g[2]);
    PC_HIP(gemm(g, s));
    hipLaunchKernelGGL(colsum_kernel, dim3(kHid / 64), dim3(256), 0, s, net->dh2_f, B, kHid, net->g[3]);
    PC_HIP(hipGetLastError());
    g = gargs(nullptr, net->dh2_f, kHid, 1, net->wb[1], nullptr, kHid, 1, B, kHid, kHid, kHid, net->dh1_f);
    g.mask = net->h1;
    PC_HIP(gemm(g, s));
    // layer 1 (the input is exactly bf16)
    g = gargs(nullptr, net->dh1_f, 1, kHid, net->xb, nullptr, kIn, 1, kHid, kIn, B, kIn, net->g[0]);
    PC_HIP(gemm(g, s));
    hipLaunchKernelGGL(colsum_kernel, dim3(kHid / 64), dim3(256), 0, s, net->dh1_f, B, kHid, net->g[1]);
    PC_HIP(hipGetLastError());
    // Adam
    AdamArgs a{};
    for (int i = 0; i < 6; ++i) {
        a.seg[i].p = net->p[i];
        a.seg[i].m = net->m[i];
        a.seg[i].v = net->v[i];
        a.seg[i].g = net->g[i];
        a.seg[i].wb = (i % 2 == 0) ? net->wb[i / 2] : nullptr;
        a.seg[i].n = net->count[i];
    }
    a.lr = lr;
    a.b1 = 0.9f;
    a.b2 = 0.999f;
    a.eps = 1e-8f;
    a.st = net->st;
    hipLaunchKernelGGL(adam_kernel, dim3(64, 6), dim3(256), 0, s, a);
    PC_HIP(hipGetLastError());
    return PCHASE_OK;
}

// Training state for a run of steps over n_batches batches, from the
// host's step count.
static hipError_t begin_steps(pchase_mlp* net, uint32_t n_batches, hipStream_t s) {
    hipLaunchKernelGGL(set_state_kernel, dim3(1), dim3(1), 0, s, net->st, net->steps, n_batches);
    return hipGetLastError();
}

static int check_net(const pchase_mlp* net) {
    if (!net) return set_error(PCHASE_EINVAL, "net is NULL");
    int dev = 0;
    PC_HIP(hipGetDevice(&dev));
    if (dev != net->device) return set_error(PCHASE_EINVAL, "net lives on device %d, current device is %d", net->device, dev);
    return PCHASE_OK;
}

// ------------------------------------------------- learned inference ---
int infer_learned(Workspace* ws, const pchase_observation* obs, const pchase_model* cands, uint32_t n_cands,
                  const std::vector<DevProbe>& dp, const std::vector<uint64_t>& len,
                  const std::vector<uint64_t>& cf, const std::vector<uint64_t>& bitoff, const uint32_t* bits,
                  uint32_t topk, const pchase_mlp* cnet, std::vector<uint8_t>* allow, bool* on_grid,
                  hipStream_t stream) {
    (void)cands;
    (void)cf;
    (void)dp;
    (void)len;
    pchase_mlp* net = const_cast<pchase_mlp*>(cnet);
    int rc = check_net(net);
    if (rc) return rc;
    if (net->n_out != n_cands)
        return set_error(PCHASE_EINVAL, "net proposes %u classes for %u candidates", net->n_out, n_cands);
    if (topk > kMaxTopK || topk > n_cands) return set_error(PCHASE_EINVAL, "topk %u out of range", topk);
    *on_grid = obs->n_probes == kIn;
    for (uint32_t p = 0; *on_grid && p < kIn; ++p) {
        pchase_probe g;
        grid_probe(p, 0, &g);
        const pchase_probe& o = obs->probes[p];
        *on_grid = o.n_bytes == g.n_bytes && o.s_bytes == g.s_bytes && o.passes == g.passes && o.j0 == 0 &&
                   o.elem_bytes == 4 && (!obs->count_from || obs->count_from[p] == dp[p].L);
    }
    if (!*on_grid) return PCHASE_OK;
    rc = ensure_act(net, 1);
    if (rc) return rc;
    // features of the observation, then the forward pass
    const size_t need = kIn * 8 + kIn * 4 + 256 + kIn * 4;
    hipError_t e = ws->aux.ensure(need);
    if (e != hipSuccess) {
        if (ws->arena) return set_error(PCHASE_ERANGE, "the learned proposal's scratch does not fit the plan's memory");
        return set_error(PCHASE_ENOMEM, "learned scratch: %s", hipGetErrorString(e));
    }
    uint64_t* d_pbit = ws->aux.as<uint64_t>();
    uint32_t* d_L = reinterpret_cast<uint32_t*>(d_pbit + kIn);
    float* d_x = reinterpret_cast<float*>(reinterpret_cast<uint8_t*>(d_L) + kIn * 4 + 256);
    std::vector<uint32_t> L(kIn);
    std::vector<uint64_t> pbit(kIn);
    for (uint32_t p = 0; p < kIn; ++p) {
        L[p] = dp[p].L;
        pbit[p] = bitoff[p] * 32;   // observation offsets are in words
    }
    CopyFence fence(stream);
    PC_HIP(hipMemcpyAsync(d_pbit, pbit.data(), kIn * 8, hipMemcpyHostToDevice, stream));
    PC_HIP(hipMemcpyAsync(d_L, L.data(), kIn * 4, hipMemcpyHostToDevice, stream));
    FeatArgs fa{};
    fa.bits = bits;
    fa.probe_bit = d_pbit;
    fa.probe_L = d_L;
    fa.rows = 1;
    fa.n_probes = kIn;
    fa.x = d_x;
    PC_HIP(launch_features(fa, stream));
    PC_HIP(to_bf16(d_x, net->xb, kIn, nullptr, stream));
    PC_HIP(forward_net(net, 1, stream));
    hipLaunchKernelGGL(topk_kernel, dim3(1), dim3(64), 0, stream, net->z, n_cands, topk, net->idx);
    PC_HIP(hipGetLastError());
    int32_t* hr = static_cast<int32_t*>(ws->host_res);
    PC_HIP(hipMemcpyAsync(hr, net->idx, topk * 4, hipMemcpyDeviceToHost, stream));
    PC_HIP(hipStreamSynchronize(stream));
    fence.done();
    allow->assign(n_cands, 0);
    for (uint32_t j = 0; j < topk; ++j)
        if (hr[j] >= 0 && (uint32_t)hr[j] < n_cands) (*allow)[hr[j]] = 1;
    return PCHASE_OK;
}

}  // namespace pc

// --------------------------------------------------------------- C ABI ---
extern "C" int pchase_mlp_grid(pchase_probe* probes, uint64_t base_offset) {
    if (!probes) return set_error(PCHASE_EINVAL, "probes is NULL");
    if (base_offset % 4 || base_offset >= (1ull << 33)) return set_error(PCHASE_EINVAL, "base offset must be a multiple of 4 below 2^33");
    for (uint32_t p = 0; p < kIn; ++p) grid_probe(p, base_offset, &probes[p]);
    return PCHASE_OK;
}

extern "C" int pchase_mlp_create(uint32_t n_out, uint64_t seed, pchase_mlp** out) {
    if (!out) return set_error(PCHASE_EINVAL, "out is NULL");
    *out = nullptr;
    if (n_out == 0 || n_out > 4096) return set_error(PCHASE_EINVAL, "n_out must be in 1..4096");
    Workspace* ws;
    std::unique_lock<std::mutex> lk;
    int rc = workspace(&ws, &lk);
    if (rc) return rc;
    std::unique_ptr<pchase_mlp> net(new pchase_mlp());
    net->device = ws->device;
    net->n_out = n_out;
    const uint64_t cnt[6] = {(uint64_t)kHid * kIn, kHid, (uint64_t)kHid * kHid, kHid, (uint64_t)n_out * kHid, n_out};
    size_t off = 0;
    size_t o[6][4], ow[3];
    for (int i = 0; i < 6; ++i) {
        net->count[i] = cnt[i];
        for (int k = 0; k < 4; ++k) {
            o[i][k] = off;
            off += (cnt[i] * 4 + 255) / 256 * 256;
        }
    }
    for (int i = 0; i < 3; ++i) {
        ow[i] = off;
        off += (cnt[2 * i] * 2 + 255) / 256 * 256;
    }
    const size_t o_st = off;
    off += 256;
    hipError_t e = net->params.ensure(off);
    if (e != hipSuccess) return set_error(PCHASE_ENOMEM, "parameters: %s", hipGetErrorString(e));
    uint8_t* b = net->params.as<uint8_t>();
    for (int i = 0; i < 6; ++i) {
        net->p[i] = reinterpret_cast<float*>(b + o[i][0]);
        net->m[i] = reinterpret_cast<float*>(b + o[i][1]);
        net->v[i] = reinterpret_cast<float*>(b + o[i][2]);
        net->g[i] = reinterpret_cast<float*>(b + o[i][3]);
    }
    for (int i = 0; i < 3; ++i) net->wb[i] = reinterpret_cast<uint16_t*>(b + ow[i]);
    net->st = reinterpret_cast<TrainState*>(b + o_st);
    PC_HIP(hipMemset(b, 0, off));
    const uint32_t fan_in[3] = {kIn, kHid, kHid};
    for (int i = 0; i < 6; ++i) {
        const bool w = i % 2 == 0;
        hipLaunchKernelGGL(init_kernel, dim3(blocks_for(cnt[i])), dim3(256), 0, 0, net->p[i],
                           w ? net->wb[i / 2] : nullptr, cnt[i], (uint32_t)i,
                           w ? 1.f / std::sqrt((float)fan_in[i / 2]) : 0.f, (uint32_t)seed, (uint32_t)(seed >> 32));
        PC_HIP(hipGetLastError());
    }
    PC_HIP(hipDeviceSynchronize());
    *out = net.release();
    return PCHASE_OK;
}

extern "C" void pchase_mlp_destroy(pchase_mlp* net) {
    if (!net) return;
    int cur = 0;
    const bool have = hipGetDevice(&cur) == hipSuccess;
    if (have && cur != net->device) (void)hipSetDevice(net->device);
    delete net;
    if (have) (void)hipSetDevice(cur);
}

extern "C" int pchase_mlp_features(const pchase_model* models, uint32_t n, float* x_dev, hipStream_t stream) {
    if (n == 0) return PCHASE_OK;
    if (!models || !x_dev) return set_error(PCHASE_EINVAL, "models and x_dev must not be NULL");
    std::vector<DevModel> dm(n);
    for (uint32_t i = 0; i < n; ++i) {
        int rc = check_model(models[i], &dm[i], i);
        if (rc) return rc;
    }
    GridTable gt;
    int rc = grid_table(&gt);
    if (rc) return rc;
    Workspace* ws;
    std::unique_lock<std::mutex> lk;
    rc = workspace(&ws, &lk);
    if (rc) return rc;
    const uint32_t per = (uint32_t)std::max<uint64_t>(1, kBankBytesMax / (gt.slot_bits / 8));
    CopyFence fence(stream);   // the grid table's arrays
    for (uint32_t c0 = 0; c0 < n; c0 += per) {
        const uint32_t cn = std::min(per, n - c0);
        std::vector<Slot> slots(cn);
        std::vector<uint64_t> bit0(cn);
        for (uint32_t i = 0; i < cn; ++i) {
            slots[i] = {c0 + i, 0};
            bit0[i] = i * gt.slot_bits;
        }
        CopyFence chunk(stream);
        BankLayout bl;
        rc = bank_alloc(ws, gt, cn, (size_t)cn * 8 + 256, &bl, stream);
        if (rc) return rc;
        rc = replay_slots(ws, gt, dm, slots, bl.bank, stream);
        if (rc) return rc;
        uint64_t* d_bit0 = reinterpret_cast<uint64_t*>(bl.rows);
        PC_HIP(hipMemcpyAsync(d_bit0, bit0.data(), cn * 8, hipMemcpyHostToDevice, stream));
        FeatArgs fa{};
        fa.bits = bl.bank;
        fa.row_bit0 = d_bit0;
        fa.probe_bit = bl.pbit;
        fa.probe_L = bl.L;
        fa.rows = cn;
        fa.n_probes = kIn;
        fa.x = x_dev + (uint64_t)c0 * kIn;
        PC_HIP(launch_features(fa, stream));
        PC_HIP(hipStreamSynchronize(stream));   // the bank is reused by the next chunk
        chunk.done();
    }
    fence.done();
    return PCHASE_OK;
}

extern "C" int pchase_mlp_labels(const pchase_model* models, uint32_t n, int32_t* labels, hipStream_t stream) {
    if (n == 0) return PCHASE_OK;
    if (!models || !labels) return set_error(PCHASE_EINVAL, "models and labels must not be NULL");
    std::vector<DevModel> dm(n);
    for (uint32_t i = 0; i < n; ++i) {
        int rc = check_model(models[i], &dm[i], i);
        if (rc) return rc;
    }
    GridTable gt;
    int rc = grid_table(&gt);
    if (rc) return rc;
    if ((uint64_t)n * (gt.slot_bits / 8) > kBankBytesMax)
        return set_error(PCHASE_ERANGE, "%u models exceed the %llu-byte grid bank", n, (unsigned long long)kBankBytesMax);
    Workspace* ws;
    std::unique_lock<std::mutex> lk;
    rc = workspace(&ws, &lk);
    if (rc) return rc;
    std::vector<uint64_t> sig(n);
    CopyFence fence(stream);
    BankLayout bl;
    rc = bank_alloc(ws, gt, n, (size_t)n * 8 + 256, &bl, stream);
    if (rc) return rc;
    std::vector<Slot> slots(n);
    for (uint32_t i = 0; i < n; ++i) slots[i] = {i, 0};
    rc = replay_slots(ws, gt, dm, slots, bl.bank, stream);
    if (rc) return rc;
    uint64_t* d_sig = reinterpret_cast<uint64_t*>(bl.rows);
    hipLaunchKernelGGL(signature_kernel, dim3(n), dim3(256), 0, stream, bl.bank, gt.slot_bits, bl.pbit, bl.L, kIn, d_sig);
    PC_HIP(hipGetLastError());
    PC_HIP(hipMemcpyAsync(sig.data(), d_sig, n * 8, hipMemcpyDeviceToHost, stream));
    PC_HIP(hipStreamSynchronize(stream));
    // exact check of every earlier model with the same signature
    std::unordered_map<uint64_t, std::vector<uint32_t>> groups;
    std::vector<uint32_t> pairs;
    for (uint32_t i = 0; i < n; ++i) {
        auto& g = groups[sig[i]];
        for (uint32_t j : g) {
            pairs.push_back(i);
            pairs.push_back(j);
        }
        g.push_back(i);
    }
    for (uint32_t i = 0; i < n; ++i) labels[i] = (int32_t)i;
    const uint32_t np = (uint32_t)(pairs.size() / 2);
    if (np) {
        hipError_t e = ws->aux.ensure((size_t)np * 12 + 256);
        if (e != hipSuccess) return set_error(PCHASE_ENOMEM, "label pairs: %s", hipGetErrorString(e));
        uint32_t* d_pairs = ws->aux.as<uint32_t>();
        uint32_t* d_diff = d_pairs + 2 * (size_t)np;
        std::vector<uint32_t> diff(np);
        CopyFence block(stream);
        PC_HIP(hipMemcpyAsync(d_pairs, pairs.data(), (size_t)np * 8, hipMemcpyHostToDevice, stream));
        hipLaunchKernelGGL(pair_differ_kernel, dim3(np), dim3(256), 0, stream, bl.bank, gt.slot_bits, bl.pbit, bl.L, kIn,
                           d_pairs, d_diff);
        PC_HIP(hipGetLastError());
        PC_HIP(hipMemcpyAsync(diff.data(), d_diff, (size_t)np * 4, hipMemcpyDeviceToHost, stream));
        PC_HIP(hipStreamSynchronize(stream));
        block.done();
        for (uint32_t k = 0; k < np; ++k) {
            const uint32_t i = pairs[2 * k], j = pairs[2 * k + 1];
            if (!diff[k] && (int32_t)j < labels[i]) labels[i] = (int32_t)j;
        }
    }
    return PCHASE_OK;
}

extern "C" int pchase_mlp_samples(const pchase_model* models, uint32_t n_models, const int32_t* class_of_model,
                                  uint64_t first, uint32_t n, uint64_t seed, uint32_t rho_q16, float* x_dev,
                                  int32_t* labels_dev, hipStream_t stream) {
    if (n == 0) return PCHASE_OK;
    if (!models || n_models == 0 || !class_of_model || !x_dev || !labels_dev)
        return set_error(PCHASE_EINVAL, "models, class_of_model, x_dev and labels_dev must be given");
    if (rho_q16 > 65535) return set_error(PCHASE_EINVAL, "rho_q16 must be below 65536");
    if (first + n < first || ((first + n - 1) >> 63)) return set_error(PCHASE_ERANGE, "sample index range too large");
    std::vector<DevModel> dm(n_models);
    for (uint32_t i = 0; i < n_models; ++i) {
        int rc = check_model(models[i], &dm[i], i);
        if (rc) return rc;
        if (models[i].line_bytes > 4 * kMaxBase4)
            return set_error(PCHASE_EINVAL, "model %u: line of %u bytes, samples support lines up to %u bytes", i,
                             models[i].line_bytes, 4 * kMaxBase4);
    }
    GridTable gt;
    int rc = grid_table(&gt);
    if (rc) return rc;
    // per-sample draws: model, base offset, flip threshold
    struct Draw {
        uint32_t key, thr, out;
        uint64_t i;
    };
    std::vector<Draw> d(n);
    std::vector<int32_t> lab(n);
    const uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
    for (uint32_t r = 0; r < n; ++r) {
        const uint64_t i = first + r;
        uint32_t o[4];
        philox4((uint32_t)i, (uint32_t)(i >> 32), 0, 0, k0, k1, o);
        const uint32_t mi = o[0] % n_models;
        const uint32_t b4 = (uint32_t)(models[mi].line_bytes / 4);
        const uint32_t base4 = o[1] % b4;
        d[r] = {mi * kMaxBase4 + base4, o[2] % (rho_q16 + 1), r, i};
        lab[r] = class_of_model[mi];
    }
    std::stable_sort(d.begin(), d.end(), [](const Draw& x, const Draw& y) { return x.key < y.key; });
    Workspace* ws;
    std::unique_lock<std::mutex> lk;
    rc = workspace(&ws, &lk);
    if (rc) return rc;
    CopyFence fence(stream);   // the labels and the grid table's arrays
    PC_HIP(hipMemcpyAsync(labels_dev, lab.data(), (size_t)n * 4, hipMemcpyHostToDevice, stream));
    const uint32_t per = (uint32_t)std::max<uint64_t>(1, kBankBytesMax / (gt.slot_bits / 8));
    size_t r0 = 0;
    while (r0 < n) {
        // the next run of samples whose distinct slots fit the bank
        std::vector<Slot> slots;
        std::vector<uint64_t> bit0;
        std::vector<uint32_t> thr, out;
        std::vector<uint64_t> smp;
        size_t r = r0;
        while (r < n) {
            if (slots.empty() || d[r].key != d[r - 1].key) {
                if (slots.size() == per) break;
                slots.push_back({d[r].key / kMaxBase4, d[r].key % kMaxBase4});
            }
            bit0.push_back((slots.size() - 1) * gt.slot_bits);
            thr.push_back(d[r].thr);
            out.push_back(d[r].out);
            smp.push_back(d[r].i);
            ++r;
        }
        const size_t rows = r - r0;
        CopyFence chunk(stream);
        BankLayout bl;
        rc = bank_alloc(ws, gt, slots.size(), rows * 24 + 1024, &bl, stream);
        if (rc) return rc;
        rc = replay_slots(ws, gt, dm, slots, bl.bank, stream);
        if (rc) return rc;
        uint64_t* d_bit0 = reinterpret_cast<uint64_t*>(bl.rows);
        uint64_t* d_smp = d_bit0 + rows;
        uint32_t* d_thr = reinterpret_cast<uint32_t*>(d_smp + rows);
        uint32_t* d_out = d_thr + rows;
        PC_HIP(hipMemcpyAsync(d_bit0, bit0.data(), rows * 8, hipMemcpyHostToDevice, stream));
        PC_HIP(hipMemcpyAsync(d_smp, smp.data(), rows * 8, hipMemcpyHostToDevice, stream));
        PC_HIP(hipMemcpyAsync(d_thr, thr.data(), rows * 4, hipMemcpyHostToDevice, stream));
        PC_HIP(hipMemcpyAsync(d_out, out.data(), rows * 4, hipMemcpyHostToDevice, stream));
        FeatArgs fa{};
        fa.bits = bl.bank;
        fa.row_bit0 = d_bit0;
        fa.probe_bit = bl.pbit;
        fa.probe_L = bl.L;
        fa.row_thr = d_thr;
        fa.row_sample = d_smp;
        fa.row_out = d_out;
        fa.rows = (uint32_t)rows;
        fa.n_probes = kIn;
        fa.key0 = k0;
        fa.key1 = k1;
        fa.x = x_dev;
        PC_HIP(launch_features(fa, stream));
        PC_HIP(hipStreamSynchronize(stream));
        chunk.done();
        r0 = r;
    }
    fence.done();
    return PCHASE_OK;
}

extern "C" int pchase_mlp_train_step(pchase_mlp* net, const float* x_dev, const int32_t* labels_dev, uint32_t batch,
                                     float lr, float* loss, hipStream_t stream) {
    int rc = check_net(net);
    if (rc) return rc;
    if (batch == 0 || !x_dev || !labels_dev) return set_error(PCHASE_EINVAL, "empty batch");
    if (batch > 65536) return set_error(PCHASE_ERANGE, "batch above 65536");
    rc = ensure_act(net, batch);
    if (rc) return rc;
    PC_HIP(begin_steps(net, 1, stream));
    rc = enqueue_step(net, x_dev, labels_dev, batch, lr, stream);
    if (rc) return rc;
    net->steps += 1;
    if (loss) {
        CopyFence fence(stream);
        PC_HIP(hipMemcpyAsync(loss, net->loss, 4, hipMemcpyDeviceToHost, stream));
        PC_HIP(hipStreamSynchronize(stream));
        fence.done();
    }
    return PCHASE_OK;
}

// The step is captured once per (samples, labels, batch, lr, buffers) and
// its graph replayed once per batch: the batch index and the Adam step
// count live on the device and advance inside the step.
extern "C" int pchase_mlp_train(pchase_mlp* net, const float* x_dev, const int32_t* labels_dev, uint64_t n_samples,
                                uint32_t batch, uint32_t epochs, float lr, float* last_loss, hipStream_t stream) {
    int rc = check_net(net);
    if (rc) return rc;
    if (batch == 0 || batch > 65536) return set_error(PCHASE_EINVAL, "batch must be in 1..65536");
    if (n_samples < batch) return set_error(PCHASE_EINVAL, "fewer samples than one batch");
    if (!x_dev || !labels_dev) return set_error(PCHASE_EINVAL, "x_dev and labels_dev must not be NULL");
    const uint64_t steps = n_samples / batch;
    if (steps >= (1ull << 32)) return set_error(PCHASE_ERANGE, "too many batches");
    rc = ensure_act(net, batch);
    if (rc) return rc;
    char kb[192];
    snprintf(kb, sizeof kb, "%p|%p|%u|%a|%p|%p", (const void*)x_dev, (const void*)labels_dev, batch, (double)lr,
             net->act.p, net->params.p);
    if (!net->gexec || net->gkey != kb) {
        if (net->gexec) {
            (void)hipGraphExecDestroy(net->gexec);
            net->gexec = nullptr;
        }
        hipStream_t cs;
        PC_HIP(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
        hipGraph_t g = nullptr;
        hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
        int rc2 = PCHASE_OK;
        if (e == hipSuccess) rc2 = enqueue_step(net, x_dev, labels_dev, batch, lr, cs);
        hipError_t e2 = e == hipSuccess ? hipStreamEndCapture(cs, &g) : hipSuccess;
        (void)hipStreamDestroy(cs);
        if (e != hipSuccess) return hip_fail(e, "hipStreamBeginCapture");
        if (rc2) {
            if (g) (void)hipGraphDestroy(g);
            return rc2;
        }
        if (e2 != hipSuccess) return hip_fail(e2, "hipStreamEndCapture");
        e = hipGraphInstantiate(&net->gexec, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (e != hipSuccess) {
            net->gexec = nullptr;
            return hip_fail(e, "hipGraphInstantiate");
        }
        net->gkey = kb;
    }
    PC_HIP(begin_steps(net, (uint32_t)steps, stream));
    for (uint32_t ep = 0; ep < epochs; ++ep)
        for (uint64_t s = 0; s < steps; ++s) PC_HIP(hipGraphLaunch(net->gexec, stream));
    net->steps += steps * epochs;
    CopyFence fence(stream);
    if (last_loss) PC_HIP(hipMemcpyAsync(last_loss, net->loss, 4, hipMemcpyDeviceToHost, stream));
    PC_HIP(hipStreamSynchronize(stream));
    fence.done();
    return PCHASE_OK;
}

extern "C" int pchase_mlp_forward(const pchase_mlp* cnet, const float* x_dev, uint32_t batch, float* logits_dev,
                                  hipStream_t stream) {
    pchase_mlp* net = const_cast<pchase_mlp*>(cnet);
    int rc = check_net(net);
    if (rc) return rc;
    if (batch == 0) return PCHASE_OK;
    if (!x_dev || !logits_dev) return set_error(PCHASE_EINVAL, "x_dev and logits_dev must not be NULL");
    if (batch > 65536) return set_error(PCHASE_ERANGE, "batch above 65536");
    rc = ensure_act(net, batch);
    if (rc) return rc;
    PC_HIP(to_bf16(x_dev, net->xb, (uint64_t)batch * kIn, nullptr, stream));
    PC_HIP(forward_net(net, batch, stream));
    PC_HIP(hipMemcpyAsync(logits_dev, net->z, (size_t)batch * net->n_out * 4, hipMemcpyDeviceToDevice, stream));
    return PCHASE_OK;
}

extern "C" int pchase_mlp_topk(const float* logits_dev, uint32_t rows, uint32_t n_classes, uint32_t k,
                               int32_t* idx_dev, hipStream_t stream) {
    if (rows == 0) return PCHASE_OK;
    if (!logits_dev || !idx_dev) return set_error(PCHASE_EINVAL, "logits_dev and idx_dev must not be NULL");
    if (k == 0 || k > kMaxTopK || k > n_classes || n_classes > 64 * 64)
        return set_error(PCHASE_EINVAL, "k must be in 1..min(64, n_classes) and n_classes <= 4096");
    hipLaunchKernelGGL(topk_kernel, dim3(rows), dim3(64), 0, stream, logits_dev, n_classes, k, idx_dev);
    PC_HIP(hipGetLastError());
    return PCHASE_OK;
}

extern "C" int pchase_mlp_param(const pchase_mlp* cnet, uint32_t which, uint32_t slot, void* data, uint64_t* bytes,
                                int write) {
    pchase_mlp* net = const_cast<pchase_mlp*>(cnet);
    int rc = check_net(net);
    if (rc) return rc;
    if (which > 5 || slot > 3) return set_error(PCHASE_EINVAL, "which must be 0..5 and slot 0..3");
    if (write && slot == 3) return set_error(PCHASE_EINVAL, "gradients are read-only");
    const uint64_t nb = net->count[which] * 4;
    if (bytes) *bytes = nb;
    if (!data) return PCHASE_OK;
    float* dev = slot == 0 ? net->p[which] : slot == 1 ? net->m[which] : slot == 2 ? net->v[which] : net->g[which];
    if (write) {
        PC_HIP(hipMemcpy(dev, data, nb, hipMemcpyHostToDevice));
        if (slot == 0 && which % 2 == 0) {
            hipLaunchKernelGGL(refresh_bf16_kernel, dim3(blocks_for(net->count[which])), dim3(256), 0, 0, dev,
                               net->wb[which / 2], net->count[which]);
            PC_HIP(hipGetLastError());
            PC_HIP(hipDeviceSynchronize());
        }
    } else {
        PC_HIP(hipDeviceSynchronize());
        PC_HIP(hipMemcpy(data, dev, nb, hipMemcpyDeviceToHost));
    }
    return PCHASE_OK;
}

extern "C" int pchase_mlp_step_count(const pchase_mlp* cnet, uint64_t* steps, int set) {
    pchase_mlp* net = const_cast<pchase_mlp*>(cnet);
    if (!net || !steps) return set_error(PCHASE_EINVAL, "net and steps must not be NULL");
    if (set) net->steps = *steps;
    else *steps = net->steps;
    return PCHASE_OK;
}
