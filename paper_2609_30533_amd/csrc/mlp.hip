// mlp.hip -- the learned proposal network: forward, loss gradient, backward
// and Adam, on BF16 MFMA with FP32 accumulation (gfx950
// v_mfma_f32_16x16x32_bf16).
//
// Network (one row per problem): a shared per-obstacle encoder
// phi = gelu(obs We + be) max-pooled over the problem's obstacles, the trunk
// x0 = [core(16), pooled(64), 0(16)] -> 4 x (Linear 256 + GELU), and the head
// z = h4 W5 + b5 with 168 outputs: 8 mixture logits, 8 x 8 means, 8 x 8 log
// standard deviations (normalised q/pi and t/60), 32 arrival-histogram logits.
// Weights live in FP32 (master copy for Adam); every GEMM rounds its operands
// to bfloat16 when it packs them for the matrix cores and accumulates in FP32.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <utility>
#include <vector>

#include "st_internal.hpp"

namespace st {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kEncIn = 65, kEncOut = 64, kCore = 16, kDin = 96, kWidth = 256, kOut = 168;
constexpr int kComp = 8, kDim = 8, kBins = 32;
static_assert(kBins % kComp == 0 && 64 % kComp == 0, "loss lane groups");

// flat parameter layout: We, be, W1, b1, W2, b2, W3, b3, W4, b4, W5, b5
struct MlpLayout {
    int64_t off[12];
    int64_t total;
    MlpLayout() {
        const int shapes[6][2] = {{kEncIn, kEncOut}, {kDin, kWidth}, {kWidth, kWidth},
                                  {kWidth, kWidth},  {kWidth, kWidth}, {kWidth, kOut}};
        int64_t o = 0;
        for (int l = 0; l < 6; ++l) {
            off[2 * l] = o;
            o += (int64_t)shapes[l][0] * shapes[l][1];
            off[2 * l + 1] = o;
            o += shapes[l][1];
        }
        total = o;
    }
};

__device__ __forceinline__ float gelu_f(float x) { return 0.5f * x * (1.0f + erff(x * 0.70710678118654752f)); }
__device__ __forceinline__ float gelu_grad_f(float x) {
    return 0.5f * (1.0f + erff(x * 0.70710678118654752f)) + x * __expf(-0.5f * x * x) * 0.39894228040143268f;
}

// ---------------------------------------------------------------------------
// GEMM  C[M][N] = A(M x K) B(K x N) (+ bias).  A is stored with k contiguous
// (A(m,k) = A[m lda + k], AK) or m contiguous (A(m,k) = A[k lda + m]); B with
// n contiguous (B(k,n) = B[k ldb + n], BN) or k contiguous (B[n ldb + k]).
// Block tile 64 x 64, k step 32: the 256 threads load the A and B tiles from
// HBM with coalesced (vector where aligned) loads, round them to bfloat16 and
// store them k-contiguous in LDS, so that every MFMA operand is one 16-byte
// LDS read; the next tile's loads are in flight while the current one is
// multiplied.  Four waves of 32 x 32, each 2 x 2 MFMA 16x16x32 tiles: lane l
// supplies row (l % 16) of A and column (l % 16) of B at k = 8 (l / 16) .. +7
// and receives rows 4 (l / 16) .. +3 of column (l % 16) of the result.
// Epilogue: 0 store C; 1 store C (pre-activation) and gelu(C) into C2;
// 2 store C * gelu'(P) (P = stored pre-activation); 3 split-K partial: block
// z multiplies k in [z kc, (z + 1) kc) and stores its product (no bias) into
// C + z M ldc, summed afterwards in split order by k_sum_splits.
// ---------------------------------------------------------------------------
struct GemmArgs {
    const float *A, *B, *bias, *P;
    float *C, *C2;
    int M, N, K, kc;
    int64_t lda, ldb, ldc;
    int mode;
    int vec;  // bit 0: A rows may be read as float4; bit 1: B rows likewise
};

constexpr int kBK = 32, kLdsK = kBK + 8;  // LDS row: 32 bf16 + 16 bytes of padding

template <bool AK, bool BN>
__device__ __forceinline__ void gemm_load(const GemmArgs &g, int m0, int n0, int k0, int k1, float (&ra)[8],
                                          float (&rb)[8]) {
    const int t = threadIdx.x;
    if (AK) {  // thread: row t / 4, k 8 (t % 4) .. +7
        const int m = m0 + (t >> 2), k = k0 + (t & 3) * 8;
        const float *src = g.A + (int64_t)m * g.lda + k;
        if ((g.vec & 1) && m < g.M && k + 8 <= k1) {
            const float4 u = *(const float4 *)src, v = *(const float4 *)(src + 4);
            ra[0] = u.x; ra[1] = u.y; ra[2] = u.z; ra[3] = u.w;
            ra[4] = v.x; ra[5] = v.y; ra[6] = v.z; ra[7] = v.w;
        } else {
#pragma unroll
            for (int e = 0; e < 8; ++e) ra[e] = (m < g.M && k + e < k1) ? src[e] : 0.f;
        }
    } else {  // thread: k t / 8, rows 8 (t % 8) .. +7
        const int k = k0 + (t >> 3), m = m0 + (t & 7) * 8;
        const float *src = g.A + (int64_t)k * g.lda + m;
        if ((g.vec & 1) && k < k1 && m + 8 <= g.M) {
            const float4 u = *(const float4 *)src, v = *(const float4 *)(src + 4);
            ra[0] = u.x; ra[1] = u.y; ra[2] = u.z; ra[3] = u.w;
            ra[4] = v.x; ra[5] = v.y; ra[6] = v.z; ra[7] = v.w;
        } else {
#pragma unroll
            for (int e = 0; e < 8; ++e) ra[e] = (k < k1 && m + e < g.M) ? src[e] : 0.f;
        }
    }
    if (BN) {  // thread: k t / 8, columns 8 (t % 8) .. +7
        const int k = k0 + (t >> 3), n = n0 + (t & 7) * 8;
        const float *src = g.B + (int64_t)k * g.ldb + n;
        if ((g.vec & 2) && k < k1 && n + 8 <= g.N) {
            const float4 u = *(const float4 *)src, v = *(const float4 *)(src + 4);
            rb[0] = u.x; rb[1] = u.y; rb[2] = u.z; rb[3] = u.w;
            rb[4] = v.x; rb[5] = v.y; rb[6] = v.z; rb[7] = v.w;
        } else {
#pragma unroll
            for (int e = 0; e < 8; ++e) rb[e] = (k < k1 && n + e < g.N) ? src[e] : 0.f;
        }
    } else {  // thread: column t / 4, k 8 (t % 4) .. +7
        const int n = n0 + (t >> 2), k = k0 + (t & 3) * 8;
        const float *src = g.B + (int64_t)n * g.ldb + k;
        if ((g.vec & 2) && n < g.N && k + 8 <= k1) {
            const float4 u = *(const float4 *)src, v = *(const float4 *)(src + 4);
            rb[0] = u.x; rb[1] = u.y; rb[2] = u.z; rb[3] = u.w;
            rb[4] = v.x; rb[5] = v.y; rb[6] = v.z; rb[7] = v.w;
        } else {
#pragma unroll
            for (int e = 0; e < 8; ++e) rb[e] = (n < g.N && k + e < k1) ? src[e] : 0.f;
        }
    }
}

template <bool AK, bool BN>
__device__ __forceinline__ void gemm_store(__bf16 (*sA)[kLdsK], __bf16 (*sB)[kLdsK], const float (&ra)[8],
                                           const float (&rb)[8]) {
    const int t = threadIdx.x;
    if (AK) {
        bf16x8 v;
#pragma unroll
        for (int e = 0; e < 8; ++e) v[e] = (__bf16)ra[e];
        *(bf16x8 *)&sA[t >> 2][(t & 3) * 8] = v;
    } else {
#pragma unroll
        for (int e = 0; e < 8; ++e) sA[(t & 7) * 8 + e][t >> 3] = (__bf16)ra[e];
    }
    if (BN) {
#pragma unroll
        for (int e = 0; e < 8; ++e) sB[(t & 7) * 8 + e][t >> 3] = (__bf16)rb[e];
    } else {
        bf16x8 v;
#pragma unroll
        for (int e = 0; e < 8; ++e) v[e] = (__bf16)rb[e];
        *(bf16x8 *)&sB[t >> 2][(t & 3) * 8] = v;
    }
}

template <bool AK, bool BN>
__global__ __launch_bounds__(256) void k_gemm(GemmArgs g) {
    __shared__ __attribute__((aligned(16))) __bf16 sA[64][kLdsK], sB[64][kLdsK];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int m0 = blockIdx.y * 64, n0 = blockIdx.x * 64;
    const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
    const int kb = blockIdx.z * g.kc, ke = min(g.K, kb + g.kc);
    f32x4 acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
    const int r16 = lane & 15, kq = (lane >> 4) * 8;
    float ra[8], rb[8];
    if (kb < ke) gemm_load<AK, BN>(g, m0, n0, kb, ke, ra, rb);
    for (int k0 = kb; k0 < ke; k0 += kBK) {
        gemm_store<AK, BN>(sA, sB, ra, rb);
        __syncthreads();
        if (k0 + kBK < ke) gemm_load<AK, BN>(g, m0, n0, k0 + kBK, ke, ra, rb);
        bf16x8 a[2], b[2];
#pragma unroll
        for (int i = 0; i < 2; ++i) a[i] = *(const bf16x8 *)&sA[wm + 16 * i + r16][kq];
#pragma unroll
        for (int j = 0; j < 2; ++j) b[j] = *(const bf16x8 *)&sB[wn + 16 * j + r16][kq];
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
        __syncthreads();
    }
    float *C = g.mode == 3 ? g.C + (int64_t)blockIdx.z * g.M * g.ldc : g.C;
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const int n = n0 + wn + 16 * j + r16;
            if (n >= g.N) continue;
            const float bn = (g.bias && g.mode != 3) ? g.bias[n] : 0.f;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int m = m0 + wm + 16 * i + (lane >> 4) * 4 + r;
                if (m >= g.M) continue;
                const float v = acc[i][j][r] + bn;
                const int64_t o = (int64_t)m * g.ldc + n;
                if (g.mode == 0 || g.mode == 3) {
                    C[o] = v;
                } else if (g.mode == 1) {
                    C[o] = v;
                    g.C2[o] = gelu_f(v);
                } else {
                    C[o] = v * gelu_grad_f(g.P[o]);
                }
            }
        }
}

// out[i] = sum over z of part[z n + i]: a block takes 16 outputs, thread
// (o, g) sums the splits z = g (mod 16) of output o in order, and the 16
// group sums are added in group order (deterministic for given n and S)
__global__ __launch_bounds__(256) void k_sum_splits(int64_t n, int S, const float *part, float *out) {
    __shared__ float red[16][17];
    const int o = threadIdx.x & 15, g = threadIdx.x >> 4;
    const int64_t i = (int64_t)blockIdx.x * 16 + o;
    float s = 0.f;
    if (i < n)
        for (int z = g; z < S; z += 16) s += part[(int64_t)z * n + i];
    red[g][o] = s;
    __syncthreads();
    if (g == 0 && i < n) {
        float t = 0.f;
#pragma unroll
        for (int k = 0; k < 16; ++k) t += red[k][o];
        out[i] = t;
    }
}

static hipError_t sum_splits(hipStream_t s, int64_t n, int S, const float *part, float *out) {
    k_sum_splits<<<(int)((n + 15) / 16), 256, 0, s>>>(n, S, part, out);
    return hipGetLastError();
}

// Split-K factor of a product with a long reduction (weight gradients: the
// reduction runs over the examples): enough blocks to fill the device, at
// least 256 k per split, at most kMaxSplits splits.
constexpr int kMaxSplits = 256;
constexpr int kMaxColSplits = 1024;  // row chunks of a bias column sum at most
static int gemm_splits(int M, int N, int64_t K, int *kc) {
    const int64_t tiles = (int64_t)((M + 63) / 64) * ((N + 63) / 64);
    int64_t S = std::min<int64_t>((2048 + tiles - 1) / tiles, K / 256);
    S = std::max<int64_t>(1, std::min<int64_t>(S, kMaxSplits));
    int64_t c = (K + S - 1) / S;
    c = (c + kBK - 1) / kBK * kBK;
    *kc = (int)c;
    return (int)((K + c - 1) / c);
}

static bool aligned16(const void *p) { return ((uintptr_t)p & 15) == 0; }

// C = op(A) op(B): ak = A stored k-contiguous, bn = B stored n-contiguous.
// ws (split-K workspace, ws_floats long) may be null: then no split.
static hipError_t gemm(hipStream_t s, bool ak, const float *A, int64_t lda, bool bn, const float *B, int64_t ldb,
                       const float *bias, float *C, int64_t ldc, int M, int N, int K, int mode = 0,
                       float *C2 = nullptr, const float *P = nullptr, float *ws = nullptr, int64_t ws_floats = 0) {
    if (M <= 0 || N <= 0) return hipSuccess;
    GemmArgs g{A, B, bias, P, C, C2, M, N, K, K, lda, ldb, ldc, mode, 0};
    g.vec = ((lda % 4 == 0 && aligned16(A)) ? 1 : 0) | ((ldb % 4 == 0 && aligned16(B)) ? 2 : 0);
    int S = 1;
    if (ws && mode == 0 && !bias) {
        int kc = K;
        S = gemm_splits(M, N, K, &kc);
        if (S > 1 && (int64_t)S * M * N <= ws_floats) {
            g.kc = kc;
            g.mode = 3;
            g.C = ws;
            g.ldc = N;
        } else {
            S = 1;
        }
    }
    dim3 grid((N + 63) / 64, (M + 63) / 64, S);
    if (ak && bn) k_gemm<true, true><<<grid, 256, 0, s>>>(g);
    else if (ak) k_gemm<true, false><<<grid, 256, 0, s>>>(g);
    else if (bn) k_gemm<false, true><<<grid, 256, 0, s>>>(g);
    else k_gemm<false, false><<<grid, 256, 0, s>>>(g);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || S == 1) return e;
    if (ldc != N) return hipErrorInvalidValue;  // split results are stored dense
    return sum_splits(s, (int64_t)M * N, S, ws, C);
}

// encoder: phi = gelu(pre_e); masked max over obstacles (first maximum wins);
// x0 = [core, pooled, 0]
__global__ void k_pool(int M, int O, const float *pre_e, const float *mask, const float *core, float *x0,
                       int32_t *arg) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= M * kDin) return;
    const int m = i / kDin, c = i % kDin;
    float v = 0.f;
    if (c < kCore) {
        v = core[m * kCore + c];
    } else if (c < kCore + kEncOut) {
        const int ch = c - kCore;
        float best = -INFINITY;
        int bo = -1;
        for (int o = 0; o < O; ++o) {
            if (!(mask[m * O + o] > 0.f)) continue;
            const float ph = gelu_f(pre_e[((int64_t)m * O + o) * kEncOut + ch]);
            if (ph > best) {
                best = ph;
                bo = o;
            }
        }
        v = bo >= 0 ? best : 0.f;
        arg[m * kEncOut + ch] = bo;
    }
    x0[i] = v;
}

__global__ void k_pool_back(int M, int O, const float *dx0, const int32_t *arg, const float *pre_e, float *dpre_e) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (int64_t)M * O * kEncOut) return;
    const int ch = (int)(i % kEncOut);
    const int64_t mo = i / kEncOut;
    const int m = (int)(mo / O), o = (int)(mo % O);
    const bool sel = arg[m * kEncOut + ch] == o;
    dpre_e[i] = sel ? dx0[m * kDin + kCore + ch] * gelu_grad_f(pre_e[i]) : 0.f;
}

// Column sums (bias gradients) in two deterministic passes: block (x, z)
// sums columns 64 x .. +63 over rows [z rc, (z + 1) rc) (four row phases per
// column, combined in LDS) into part[z N + n]; k_sum_splits adds the splits.
__global__ __launch_bounds__(256) void k_colsum_part(int M, int N, int rc, const float *X, float *part) {
    __shared__ float red[4][64];
    const int c = threadIdx.x & 63, ph = threadIdx.x >> 6;
    const int n = blockIdx.x * 64 + c;
    const int r0 = blockIdx.y * rc, r1 = min(M, r0 + rc);
    float s = 0.f;
    if (n < N)
        for (int m = r0 + ph; m < r1; m += 4) s += X[(int64_t)m * N + n];
    red[ph][c] = s;
    __syncthreads();
    if (ph == 0 && n < N) part[(int64_t)blockIdx.y * N + n] = ((red[0][c] + red[1][c]) + red[2][c]) + red[3][c];
}

static hipError_t colsum(hipStream_t s, int64_t M, int N, const float *X, float *out, float *ws) {
    // row chunks of at least 64 rows (16 per thread), at most kMaxColSplits
    const int S = (int)std::max<int64_t>(1, std::min<int64_t>(kMaxColSplits, M / 64));
    const int rc = (int)((M + S - 1) / S);
    k_colsum_part<<<dim3((N + 63) / 64, S), 256, 0, s>>>((int)M, N, rc, X, ws);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return sum_splits(s, N, S, ws, out);
}

// Reductions over the kComp lanes of one example (groups of 8 lanes).
__device__ __forceinline__ float group_max(float v) {
#pragma unroll
    for (int o = 1; o < kComp; o <<= 1) v = fmaxf(v, __shfl_xor(v, o, kComp));
    return v;
}
__device__ __forceinline__ float group_sum(float v) {
#pragma unroll
    for (int o = 1; o < kComp; o <<= 1) v += __shfl_xor(v, o, kComp);
    return v;
}

// Mixture NLL of the path states plus the arrival-bin cross-entropy, and
// dL/dz, the mean over examples folded into dz.  One group of kComp lanes per
// example: lane c owns mixture component c (its means, log standard
// deviations and their gradients, in registers) and arrival bins c, c + 8,
// c + 16, c + 24; the per-state log-sum-exp over components is a reduction
// inside the group.
__global__ __launch_bounds__(256) void k_loss(int M, int K, const float *z, const float *y, const float *ymask,
                                              const float *dmask, const int32_t *ubin, float *dz, float *loss_per) {
    const int gid = blockIdx.x * blockDim.x + threadIdx.x;
    const int m = gid / kComp, c = gid % kComp;
    if (m >= M) return;  // whole groups leave together
    const float *zr = z + (int64_t)m * kOut;
    float *dr = dz + (int64_t)m * kOut;
    const float *dm = dmask + m * kDim;
    float mu[kDim], lsv[kDim], isg[kDim];
    bool on[kDim];
#pragma unroll
    for (int j = 0; j < kDim; ++j) {
        mu[j] = zr[kComp + c * kDim + j];
        lsv[j] = zr[kComp + kComp * kDim + c * kDim + j];
        isg[j] = __expf(-lsv[j]);
        on[j] = dm[j] > 0.f;
    }
    const float zc = zr[c];
    const float lmax = group_max(zc);
    const float lse = lmax + __logf(group_sum(__expf(zc - lmax)));
    float cnt = 0.f;
    for (int k = 0; k < K; ++k) cnt += ymask[m * K + k];
    cnt = fmaxf(cnt, 1.f);
    const float inv = 1.f / (cnt * (float)M);
    float nll = 0.f, rsum = 0.f, gmu[kDim], gls[kDim];
#pragma unroll
    for (int j = 0; j < kDim; ++j) gmu[j] = gls[j] = 0.f;
    for (int k = 0; k < K; ++k) {
        const float wk = ymask[m * K + k];
        if (!(wk > 0.f)) continue;  // the same for the whole group
        const float *yk = y + ((int64_t)m * K + k) * kDim;
        float s = zc - lse, df[kDim];
#pragma unroll
        for (int j = 0; j < kDim; ++j) {
            df[j] = (yk[j] - mu[j]) * isg[j];
            if (on[j]) s += -0.5f * df[j] * df[j] - lsv[j] - 0.91893853320467274f;
        }
        const float jmax = group_max(s);
        const float lp = jmax + __logf(group_sum(__expf(s - jmax)));
        nll -= wk * lp;
        const float r = __expf(s - lp) * wk * inv;
        rsum += r;
#pragma unroll
        for (int j = 0; j < kDim; ++j) {
            if (on[j]) {
                gmu[j] -= r * df[j] * isg[j];
                gls[j] -= r * (df[j] * df[j] - 1.f);
            }
        }
    }
#pragma unroll
    for (int j = 0; j < kDim; ++j) {
        dr[kComp + c * kDim + j] = gmu[j];
        dr[kComp + kComp * kDim + c * kDim + j] = gls[j];
    }
    const float rtot = group_sum(rsum);
    dr[c] = -(rsum - __expf(zc - lse) * rtot);
    const float *hist = zr + kComp * (1 + 2 * kDim);
    float hb[kBins / kComp];
    float hm = -INFINITY;
#pragma unroll
    for (int i = 0; i < kBins / kComp; ++i) {
        hb[i] = hist[c + kComp * i];
        hm = fmaxf(hm, hb[i]);
    }
    const float hmax = group_max(hm);
    float hs = 0.f;
#pragma unroll
    for (int i = 0; i < kBins / kComp; ++i) hs += __expf(hb[i] - hmax);
    const float hl = hmax + __logf(group_sum(hs));
    const int ub = ubin[m];
#pragma unroll
    for (int i = 0; i < kBins / kComp; ++i) {
        const int bin = c + kComp * i;
        dr[kComp * (1 + 2 * kDim) + bin] = (__expf(hb[i] - hl) - (bin == ub ? 1.f : 0.f)) / (float)M;
    }
    if (c == 0) loss_per[m] = nll / cnt + (hl - hist[ub]);
}

__global__ void k_adam(int64_t n, float *p, const float *g, float *m, float *v, float lr, float b1, float b2,
                       float eps, float c1, float c2) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

}  // namespace st

using namespace st;

struct st_mlp {
    MlpLayout lay;
    int max_M = 0, max_O = 0;
    float *param = nullptr, *grad = nullptr, *am = nullptr, *av = nullptr;
    // activations of the last forward pass
    float *xo = nullptr, *pre_e = nullptr, *x0 = nullptr, *pre[5] = {}, *h[5] = {}, *z = nullptr;
    int32_t *arg = nullptr;
    float *mask = nullptr;
    // gradients of activations
    float *dz = nullptr, *dh = nullptr, *dpre = nullptr, *dx0 = nullptr, *dpre_e = nullptr, *loss_per = nullptr;
    // split-K partial products and partial column sums of the weight and
    // bias gradients
    float *ws = nullptr;
    int64_t ws_floats = 0;
    int M = 0, O = 0;
    int64_t step = 0;
};

namespace st {
static void mlp_free(st_mlp *n) {
    void *b[] = {n->param, n->grad, n->am, n->av, n->xo, n->pre_e, n->x0, n->z, n->arg, n->mask, n->dz, n->dh,
                 n->dpre, n->dx0, n->dpre_e, n->loss_per, n->ws};
    for (void *x : b)
        if (x) (void)hipFree(x);
    for (int l = 0; l < 5; ++l) {
        if (n->pre[l]) (void)hipFree(n->pre[l]);
        if (n->h[l]) (void)hipFree(n->h[l]);
    }
    delete n;
}
}  // namespace st

extern "C" {

int st_mlp_create(int32_t max_batch, int32_t max_obstacles, st_mlp **out) {
    if (!out || max_batch < 1 || max_obstacles < 1 || max_obstacles > ST_MAX_OBSTACLES) {
        set_error("st_mlp_create: bad arguments");
        return ST_EINVAL;
    }
    st_mlp *n = new (std::nothrow) st_mlp();
    if (!n) {
        set_error("st_mlp_create: out of host memory");
        return ST_ENOMEM;
    }
    n->max_M = max_batch;
    n->max_O = max_obstacles;
    const int64_t P = n->lay.total, M = max_batch, MO = (int64_t)max_batch * max_obstacles;
    auto al = [&](float **p, int64_t cnt) { return hipMalloc((void **)p, (size_t)std::max<int64_t>(cnt, 1) * 4); };
    hipError_t e = hipSuccess;
    for (float **p : {&n->param, &n->grad, &n->am, &n->av})
        if (e == hipSuccess) e = al(p, P);
    if (e == hipSuccess) e = al(&n->xo, MO * kEncIn);
    if (e == hipSuccess) e = al(&n->pre_e, MO * kEncOut);
    if (e == hipSuccess) e = al(&n->dpre_e, MO * kEncOut);
    if (e == hipSuccess) e = al(&n->mask, MO);
    if (e == hipSuccess) e = al(&n->x0, M * kDin);
    if (e == hipSuccess) e = al(&n->dx0, M * kDin);
    for (int l = 1; l <= 4 && e == hipSuccess; ++l) {
        e = al(&n->pre[l], M * kWidth);
        if (e == hipSuccess) e = al(&n->h[l], M * kWidth);
    }
    if (e == hipSuccess) e = al(&n->z, M * kOut);
    if (e == hipSuccess) e = al(&n->dz, M * kOut);
    if (e == hipSuccess) e = al(&n->dh, M * kWidth);
    if (e == hipSuccess) e = al(&n->dpre, M * kWidth);
    if (e == hipSuccess) e = al(&n->loss_per, M);
    {
        // the largest split-K workspace any weight-gradient product or bias
        // column sum of a batch up to max_batch rows needs
        const int shapes[4][3] = {{kWidth, kOut, 0}, {kWidth, kWidth, 0}, {kDin, kWidth, 0}, {kEncIn, kEncOut, 1}};
        int64_t need = (int64_t)kMaxColSplits * kWidth;
        for (const auto &sh : shapes) {
            int kc = 0;
            const int64_t K = sh[2] ? MO : M;
            const int S = gemm_splits(sh[0], sh[1], K, &kc);
            need = std::max<int64_t>(need, (int64_t)S * sh[0] * sh[1]);
        }
        n->ws_floats = need;
        if (e == hipSuccess) e = al(&n->ws, need);
    }
    if (e == hipSuccess) e = hipMalloc((void **)&n->arg, (size_t)M * kEncOut * 4);
    if (e == hipSuccess) e = hipMemset(n->am, 0, (size_t)P * 4);
    if (e == hipSuccess) e = hipMemset(n->av, 0, (size_t)P * 4);
    if (e == hipSuccess) e = hipMemset(n->param, 0, (size_t)P * 4);
    if (e != hipSuccess) {
        set_error("st_mlp_create: %s", hipGetErrorString(e));
        mlp_free(n);
        return ST_EHIP;
    }
    *out = n;
    return ST_OK;
}

void st_mlp_destroy(st_mlp *n) {
    if (n) mlp_free(n);
}

int64_t st_mlp_param_count(void) { return MlpLayout().total; }

int st_mlp_params(st_mlp *n, const float *host_in, float *host_out) {
    if (!n) {
        set_error("st_mlp_params: null network");
        return ST_EINVAL;
    }
    const size_t bytes = (size_t)n->lay.total * 4;
    if (host_in) {
        ST_HIP(hipMemcpy(n->param, host_in, bytes, hipMemcpyHostToDevice));
        ST_HIP(hipMemset(n->am, 0, bytes));
        ST_HIP(hipMemset(n->av, 0, bytes));
        n->step = 0;
    }
    if (host_out) ST_HIP(hipMemcpy(host_out, n->param, bytes, hipMemcpyDeviceToHost));
    return ST_OK;
}

int st_mlp_grads(st_mlp *n, float *host_out) {
    if (!n || !host_out) {
        set_error("st_mlp_grads: bad arguments");
        return ST_EINVAL;
    }
    ST_HIP(hipDeviceSynchronize());
    ST_HIP(hipMemcpy(host_out, n->grad, (size_t)n->lay.total * 4, hipMemcpyDeviceToHost));
    return ST_OK;
}

int st_mlp_forward(st_mlp *n, int32_t M, int32_t O, const float *core, const float *obs, const float *mask,
                   float *z_out, void *stream) {
    if (!n || M < 1 || M > n->max_M || O < 1 || O > n->max_O || !core || !obs || !mask) {
        set_error("st_mlp_forward: bad arguments");
        return ST_EINVAL;
    }
    hipStream_t s = (hipStream_t)stream;
    n->M = M;
    n->O = O;
    const MlpLayout &L = n->lay;
    const float *P = n->param;
    ST_HIP(hipMemcpyAsync(n->xo, obs, (size_t)M * O * kEncIn * 4, hipMemcpyDeviceToDevice, s));
    ST_HIP(hipMemcpyAsync(n->mask, mask, (size_t)M * O * 4, hipMemcpyDeviceToDevice, s));
    // encoder: pre_e = obs We + be over M*O rows
    ST_HIP(gemm(s, true, n->xo, kEncIn, true, P + L.off[0], kEncOut, P + L.off[1], n->pre_e, kEncOut, M * O, kEncOut,
                kEncIn));
    k_pool<<<(M * kDin + 255) / 256, 256, 0, s>>>(M, O, n->pre_e, n->mask, core, n->x0, n->arg);
    ST_HIP(hipGetLastError());
    const float *x = n->x0;
    int K = kDin;
    for (int l = 1; l <= 4; ++l) {
        ST_HIP(gemm(s, true, x, K, true, P + L.off[2 * l], kWidth, P + L.off[2 * l + 1], n->pre[l], kWidth, M, kWidth, K,
                    1, n->h[l]));
        x = n->h[l];
        K = kWidth;
    }
    ST_HIP(gemm(s, true, x, kWidth, true, P + L.off[10], kOut, P + L.off[11], n->z, kOut, M, kOut, kWidth));
    if (z_out) ST_HIP(hipMemcpyAsync(z_out, n->z, (size_t)M * kOut * 4, hipMemcpyDeviceToDevice, s));
    return ST_OK;
}

int st_mlp_loss(st_mlp *n, int32_t K, const float *y, const float *ymask, const float *dmask, const int32_t *ubin,
                float *loss_per_out, void *stream) {
    if (!n || n->M < 1 || K < 1 || !y || !ymask || !dmask || !ubin) {
        set_error("st_mlp_loss: bad arguments (run st_mlp_forward first)");
        return ST_EINVAL;
    }
    hipStream_t s = (hipStream_t)stream;
    k_loss<<<(n->M * kComp + 255) / 256, 256, 0, s>>>(n->M, K, n->z, y, ymask, dmask, ubin, n->dz, n->loss_per);
    ST_HIP(hipGetLastError());
    if (loss_per_out) ST_HIP(hipMemcpyAsync(loss_per_out, n->loss_per, (size_t)n->M * 4, hipMemcpyDeviceToDevice, s));
    return ST_OK;
}

int st_mlp_backward(st_mlp *n, void *stream) {
    if (!n || n->M < 1) {
        set_error("st_mlp_backward: run st_mlp_forward and st_mlp_loss first");
        return ST_EINVAL;
    }
    hipStream_t s = (hipStream_t)stream;
    const MlpLayout &L = n->lay;
    const float *P = n->param;
    float *G = n->grad;
    const int M = n->M, O = n->O;
    // head: dW5 = h4^T dz, db5 = sum dz, dh4 = dz W5^T
    ST_HIP(gemm(s, false, n->h[4], kWidth, true, n->dz, kOut, nullptr, G + L.off[10], kOut, kWidth, kOut, M, 0,
                nullptr, nullptr, n->ws, n->ws_floats));
    ST_HIP(colsum(s, M, kOut, n->dz, G + L.off[11], n->ws));
    // dpre4 = (dz W5^T) * gelu'(pre4)
    ST_HIP(gemm(s, true, n->dz, kOut, false, P + L.off[10], kOut, nullptr, n->dpre, kWidth, M, kWidth, kOut, 2,
                nullptr, n->pre[4]));
    for (int l = 4; l >= 1; --l) {
        const float *xin = l == 1 ? n->x0 : n->h[l - 1];
        const int K = l == 1 ? kDin : kWidth;
        // dW_l = x_{l-1}^T dpre_l, db_l = sum dpre_l
        ST_HIP(gemm(s, false, xin, K, true, n->dpre, kWidth, nullptr, G + L.off[2 * l], kWidth, K, kWidth, M, 0,
                    nullptr, nullptr, n->ws, n->ws_floats));
        ST_HIP(colsum(s, M, kWidth, n->dpre, G + L.off[2 * l + 1], n->ws));
        if (l > 1) {
            // dpre_{l-1} = (dpre_l W_l^T) * gelu'(pre_{l-1}) into dh, then the
            // two buffers trade places
            ST_HIP(gemm(s, true, n->dpre, kWidth, false, P + L.off[2 * l], kWidth, nullptr, n->dh, kWidth, M, kWidth,
                        kWidth, 2, nullptr, n->pre[l - 1]));
            std::swap(n->dpre, n->dh);
        } else {
            ST_HIP(gemm(s, true, n->dpre, kWidth, false, P + L.off[2], kWidth, nullptr, n->dx0, kDin, M, kDin, kWidth));
        }
    }
    // encoder: route the pooled gradient to the arg-max obstacle
    const int64_t cnt = (int64_t)M * O * kEncOut;
    k_pool_back<<<(int)((cnt + 255) / 256), 256, 0, s>>>(M, O, n->dx0, n->arg, n->pre_e, n->dpre_e);
    ST_HIP(hipGetLastError());
    ST_HIP(gemm(s, false, n->xo, kEncIn, true, n->dpre_e, kEncOut, nullptr, G + L.off[0], kEncOut, kEncIn, kEncOut,
                M * O, 0, nullptr, nullptr, n->ws, n->ws_floats));
    ST_HIP(colsum(s, (int64_t)M * O, kEncOut, n->dpre_e, G + L.off[1], n->ws));
    return ST_OK;
}

int st_mlp_adam(st_mlp *n, float lr, void *stream) {
    if (!n || !(lr > 0.f)) {
        set_error("st_mlp_adam: bad arguments");
        return ST_EINVAL;
    }
    n->step++;
    const float b1 = 0.9f, b2 = 0.999f;
    const float c1 = 1.f - powf(b1, (float)n->step), c2 = 1.f - powf(b2, (float)n->step);
    const int64_t P = n->lay.total;
    k_adam<<<(int)((P + 255) / 256), 256, 0, (hipStream_t)stream>>>(P, n->param, n->grad, n->am, n->av, lr, b1, b2,
                                                                    1e-8f, c1, c2);
    ST_HIP(hipGetLastError());
    return ST_OK;
}

}  // extern "C"
