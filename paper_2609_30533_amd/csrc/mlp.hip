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

#include <vector>

#include "st_internal.hpp"

namespace st {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kEncIn = 65, kEncOut = 64, kCore = 16, kDin = 96, kWidth = 256, kOut = 168;
constexpr int kComp = 8, kDim = 8, kBins = 32;

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
// GEMM  C[M][N] = A(M x K) B(K x N) (+ bias), A(m,k) = A[m*sam + k*sak],
// B(k,n) = B[k*sbk + n*sbn].  Block tile 64 x 64, four waves of 32 x 32,
// each wave 2 x 2 MFMA 16x16x32 tiles.  Lane l of a 16x16x32 tile supplies
// row (l % 16) of A and column (l % 16) of B at k = 8 (l / 16) .. +7, and
// receives rows 4 (l / 16) .. +3 of column (l % 16) of the result.
// Epilogue: 0 store C; 1 store C (pre-activation) and gelu(C) into C2;
// 2 store C * gelu'(P) (P = stored pre-activation).
// ---------------------------------------------------------------------------
struct GemmArgs {
    const float *A, *B, *bias, *P;
    float *C, *C2;
    int M, N, K;
    int64_t sam, sak, sbk, sbn, ldc;
    int mode;
};

__global__ __launch_bounds__(256) void k_gemm(GemmArgs g) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int tm = blockIdx.y * 64 + (wave >> 1) * 32, tn = blockIdx.x * 64 + (wave & 1) * 32;
    f32x4 acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
    const int r16 = lane & 15, kq = (lane >> 4) * 8;
    for (int k0 = 0; k0 < g.K; k0 += 32) {
        bf16x8 a[2], b[2];
#pragma unroll
        for (int i = 0; i < 2; ++i) {
            const int m = tm + 16 * i + r16;
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const int k = k0 + kq + e;
                const float v = (m < g.M && k < g.K) ? g.A[(int64_t)m * g.sam + (int64_t)k * g.sak] : 0.f;
                a[i][e] = (__bf16)v;
            }
        }
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const int n = tn + 16 * j + r16;
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const int k = k0 + kq + e;
                const float v = (n < g.N && k < g.K) ? g.B[(int64_t)k * g.sbk + (int64_t)n * g.sbn] : 0.f;
                b[j][e] = (__bf16)v;
            }
        }
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
    }
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const int n = tn + 16 * j + r16;
            if (n >= g.N) continue;
            const float bn = g.bias ? g.bias[n] : 0.f;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int m = tm + 16 * i + (lane >> 4) * 4 + r;
                if (m >= g.M) continue;
                const float v = acc[i][j][r] + bn;
                const int64_t o = (int64_t)m * g.ldc + n;
                if (g.mode == 0) {
                    g.C[o] = v;
                } else if (g.mode == 1) {
                    g.C[o] = v;
                    g.C2[o] = gelu_f(v);
                } else {
                    g.C[o] = v * gelu_grad_f(g.P[o]);
                }
            }
        }
}

static hipError_t gemm(hipStream_t s, const float *A, int64_t sam, int64_t sak, const float *B, int64_t sbk,
                       int64_t sbn, const float *bias, float *C, int64_t ldc, int M, int N, int K, int mode = 0,
                       float *C2 = nullptr, const float *P = nullptr) {
    GemmArgs g{A, B, bias, P, C, C2, M, N, K, sam, sak, sbk, sbn, ldc, mode};
    dim3 grid((N + 63) / 64, (M + 63) / 64);
    k_gemm<<<grid, 256, 0, s>>>(g);
    return hipGetLastError();
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

// column sums (bias gradients)
__global__ void k_colsum(int M, int N, const float *X, float *out) {
    const int n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= N) return;
    float s = 0.f;
    for (int m = 0; m < M; ++m) s += X[(int64_t)m * N + n];
    out[n] = s;
}

// Mixture NLL of the path states plus the arrival-bin cross-entropy, and
// dL/dz; one thread per example, the mean over examples folded into dz.
__global__ void k_loss(int M, int K, const float *z, const float *y, const float *ymask, const float *dmask,
                       const int32_t *ubin, float *dz, float *loss_per) {
    const int m = blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= M) return;
    const float *zr = z + (int64_t)m * kOut;
    float *dr = dz + (int64_t)m * kOut;
    const float *mu = zr + kComp, *ls = zr + kComp + kComp * kDim, *hist = zr + kComp * (1 + 2 * kDim);
    const float *dm = dmask + m * kDim;
    float lmax = -INFINITY;
    for (int c = 0; c < kComp; ++c) lmax = fmaxf(lmax, zr[c]);
    float lse = 0.f;
    for (int c = 0; c < kComp; ++c) lse += __expf(zr[c] - lmax);
    lse = lmax + __logf(lse);
    for (int i = 0; i < kOut; ++i) dr[i] = 0.f;
    float cnt = 0.f;
    for (int k = 0; k < K; ++k) cnt += ymask[m * K + k];
    cnt = fmaxf(cnt, 1.f);
    const float inv = 1.f / (cnt * (float)M);
    float nll = 0.f;
    float rsum[kComp];
    for (int c = 0; c < kComp; ++c) rsum[c] = 0.f;
    for (int k = 0; k < K; ++k) {
        const float wk = ymask[m * K + k];
        if (!(wk > 0.f)) continue;
        const float *yk = y + ((int64_t)m * K + k) * kDim;
        float lj[kComp];
        float jmax = -INFINITY;
        for (int c = 0; c < kComp; ++c) {
            float s = zr[c] - lse;
            for (int j = 0; j < kDim; ++j) {
                if (!(dm[j] > 0.f)) continue;
                const float df = (yk[j] - mu[c * kDim + j]) * __expf(-ls[c * kDim + j]);
                s += -0.5f * df * df - ls[c * kDim + j] - 0.91893853320467274f;
            }
            lj[c] = s;
            jmax = fmaxf(jmax, s);
        }
        float se = 0.f;
        for (int c = 0; c < kComp; ++c) se += __expf(lj[c] - jmax);
        const float lp = jmax + __logf(se);
        nll -= wk * lp;
        for (int c = 0; c < kComp; ++c) {
            const float r = __expf(lj[c] - lp) * wk * inv;
            rsum[c] += r;
            for (int j = 0; j < kDim; ++j) {
                if (!(dm[j] > 0.f)) continue;
                const float isg = __expf(-ls[c * kDim + j]);
                const float df = (yk[j] - mu[c * kDim + j]) * isg;
                dr[kComp + c * kDim + j] -= r * df * isg;
                dr[kComp + kComp * kDim + c * kDim + j] -= r * (df * df - 1.f);
            }
        }
    }
    float rtot = 0.f;
    for (int c = 0; c < kComp; ++c) rtot += rsum[c];
    for (int c = 0; c < kComp; ++c) dr[c] = -(rsum[c] - __expf(zr[c] - lse) * rtot);
    float hmax = -INFINITY;
    for (int b = 0; b < kBins; ++b) hmax = fmaxf(hmax, hist[b]);
    float hs = 0.f;
    for (int b = 0; b < kBins; ++b) hs += __expf(hist[b] - hmax);
    const float hl = hmax + __logf(hs);
    const int ub = ubin[m];
    for (int b = 0; b < kBins; ++b)
        dr[kComp * (1 + 2 * kDim) + b] = (__expf(hist[b] - hl) - (b == ub ? 1.f : 0.f)) / (float)M;
    loss_per[m] = nll / cnt + (hl - hist[ub]);
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
    int M = 0, O = 0;
    int64_t step = 0;
};

namespace st {
static void mlp_free(st_mlp *n) {
    void *b[] = {n->param, n->grad, n->am, n->av, n->xo, n->pre_e, n->x0, n->z, n->arg, n->mask, n->dz, n->dh,
                 n->dpre, n->dx0, n->dpre_e, n->loss_per};
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
    ST_HIP(gemm(s, n->xo, kEncIn, 1, P + L.off[0], kEncOut, 1, P + L.off[1], n->pre_e, kEncOut, M * O, kEncOut, kEncIn));
    k_pool<<<(M * kDin + 255) / 256, 256, 0, s>>>(M, O, n->pre_e, n->mask, core, n->x0, n->arg);
    ST_HIP(hipGetLastError());
    const float *x = n->x0;
    int K = kDin;
    for (int l = 1; l <= 4; ++l) {
        ST_HIP(gemm(s, x, K, 1, P + L.off[2 * l], kWidth, 1, P + L.off[2 * l + 1], n->pre[l], kWidth, M, kWidth, K, 1,
                    n->h[l]));
        x = n->h[l];
        K = kWidth;
    }
    ST_HIP(gemm(s, x, kWidth, 1, P + L.off[10], kOut, 1, P + L.off[11], n->z, kOut, M, kOut, kWidth));
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
    k_loss<<<(n->M + 63) / 64, 64, 0, s>>>(n->M, K, n->z, y, ymask, dmask, ubin, n->dz, n->loss_per);
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
    ST_HIP(gemm(s, n->h[4], 1, kWidth, n->dz, kOut, 1, nullptr, G + L.off[10], kOut, kWidth, kOut, M));
    k_colsum<<<(kOut + 255) / 256, 256, 0, s>>>(M, kOut, n->dz, G + L.off[11]);
    // dpre4 = (dz W5^T) * gelu'(pre4)
    ST_HIP(gemm(s, n->dz, kOut, 1, P + L.off[10], 1, kOut, nullptr, n->dpre, kWidth, M, kWidth, kOut, 2, nullptr,
                n->pre[4]));
    for (int l = 4; l >= 1; --l) {
        const float *xin = l == 1 ? n->x0 : n->h[l - 1];
        const int K = l == 1 ? kDin : kWidth;
        // dW_l = x_{l-1}^T dpre_l, db_l = sum dpre_l
        ST_HIP(gemm(s, xin, 1, K, n->dpre, kWidth, 1, nullptr, G + L.off[2 * l], kWidth, K, kWidth, M));
        k_colsum<<<(kWidth + 255) / 256, 256, 0, s>>>(M, kWidth, n->dpre, G + L.off[2 * l + 1]);
        if (l > 1) {
            // dpre_{l-1} = (dpre_l W_l^T) * gelu'(pre_{l-1}); dh reused as scratch
            ST_HIP(gemm(s, n->dpre, kWidth, 1, P + L.off[2 * l], 1, kWidth, nullptr, n->dh, kWidth, M, kWidth, kWidth,
                        2, nullptr, n->pre[l - 1]));
            ST_HIP(hipMemcpyAsync(n->dpre, n->dh, (size_t)M * kWidth * 4, hipMemcpyDeviceToDevice, s));
        } else {
            ST_HIP(gemm(s, n->dpre, kWidth, 1, P + L.off[2], 1, kWidth, nullptr, n->dx0, kDin, M, kDin, kWidth));
        }
    }
    // encoder: route the pooled gradient to the arg-max obstacle
    const int64_t cnt = (int64_t)M * O * kEncOut;
    k_pool_back<<<(int)((cnt + 255) / 256), 256, 0, s>>>(M, O, n->dx0, n->arg, n->pre_e, n->dpre_e);
    ST_HIP(hipGetLastError());
    ST_HIP(gemm(s, n->xo, 1, kEncIn, n->dpre_e, kEncOut, 1, nullptr, G + L.off[0], kEncOut, kEncIn, kEncOut, M * O));
    k_colsum<<<1, 64, 0, s>>>(M * O, kEncOut, n->dpre_e, G + L.off[1]);
    ST_HIP(hipGetLastError());
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
