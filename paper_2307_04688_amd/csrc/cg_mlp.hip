// cg_mlp.hip -- the learned warm start on gfx950: a 9 -> 256 -> 256 -> 256 -> 3
// GELU network in binary32 (forward, MSE loss, back-propagation, Adam,
// minibatch sampling), the features of a game's nodes, and the warm-started
// solve with its fallback to the zero start.
//
// Dense layers are GEMMs on the f32 16x16x4 MFMA with fused epilogues (bias,
// GELU, GELU derivative).  The weight gradient of a layer is one GEMM over the
// batch with an extra all-ones input row, so its last output row is the bias
// gradient and the result lands on [W; b] of the flat parameter vector; the
// batch dimension is split over blocks and the partial sums are reduced in a
// fixed order (reruns are bitwise equal).
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <vector>

#include "cg_internal.h"

using namespace cg;

namespace {

constexpr int IN = CG_MLP_IN, HID = CG_MLP_HIDDEN, OUT = CG_MLP_OUT;
constexpr int NL = 4;
constexpr int FAN_IN[NL] = {IN, HID, HID, HID};
constexpr int FAN_OUT[NL] = {HID, HID, HID, OUT};
constexpr long long layer_off(int l)
{
    long long o = 0;
    for (int k = 0; k < l; ++k) o += (long long)(FAN_IN[k] + 1) * FAN_OUT[k];
    return o;
}
constexpr long long P_TOTAL = layer_off(NL);
static_assert(P_TOTAL == 134915, "parameter count");

constexpr int MAX_BATCH = 65536;
constexpr int MAX_SPLIT = 32;
constexpr int MAX_NODES = CG_MAX_N * CG_MAX_N * CG_MAX_N;  // d = 3
constexpr int LOSS_BLOCKS = 256;

enum Epi { EPI_STORE = 0, EPI_BIAS = 1, EPI_BIAS_GELU = 2, EPI_GELU_ONLY = 3, EPI_GELU_BWD = 4 };

__device__ __forceinline__ float gelu(float z) { return 0.5f * z * (1.0f + erff(z * 0.70710678118654752f)); }
__device__ __forceinline__ float gelu_grad(float z)
{
    return 0.5f * (1.0f + erff(z * 0.70710678118654752f)) + z * 0.39894228040143268f * expf(-0.5f * z * z);
}

// C = op(A) op(B) over the K range of this block's split (blockIdx.z), 64 x 64
// tile per block of 4 waves (32 x 32 each, 2 x 2 MFMA tiles).  op(A) is M x K:
// A is stored [M][K] (TA = false) or [K][M] (TA = true); op(B) is K x N: B is
// stored [K][N] (TB = false) or [N][K] (TB = true).  ONES: row M-1 of op(A) is
// all ones (A itself has M-1 rows).  Out-of-range operand elements are zero.
template <bool TA, bool TB, bool ONES, int EPI>
__global__ __launch_bounds__(256) void k_gemm(int M, int N, int K, int kchunk, const float *__restrict__ A, int lda,
                                              const float *__restrict__ B, int ldb, float *__restrict__ C, int ldc,
                                              long long split_stride, const float *__restrict__ bias,
                                              float *__restrict__ H, const float *__restrict__ Zs)
{
    constexpr int BM = 64, BN = 64, BK = 16, LD = 68;
    __shared__ float As[BK][LD];
    __shared__ float Bs[BK][LD];
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int r16 = lane & 15, g4 = lane >> 4;
    const int m0 = blockIdx.x * BM, n0 = blockIdx.y * BN;
    const int kbeg = blockIdx.z * kchunk;
    const int kend = min(K, kbeg + kchunk);
    const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
    const int Ma = ONES ? M - 1 : M;

    f32x4 acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};

    for (int k0 = kbeg; k0 < kend; k0 += BK) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int e = tid + q * 256;
            const int kk = TA ? (e >> 6) : (e & 15);
            const int mm = TA ? (e & 63) : (e >> 4);
            const int gk = k0 + kk, gm = m0 + mm;
            float val = 0.f;
            if (gk < kend) {
                if (gm < Ma)
                    val = TA ? A[(long long)gk * lda + gm] : A[(long long)gm * lda + gk];
                else if (ONES && gm == Ma)
                    val = 1.0f;
            }
            As[kk][mm] = val;
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int e = tid + q * 256;
            const int kk = TB ? (e & 15) : (e >> 6);
            const int nn = TB ? (e >> 4) : (e & 63);
            const int gk = k0 + kk, gn = n0 + nn;
            float val = 0.f;
            if (gk < kend && gn < N) val = TB ? B[(long long)gn * ldb + gk] : B[(long long)gk * ldb + gn];
            Bs[kk][nn] = val;
        }
        __syncthreads();
#pragma unroll
        for (int ks = 0; ks < BK; ks += 4) {
            float a[2], b[2];
#pragma unroll
            for (int i = 0; i < 2; ++i) a[i] = As[ks + g4][wm + i * 16 + r16];
#pragma unroll
            for (int j = 0; j < 2; ++j) b[j] = Bs[ks + g4][wn + j * 16 + r16];
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int j = 0; j < 2; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[i], b[j], acc[i][j], 0, 0, 0);
        }
        __syncthreads();
    }

    float *Cs = C + (long long)blockIdx.z * split_stride;
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int row = m0 + wm + i * 16 + 4 * g4 + v;  // f32 16x16 form: rows 4g + v
                const int col = n0 + wn + j * 16 + r16;
                if (row < M && col < N) {
                    const long long idx = (long long)row * ldc + col;
                    const float x = acc[i][j][v];
                    if (EPI == EPI_STORE) {
                        Cs[idx] = x;
                    } else if (EPI == EPI_BIAS) {
                        Cs[idx] = x + bias[col];
                    } else if (EPI == EPI_BIAS_GELU) {
                        const float z = x + bias[col];
                        Cs[idx] = z;
                        H[idx] = gelu(z);
                    } else if (EPI == EPI_GELU_ONLY) {
                        H[idx] = gelu(x + bias[col]);
                    } else {
                        Cs[idx] = x * gelu_grad(Zs[idx]);
                    }
                }
            }
}

// grad[e] = sum_s part[s][e] in order s = 0, 1, ...
__global__ void k_split_reduce(const float *__restrict__ part, long long stride, int S, long long n,
                               float *__restrict__ out)
{
    const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n) return;
    float s = 0.f;
    for (int k = 0; k < S; ++k) s += part[k * stride + e];
    out[e] = s;
}

// dY = 2 (Y - T) / (3 n); per-block partial sums of (Y - T)^2 (fixed order).
__global__ __launch_bounds__(256) void k_mse(const float *__restrict__ Y, const float *__restrict__ T, int n,
                                             float *__restrict__ dY, float *__restrict__ part)
{
    __shared__ float red[256];
    const long long total = (long long)n * OUT;
    const float scale = 2.0f / (float)total;
    float s = 0.f;
    for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (long long)gridDim.x * blockDim.x) {
        const float r = Y[e] - T[e];
        dY[e] = scale * r;
        s += r * r;
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

__global__ void k_loss_final(const float *__restrict__ part, int nparts, int n, float *__restrict__ loss)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double s = 0.0;
    for (int k = 0; k < nparts; ++k) s += (double)part[k];
    *loss = (float)(s / ((double)n * OUT));
}

__global__ void k_adam(float *__restrict__ p, const float *__restrict__ g, float *__restrict__ m,
                       float *__restrict__ v, long long n, float lr, float b1, float b2, float eps, float c1, float c2)
{
    for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < n;
         e += (long long)gridDim.x * blockDim.x) {
        const float ge = g[e];
        const float me = b1 * m[e] + (1.0f - b1) * ge;
        const float ve = b2 * v[e] + (1.0f - b2) * ge * ge;
        m[e] = me;
        v[e] = ve;
        p[e] -= lr * (me * c1) / (sqrtf(ve * c2) + eps);
    }
}

// SplitMix64 (Steele, Lea and Flood, 2014) of a counter: the minibatch rows.
__device__ __forceinline__ unsigned long long splitmix64(unsigned long long x)
{
    x += 0x9E3779B97F4A7C15ull;
    x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
    x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
    return x ^ (x >> 31);
}

__global__ void k_gather(const float *__restrict__ X, const float *__restrict__ T, long long nsamp, int nb,
                         unsigned long long seed, long long step, float *__restrict__ Xb, float *__restrict__ Tb)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= nb) return;
    const unsigned long long r = splitmix64(seed ^ splitmix64((unsigned long long)step * (unsigned long long)nb + k));
    const long long src = (long long)(r % (unsigned long long)nsamp);
#pragma unroll
    for (int c = 0; c < IN; ++c) Xb[(long long)k * IN + c] = X[src * IN + c];
#pragma unroll
    for (int c = 0; c < OUT; ++c) Tb[(long long)k * OUT + c] = T[src * OUT + c];
}

struct Theta {
    float t[6];
};

// Rows [r0, r0 + cnt) of a d = 3 game's features: (theta, x_0, x_1, x_2) with
// x_l the Lobatto node of mode l; targets t_scale * V_i at the node.
__global__ void k_features(const GameConst *__restrict__ gc, const GameStatus *__restrict__ st,
                           const double *__restrict__ V, Theta th, double t_scale, long long r0, int cnt,
                           float *__restrict__ X, float *__restrict__ T)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= cnt) return;
    const long long j = r0 + k;
    const int N = gc->N;
    const long long NN = gc->NN;
    int rem = (int)j;
    const int k2 = rem % N;
    rem /= N;
    const int k1 = rem % N;
    const int k0 = rem / N;
#pragma unroll
    for (int c = 0; c < 6; ++c) X[(long long)k * IN + c] = th.t[c];
    X[(long long)k * IN + 6] = (float)gc->xnode[k0];
    X[(long long)k * IN + 7] = (float)gc->xnode[k1];
    X[(long long)k * IN + 8] = (float)gc->xnode[k2];
    if (T) {
        const double *Vc = V + (long long)st->cur * 3 * NN;
#pragma unroll
        for (int i = 0; i < OUT; ++i) T[(long long)k * OUT + i] = (float)(t_scale * Vc[i * NN + j]);
    }
}

// V0[i][r0 + k] = out_scale * Y[k][i]; flags a non-finite value.
__global__ void k_warm_write(const float *__restrict__ Y, int cnt, long long r0, long long NN, double out_scale,
                             double *__restrict__ V0, int *__restrict__ bad)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= cnt) return;
#pragma unroll
    for (int i = 0; i < OUT; ++i) {
        const double v = out_scale * (double)Y[(long long)k * OUT + i];
        if (!(fabs(v) <= 1.7976931348623157e308)) atomicOr(bad, 1);
        V0[i * NN + r0 + k] = v;
    }
}

// u^[0]_i = clip(A_i + delta beta_i dV_i/dp_i, 0, U_M) at every node: the
// maximiser of Step 3's objective with V expanded to first order around the
// node (dV_i/dp_i from the nodal differentiation matrix along mode i).
__global__ void k_warm_controls(const GameConst *__restrict__ gc, const double *__restrict__ V0,
                                double *__restrict__ U0)
{
    const long long j = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long NN = gc->NN;
    if (j >= NN) return;
    const int N = gc->N;
    int dig[3];
    int rem = (int)j;
    dig[2] = rem % N;
    rem /= N;
    dig[1] = rem % N;
    dig[0] = rem / N;
    const double dxdp = 2.0 / gc->pmax;
    for (int i = 0; i < 3; ++i) {
        const long long stride = i == 0 ? (long long)N * N : (i == 1 ? N : 1);
        const long long base = j - dig[i] * stride;
        const double *Vi = V0 + i * NN;
        double dv = 0.0;
        for (int k = 0; k < N; ++k) dv += gc->Dd[dig[i] * kMaxN + k] * Vi[base + k * stride];
        const double u = gc->A[i] + gc->delta * gc->beta[i] * dxdp * dv;
        U0[i * NN + j] = u < 0.0 ? 0.0 : (u > gc->umax ? gc->umax : u);
    }
}

__global__ void k_fill_f64(double *p, long long n, double v)
{
    for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < n;
         e += (long long)gridDim.x * blockDim.x)
        p[e] = v;
}

__global__ void k_fill_i32(int *p, int v) { *p = v; }

inline size_t a256(size_t x) { return (x + 255) & ~(size_t)255; }

// Workspace sections for minibatches of up to nb rows.
struct MlpWs {
    size_t Xb, Tb, Z[3], H[3], Y, dY, dZa, dZb, part, lossp, loss, grad, V0, U0, bad, total;
    MlpWs(int nb)
    {
        size_t o = 0;
        auto take = [&](size_t bytes) { size_t r = o; o = a256(o + bytes); return r; };
        Xb = take(sizeof(float) * nb * IN);
        Tb = take(sizeof(float) * nb * OUT);
        for (int l = 0; l < 3; ++l) {
            Z[l] = take(sizeof(float) * nb * HID);
            H[l] = take(sizeof(float) * nb * HID);
        }
        Y = take(sizeof(float) * nb * OUT);
        dY = take(sizeof(float) * nb * OUT);
        dZa = take(sizeof(float) * nb * HID);
        dZb = take(sizeof(float) * nb * HID);
        part = take(sizeof(float) * MAX_SPLIT * (HID + 1) * HID);
        lossp = take(sizeof(float) * LOSS_BLOCKS);
        loss = take(sizeof(float) * 4);
        grad = take(sizeof(float) * P_TOTAL);
        V0 = take(sizeof(double) * 3 * MAX_NODES);
        U0 = take(sizeof(double) * 3 * MAX_NODES);
        bad = take(sizeof(int) * 4);
        total = o;
    }
};

// Splits of a K range of length K into at most S chunks of a multiple of 16.
inline int plan_split(int K, int S, int &kchunk)
{
    kchunk = (K + S - 1) / S;
    kchunk = (kchunk + 15) / 16 * 16;
    if (kchunk < 16) kchunk = 16;
    const int n = (K + kchunk - 1) / kchunk;
    return n < 1 ? 1 : n;
}

template <bool TA, bool TB, bool ONES, int EPI>
hipError_t gemm(int M, int N, int K, int S, const float *A, int lda, const float *B, int ldb, float *C, int ldc,
                long long split_stride, const float *bias, float *H, const float *Zs, hipStream_t s)
{
    if (M <= 0 || N <= 0) return hipSuccess;
    int kchunk;
    S = plan_split(K, S, kchunk);
    dim3 grid((M + 63) / 64, (N + 63) / 64, S);
    hipLaunchKernelGGL((k_gemm<TA, TB, ONES, EPI>), grid, dim3(256), 0, s, M, N, K, kchunk, A, lda, B, ldb, C, ldc,
                       split_stride, bias, H, Zs);
    return hipGetLastError();
}

inline int splits_for(int n)
{
    int S = n / 128;
    return S < 1 ? 1 : (S > MAX_SPLIT ? MAX_SPLIT : S);
}

// Forward over nb rows of Xb.  train: keep Z and H of every hidden layer; else
// only H (ping-pong through H[0], H[1]).
hipError_t forward(const float *P, const float *Xb, int nb, char *ws, const MlpWs &L, float *Y, bool train,
                   hipStream_t s)
{
    hipError_t e = hipSuccess;
    const float *a = Xb;
    int lda = IN;
    for (int l = 0; l < 3 && e == hipSuccess; ++l) {
        const float *W = P + layer_off(l);
        const float *b = W + (long long)FAN_IN[l] * FAN_OUT[l];
        float *Hl = (float *)(ws + L.H[train ? l : (l & 1)]);
        if (train)
            e = gemm<false, false, false, EPI_BIAS_GELU>(nb, HID, FAN_IN[l], 1, a, lda, W, HID,
                                                          (float *)(ws + L.Z[l]), HID, 0, b, Hl, nullptr, s);
        else
            e = gemm<false, false, false, EPI_GELU_ONLY>(nb, HID, FAN_IN[l], 1, a, lda, W, HID, nullptr, HID, 0, b,
                                                          Hl, nullptr, s);
        a = Hl;
        lda = HID;
    }
    if (e != hipSuccess) return e;
    const float *W4 = P + layer_off(3);
    return gemm<false, false, false, EPI_BIAS>(nb, OUT, HID, 1, a, HID, W4, OUT, Y, OUT, 0,
                                               W4 + (long long)HID * OUT, nullptr, nullptr, s);
}

// Loss and gradient of the minibatch (Xb, Tb) of nb rows; grad = [W; b] per layer.
hipError_t grad_pass(const float *P, const float *Xb, const float *Tb, int nb, char *ws, const MlpWs &L, float *grad,
                     float *loss, hipStream_t s)
{
    float *Y = (float *)(ws + L.Y), *dY = (float *)(ws + L.dY);
    hipError_t e = forward(P, Xb, nb, ws, L, Y, true, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_mse, dim3(LOSS_BLOCKS), dim3(256), 0, s, Y, Tb, nb, dY, (float *)(ws + L.lossp));
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if (loss) {
        hipLaunchKernelGGL(k_loss_final, dim3(1), dim3(64), 0, s, (const float *)(ws + L.lossp), LOSS_BLOCKS, nb, loss);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    const int S = splits_for(nb);
    float *part = (float *)(ws + L.part);
    const float *dz = dY;
    float *dz_next[2] = {(float *)(ws + L.dZa), (float *)(ws + L.dZb)};
    for (int l = NL - 1; l >= 0; --l) {
        const int fi = FAN_IN[l], fo = FAN_OUT[l];
        const float *a_in = l == 0 ? Xb : (const float *)(ws + L.H[l - 1]);
        const long long n_wb = (long long)(fi + 1) * fo;
        // [dW; db] = [a_in | 1]^T dz over the batch, split over the batch
        e = gemm<true, false, true, EPI_STORE>(fi + 1, fo, nb, S, a_in, fi, dz, fo, part, fo, n_wb, nullptr, nullptr,
                                               nullptr, s);
        if (e != hipSuccess) return e;
        int kchunk;
        const int Su = plan_split(nb, S, kchunk);
        hipLaunchKernelGGL(k_split_reduce, dim3((unsigned)((n_wb + 255) / 256)), dim3(256), 0, s, part, n_wb, Su,
                           n_wb, grad + layer_off(l));
        if ((e = hipGetLastError()) != hipSuccess) return e;
        if (l == 0) break;
        // dz_{l-1} = (dz W_l^T) * gelu'(z_{l-1})
        float *out = dz_next[l & 1];
        e = gemm<false, true, false, EPI_GELU_BWD>(nb, fi, fo, 1, dz, fo, P + layer_off(l), fo, out, fi, 0, nullptr,
                                                   nullptr, (const float *)(ws + L.Z[l - 1]), s);
        if (e != hipSuccess) return e;
        dz = out;
    }
    return hipSuccess;
}

bool ws_ok(const void *ws, size_t ws_bytes, int nb)
{
    return ws && !((uintptr_t)ws & 255) && ws_bytes >= MlpWs(nb).total;
}

hipError_t infer_game(const GameConst &hc, const float *P, const float *theta, double out_scale, char *ws, int nb,
                      const MlpWs &L, double *V0, int *bad, const cg_game *g, hipStream_t s)
{
    Theta th;
    for (int c = 0; c < 6; ++c) th.t[c] = theta[c];
    const InstPtrs &I = game_inst(g);
    hipError_t e = hipSuccess;
    for (long long r0 = 0; r0 < hc.NN && e == hipSuccess; r0 += nb) {
        const int cnt = (int)(hc.NN - r0 < nb ? hc.NN - r0 : nb);
        float *Xb = (float *)(ws + L.Xb), *Y = (float *)(ws + L.Y);
        hipLaunchKernelGGL(k_features, dim3((cnt + 255) / 256), dim3(256), 0, s, I.gc, I.st, I.V, th, 0.0, r0, cnt,
                           Xb, (float *)nullptr);
        if ((e = hipGetLastError()) != hipSuccess) break;
        e = forward(P, Xb, cnt, ws, L, Y, false, s);
        if (e != hipSuccess) break;
        hipLaunchKernelGGL(k_warm_write, dim3((cnt + 255) / 256), dim3(256), 0, s, Y, cnt, r0, hc.NN, out_scale, V0,
                           bad);
        e = hipGetLastError();
    }
    return e;
}

int dev_err(hipError_t e, const char *where)
{
    static thread_local char buf[256];
    snprintf(buf, sizeof buf, "%s: %s", where, hipGetErrorString(e));
    return set_error(CG_EDEVICE, buf);
}

}  // namespace

extern "C" {

int64_t cg_mlp_param_count(void) { return P_TOTAL; }

size_t cg_mlp_workspace_bytes(int32_t batch)
{
    if (batch < 1 || batch > MAX_BATCH) return 0;
    return MlpWs(batch).total;
}

int cg_mlp_forward(const float *params, const float *X, int64_t n, float *Y, int32_t batch, void *ws,
                   size_t ws_bytes, void *stream)
{
    if (n < 0) return set_error(CG_EINVAL, "n < 0");
    if (n == 0) return CG_OK;
    if (!params || !X || !Y) return set_error(CG_EINVAL, "NULL pointer");
    if (batch < 1 || batch > MAX_BATCH) return set_error(CG_EINVAL, "batch out of range");
    if (!ws_ok(ws, ws_bytes, batch)) return set_error(CG_ENOMEM, "workspace NULL, misaligned or too small");
    const MlpWs L(batch);
    hipStream_t s = (hipStream_t)stream;
    for (long long r0 = 0; r0 < n; r0 += batch) {
        const int cnt = (int)(n - r0 < batch ? n - r0 : batch);
        hipError_t e = forward(params, X + r0 * IN, cnt, (char *)ws, L, Y + r0 * OUT, false, s);
        if (e != hipSuccess) return dev_err(e, "mlp forward");
    }
    return CG_OK;
}

int cg_mlp_grad(const float *params, const float *X, const float *T, int32_t n, float *grad, float *loss, void *ws,
                size_t ws_bytes, void *stream)
{
    if (!params || !X || !T || !grad) return set_error(CG_EINVAL, "NULL pointer");
    if (n < 1 || n > MAX_BATCH) return set_error(CG_EINVAL, "n out of range");
    if (!ws_ok(ws, ws_bytes, n)) return set_error(CG_ENOMEM, "workspace NULL, misaligned or too small");
    const MlpWs L(n);
    hipError_t e = grad_pass(params, X, T, n, (char *)ws, L, grad, loss, (hipStream_t)stream);
    return e == hipSuccess ? CG_OK : dev_err(e, "mlp grad");
}

int cg_mlp_adam(float *params, const float *grad, float *m, float *v, int32_t t, float lr, float beta1, float beta2,
                float eps, void *stream)
{
    if (!params || !grad || !m || !v) return set_error(CG_EINVAL, "NULL pointer");
    if (t < 1) return set_error(CG_EINVAL, "Adam step t < 1");
    const float c1 = (float)(1.0 / (1.0 - pow((double)beta1, t)));
    const float c2 = (float)(1.0 / (1.0 - pow((double)beta2, t)));
    hipLaunchKernelGGL(k_adam, dim3(264), dim3(512), 0, (hipStream_t)stream, params, grad, m, v, P_TOTAL, lr, beta1,
                       beta2, eps, c1, c2);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? CG_OK : dev_err(e, "adam");
}

int cg_mlp_train(float *params, float *m, float *v, const float *X, const float *T, int64_t n_samples, int32_t batch,
                 int32_t steps, int32_t t0, float lr, uint64_t seed, float *losses, void *ws, size_t ws_bytes,
                 void *stream)
{
    if (!params || !m || !v || !X || !T) return set_error(CG_EINVAL, "NULL pointer");
    if (n_samples < 1 || steps < 0 || t0 < 0) return set_error(CG_EINVAL, "n_samples < 1, steps < 0 or t0 < 0");
    if (batch < 1 || batch > MAX_BATCH) return set_error(CG_EINVAL, "batch out of range");
    if (!ws_ok(ws, ws_bytes, batch)) return set_error(CG_ENOMEM, "workspace NULL, misaligned or too small");
    const MlpWs L(batch);
    char *w = (char *)ws;
    hipStream_t s = (hipStream_t)stream;
    float *Xb = (float *)(w + L.Xb), *Tb = (float *)(w + L.Tb), *g = (float *)(w + L.grad);
    for (int k = 0; k < steps; ++k) {
        const long long t = (long long)t0 + k;
        hipLaunchKernelGGL(k_gather, dim3((batch + 255) / 256), dim3(256), 0, s, X, T, (long long)n_samples, batch,
                           (unsigned long long)seed, t, Xb, Tb);
        hipError_t e = hipGetLastError();
        if (e == hipSuccess) e = grad_pass(params, Xb, Tb, batch, w, L, g, losses ? losses + k : nullptr, s);
        if (e != hipSuccess) return dev_err(e, "mlp train");
        const int rc = cg_mlp_adam(params, g, m, v, (int32_t)(t + 1), lr, 0.9f, 0.999f, 1e-8f, stream);
        if (rc != CG_OK) return rc;
    }
    return CG_OK;
}

int cg_mlp_features(cg_game *game, const float *theta, double t_scale, float *X, float *T)
{
    if (!game || !theta || !X) return set_error(CG_EINVAL, "NULL pointer");
    const GameConst &hc = game_consts(game);
    if (hc.d != 3) return set_error(CG_EUNSUPPORTED, "the warm-start network is for d = 3 games");
    Theta th;
    for (int c = 0; c < 6; ++c) th.t[c] = theta[c];
    const InstPtrs &I = game_inst(game);
    hipStream_t s = game_stream(game);
    hipLaunchKernelGGL(k_features, dim3((unsigned)((hc.NN + 255) / 256)), dim3(256), 0, s, I.gc, I.st, I.V, th,
                       t_scale, 0LL, (int)hc.NN, X, T);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? CG_OK : dev_err(e, "features");
}

int cg_warm_start(cg_game *game, const float *params, const float *theta, double out_scale, void *ws,
                  size_t ws_bytes, int32_t batch, int32_t *nonfinite)
{
    if (!game || !params || !theta) return set_error(CG_EINVAL, "NULL pointer");
    const GameConst &hc = game_consts(game);
    if (hc.d != 3) return set_error(CG_EUNSUPPORTED, "the warm-start network is for d = 3 games");
    if (batch < 1 || batch > MAX_BATCH) return set_error(CG_EINVAL, "batch out of range");
    if (!ws_ok(ws, ws_bytes, batch)) return set_error(CG_ENOMEM, "workspace NULL, misaligned or too small");
    const MlpWs L(batch);
    char *w = (char *)ws;
    hipStream_t s = game_stream(game);
    double *V0 = (double *)(w + L.V0);
    int *bad = (int *)(w + L.bad);
    hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(1), 0, s, bad, 0);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = infer_game(hc, params, theta, out_scale, w, batch, L, V0, bad, game, s);
    if (e != hipSuccess) return dev_err(e, "warm start");
    int hbad = 0;
    e = hipMemcpyAsync(&hbad, bad, sizeof(int), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return dev_err(e, "warm start flag");
    if (nonfinite) *nonfinite = hbad;
    if (hbad) {  // fall back to the zero start
        hipLaunchKernelGGL(k_fill_f64, dim3(256), dim3(256), 0, s, V0, 3 * hc.NN, 0.0);
        if ((e = hipGetLastError()) != hipSuccess) return dev_err(e, "warm start fallback");
        return cg_set_state(game, V0, nullptr);
    }
    double *U0 = (double *)(w + L.U0);
    hipLaunchKernelGGL(k_warm_controls, dim3((unsigned)((hc.NN + 255) / 256)), dim3(256), 0, s, game_inst(game).gc,
                       V0, U0);
    if ((e = hipGetLastError()) != hipSuccess) return dev_err(e, "warm controls");
    return cg_set_state(game, V0, U0);
}

int cg_solve_warm(cg_game *game, const float *params, const float *theta, double out_scale, int32_t max_steps,
                  double tol, int32_t probe_steps, void *ws, size_t ws_bytes, int32_t batch, int32_t *steps_done,
                  double *residual, int32_t *fell_back)
{
    if (!game || !params || !theta) return set_error(CG_EINVAL, "NULL pointer");
    if (max_steps < 2 || probe_steps < 1 || probe_steps >= max_steps)
        return set_error(CG_EINVAL, "need 1 <= probe_steps < max_steps");
    if (!(tol > 0.0)) return set_error(CG_EINVAL, "tol must be > 0");
    if (game_consts(game).d != 3) return set_error(CG_EUNSUPPORTED, "the warm-start network is for d = 3 games");
    if (batch < 1 || batch > MAX_BATCH) return set_error(CG_EINVAL, "batch out of range");
    if (!ws_ok(ws, ws_bytes, batch)) return set_error(CG_ENOMEM, "workspace NULL, misaligned or too small");
    const GameConst &hc = game_consts(game);
    const MlpWs L(batch);
    double *V0 = (double *)((char *)ws + L.V0);
    hipStream_t s = game_stream(game);
    int total = 0, n = 0, rc;
    double r0 = 0.0, r = 0.0;
    // residual of the first iteration from the zero start: the bar a warm start must beat
    auto zero_state = [&]() -> int {
        hipLaunchKernelGGL(k_fill_f64, dim3(256), dim3(256), 0, s, V0, 3 * hc.NN, 0.0);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return dev_err(e, "zero state");
        return cg_set_state(game, V0, nullptr);
    };
    if ((rc = zero_state()) != CG_OK) return rc;
    rc = cg_solve(game, 1, 0.0, &n, &r0);
    total += n;
    if (rc < 0) return rc;
    int32_t bad = 0;
    if ((rc = cg_warm_start(game, params, theta, out_scale, ws, ws_bytes, batch, &bad)) != CG_OK) return rc;
    bool fallback = bad != 0;
    if (!fallback) {
        rc = cg_solve(game, probe_steps, tol, &n, &r);
        total += n;
        if (rc == CG_ENONFINITE || (rc >= 0 && !(r <= r0))) fallback = true;
        else if (rc < 0) return rc;
        else if (rc == CG_OK) {  // converged within the probe
            if (steps_done) *steps_done = total;
            if (residual) *residual = r;
            if (fell_back) *fell_back = 0;
            return CG_OK;
        } else {
            rc = cg_solve(game, max_steps - total, tol, &n, &r);
            total += n;
            if (steps_done) *steps_done = total;
            if (residual) *residual = r;
            if (fell_back) *fell_back = 0;
            return rc;
        }
    }
    // the plain method from the zero start
    if ((rc = zero_state()) != CG_OK) return rc;
    rc = cg_solve(game, max_steps - total > 0 ? max_steps - total : 1, tol, &n, &r);
    total += n;
    if (steps_done) *steps_done = total;
    if (residual) *residual = r;
    if (fell_back) *fell_back = 1;
    return rc;
}

}  // extern "C"
