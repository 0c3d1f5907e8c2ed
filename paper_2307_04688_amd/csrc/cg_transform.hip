// cg_transform.hip -- coefficient transform of Algorithm Cnv (Section 3.1):
// the 1-D interpolation rule of eq. (forcoef) applied along every mode.
//
// Along one mode of size N (n = N-1 intervals) the rule is the DCT-I
//   c_l = (w_l / n) sum_k e_k F_k cos(pi l k / n),  w_0 = w_n = 1, else 2,
//   e_0 = e_n = 1/2, else 1.
// One thread owns one fibre: it loads the N values into registers, then
// writes the N coefficients back, so a pass may run in place.  The N x N
// matrix is built in LDS by each block.  The transform is a small share of a
// step (2 d N^(d+1) flops per tensor against 2 N^(2d) for the contraction).
#include "cg_internal.h"

namespace cg {

__device__ inline double dct1_entry(int l, int k, int N)
{
    const int n = N - 1;
    const int r = (l * k) % (2 * n);
    double v = cospi((double)r / (double)n);
    if (k == 0 || k == n) v *= 0.5;
    return v * ((l == 0 || l == n) ? 1.0 : 2.0) / (double)n;
}

__global__ __launch_bounds__(256) void k_transform_mode(const double *in, double *out, long long fibers,
                                                        long long fpt, long long stride, int N,
                                                        long long total)
{
    __shared__ double Dm[kMaxN * kMaxN];
    for (int e = threadIdx.x; e < N * N; e += blockDim.x) Dm[e] = dct1_entry(e / N, e % N, N);
    __syncthreads();
    const long long f = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (f >= fibers) return;
    const long long b = f / fpt, r = f % fpt;
    const long long o = r / stride, i = r % stride;
    const long long base = b * total + o * (long long)N * stride + i;
    double x[kMaxN];
#pragma unroll
    for (int k = 0; k < kMaxN; ++k)
        if (k < N) x[k] = in[base + k * stride];
    for (int l = 0; l < N; ++l) {
        double acc = 0.0;
#pragma unroll
        for (int k = 0; k < kMaxN; ++k)
            if (k < N) acc = fma(Dm[l * N + k], x[k], acc);
        out[base + l * stride] = acc;
    }
}

hipError_t launch_transform_mode(const double *in, double *out, int d, const int *n, int mode,
                                 long long batch, const double *, hipStream_t s)
{
    long long total = 1, stride = 1;
    for (int l = 0; l < d; ++l) total *= n[l];
    for (int l = mode + 1; l < d; ++l) stride *= n[l];
    const long long fpt = total / n[mode];
    const long long fibers = fpt * batch;
    if (fibers == 0) return hipSuccess;
    const int threads = 256;
    const long long blocks = (fibers + threads - 1) / threads;
    hipLaunchKernelGGL(k_transform_mode, dim3((unsigned)blocks), dim3(threads), 0, s, in, out, fibers, fpt,
                       stride, n[mode], total);
    return hipGetLastError();
}

hipError_t run_transform(int d, const int *n, const double *vals, double *coef, long long batch,
                         hipStream_t s)
{
    for (int m = 0; m < d; ++m) {
        hipError_t e = launch_transform_mode(m == 0 ? vals : coef, coef, d, n, m, batch, nullptr, s);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

// Game transform, one mode per launch, one thread per output coefficient:
//   out[i][.., l, ..] = sum_k Dx[l][k] in[i][.., k, ..]
// Mode 0 reads the current state buffer (chosen on the device by the status
// word); the last pass writes the packed contraction operand of each player
// directly: Bp[i][kidx][col] with col = k_i and kidx enumerating the other
// modes in increasing order, the last of them padded to N4 (the padding
// entries are zero from initialisation and never written).
__global__ __launch_bounds__(256) void k_transform_pass(const GameConst *__restrict__ gc, const GameStatus *st,
                                                        const double *Vbuf, const double *in, double *out,
                                                        double *Bp, int mode, int last)
{
    __shared__ double Dm[kMaxN * kMaxN];
    if (st->converged) return;
    const int N = gc->N, d = gc->d;
    for (int e = threadIdx.x; e < N * N; e += blockDim.x) Dm[e] = gc->Dx[(e / N) * kMaxN + e % N];
    __syncthreads();
    const int NN = (int)gc->NN;
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= d * NN) return;
    const int i = t / NN, idx = t % NN;
    int stride = 1;
    for (int l = mode + 1; l < d; ++l) stride *= N;
    const int lo = (idx / stride) % N;
    const int base = idx - lo * stride;
    const double *src = (mode == 0 ? Vbuf + (long long)st->cur * d * NN : in) + (long long)i * NN + base;
    const double *Drow = Dm + lo * N;
    double acc = 0.0;
    for (int k = 0; k < N; ++k) acc = fma(Drow[k], src[(long long)k * stride], acc);
    if (!last) {
        out[t] = acc;
        return;
    }
    const int lastother = (i == d - 1) ? d - 2 : d - 1;
    int rem = idx, col = 0, kl = 0, kout = 0, mul = 1;
    int dig[kMaxD];
    for (int l = d - 1; l >= 0; --l) { dig[l] = rem % N; rem /= N; }
    for (int l = 0; l < d; ++l) {
        if (l == i) col = dig[l];
        else if (l == lastother) kl = dig[l];
        else kout = kout * N + dig[l];
    }
    (void)mul;
    const long long kidx = (long long)kout * gc->N4 + kl;
    Bp[((long long)i * gc->K + kidx) * gc->NC + col] = acc;
}

hipError_t launch_transform_game(const GameConst &hc, const StepBuffers &b, hipStream_t s)
{
    const long long total = hc.NN * hc.d;
    const int threads = 256;
    const unsigned blocks = (unsigned)((total + threads - 1) / threads);
    // ping-pong: V -> tmp -> coef -> tmp ... ; the last pass writes Bp
    const double *in = nullptr;
    for (int m = 0; m < hc.d; ++m) {
        const int last = (m == hc.d - 1);
        double *out = (m % 2 == 0) ? b.tmp : b.coef;
        hipLaunchKernelGGL(k_transform_pass, dim3(blocks), dim3(threads), 0, s, b.gc, b.status, b.V, in, out, b.Bp,
                           m, last);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        in = out;
    }
    return hipSuccess;
}

}  // namespace cg
