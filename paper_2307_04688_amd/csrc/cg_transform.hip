// cg_transform.hip -- coefficient transform of Algorithm Cnv (Section 3.1):
// the 1-D interpolation rule of eq. (forcoef) applied along every mode.
//
// Along one mode of size N (n = N-1 intervals) the rule is the DCT-I
//   c_l = (w_l / n) sum_k e_k F_k cos(pi l k / n),  w_0 = w_n = 1, else 2,
//   e_0 = e_n = 1/2, else 1.
// The generic pass (any shape, any batch) stages whole fibres in LDS and
// writes one coefficient per thread, so it may run in place; the N x N
// matrix is built in LDS by each block.  The transform is a small share of a
// step (2 d N^(d+1) flops per tensor against 2 N^(2d) for the contraction).
#include "cg_tf.h"

namespace cg {

// One pass along a mode: a block owns 256 / N whole fibres, stages them in
// LDS and writes their N coefficients with one thread per output (so a pass
// may run in place: every fibre is read before any of it is written, and
// blocks own disjoint fibres).  Consecutive threads take consecutive fibres
// of the same coefficient, which are adjacent in memory for every mode but
// the last.
__global__ __launch_bounds__(256) void k_transform_mode(const double *in, double *out, long long fibers,
                                                        long long fpt, long long stride, int N,
                                                        long long total)
{
    __shared__ double Dm[kMaxN * kMaxN];
    __shared__ double X[256];
    for (int e = threadIdx.x; e < N * N; e += blockDim.x) Dm[e] = dct1_entry(e / N, e % N, N);
    const int FB = 256 / N;
    const int t = threadIdx.x;
    const int l = t / FB, fl = t % FB;
    const long long f = (long long)blockIdx.x * FB + fl;
    const bool ok = l < N && f < fibers;
    long long base = 0;
    if (ok) {
        const long long b = f / fpt, r = f % fpt;
        const long long o = r / stride, i = r % stride;
        base = b * total + o * (long long)N * stride + i;
        X[fl * N + l] = in[base + l * stride];
    }
    __syncthreads();
    if (ok) {
        double acc = 0.0;
        for (int k = 0; k < N; ++k) acc = fma(Dm[l * N + k], X[fl * N + k], acc);
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
    const long long fb = threads / n[mode];
    const long long blocks = (fibers + fb - 1) / fb;
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

// Game transform in two launches, both tiled through LDS.
//  1. k_tf_fast: the two fastest modes (d-2, d-1) of every N x N slice:
//     S -> D S D^T.  For d = 2 that is the whole transform and the result goes
//     straight to the packed operand.
//  2. k_tf_outer (d >= 3): the remaining modes 0..d-3 on a tile of N^(d-2)
//     fibres x Q consecutive inner positions, then the packed operand:
//     Bp[i][kidx][col], col = k_i, kidx enumerating the other modes in
//     increasing order with the last of them padded to N4 (padding entries are
//     zero from initialisation and never written).
template <int NP>
__global__ __launch_bounds__(256) void k_tf_fast(const Inst *__restrict__ tab, int bpi, int mixed)
{
    __shared__ double sm[3 * kMaxN * (kMaxN + 1)];
    tf_fast_block<NP>(tab, bpi, mixed, blockIdx.x, sm);
}

// Tile of the outer modes: X[f][q], f over the N^(d-2) outer positions,
// q over Q consecutive inner positions (the two fast modes flattened).
__global__ __launch_bounds__(256) void k_tf_outer(const Inst *__restrict__ tab, int bpi, int mixed, int Q)
{
    const InstView I = inst_view(tab, blockIdx.x / bpi);
    const int blk = blockIdx.x % bpi;
    const GameConst *__restrict__ gc = I.gc;
    const GameStatus *st = I.st;
    const double *__restrict__ in = I.tmp;
    double *Bp = I.Bp;
    float *Bp32 = mixed ? I.Bp32 : nullptr;
    unsigned short *Bs16 = mixed && corr3_split16(gc->d, gc->N4) ? I.Bs16 : nullptr;
    extern __shared__ double sh[];
    if (st->converged) return;
    const int N = gc->N, d = gc->d, NN2 = N * N;
    const long long NN = gc->NN;
    const int F = (int)(NN / NN2);          // N^(d-2) outer positions
    const int nq = (NN2 + Q - 1) / Q;       // tiles per player
    const int i = blk / nq, q0 = (blk % nq) * Q;
    constexpr int LD = kMaxN + 1;
    double *Dm = sh;                        // N x N, row stride LD
    double *X = sh + kMaxN * LD;            // F x Q
    double *Y = X + F * Q;                  // F x Q (d == 4 intermediate)
    const double *src = in + (long long)i * NN;
    for (int e = threadIdx.x; e < NN2; e += blockDim.x) Dm[(e / N) * LD + e % N] = gc->Dx[(e / N) * kMaxN + e % N];
    for (int e = threadIdx.x; e < F * Q; e += blockDim.x) {
        const int f = e / Q, q = q0 + e % Q;
        X[e] = q < NN2 ? src[(long long)f * NN2 + q] : 0.0;
    }
    __syncthreads();
    if (d == 3) {  // mode 0
        for (int e = threadIdx.x; e < F * Q; e += blockDim.x) {
            const int l = e / Q, qq = e % Q, q = q0 + qq;
            if (q >= NN2) continue;
            double acc = 0.0;
            for (int k = 0; k < N; ++k) acc = fma(Dm[l * LD + k], X[k * Q + qq], acc);
            int dig[kMaxD] = {l, q / N, q % N, 0};
            if (Bs16) { store_split16(Bs16, gc, i, dig, acc); continue; }
            const long long o = packed_index(gc, i, dig);
            if (Bp32) Bp32[o] = (float)acc; else Bp[o] = acc;
        }
    } else {  // d == 4: mode 0 then mode 1; f = a * N + b
        for (int e = threadIdx.x; e < F * Q; e += blockDim.x) {
            const int la = e / (N * Q), b = (e / Q) % N, qq = e % Q;
            double acc = 0.0;
            for (int k = 0; k < N; ++k) acc = fma(Dm[la * LD + k], X[(k * N + b) * Q + qq], acc);
            Y[e] = acc;
        }
        __syncthreads();
        for (int e = threadIdx.x; e < F * Q; e += blockDim.x) {
            const int a = e / (N * Q), lb = (e / Q) % N, qq = e % Q, q = q0 + qq;
            if (q >= NN2) continue;
            double acc = 0.0;
            for (int k = 0; k < N; ++k) acc = fma(Dm[lb * LD + k], Y[(a * N + k) * Q + qq], acc);
            int dig[kMaxD] = {a, lb, q / N, q % N};
            const long long o = packed_index(gc, i, dig);
            if (Bp32) Bp32[o] = (float)acc; else Bp[o] = acc;
        }
    }
}

// d = 3: mode 0 on FP64 MFMA.  Block = (player, NP consecutive inner
// positions q of the two fast modes): Out[l][q] = sum_k D[l][k] X[k][q], then
// the packed operand.
template <int NP>
__global__ __launch_bounds__(256) void k_tf_mode0(const Inst *__restrict__ tab, int bpi, int mixed)
{
    const InstView I = inst_view(tab, blockIdx.x / bpi);
    const int blk = blockIdx.x % bpi;
    const GameConst *__restrict__ gc = I.gc;
    const GameStatus *st = I.st;
    const double *__restrict__ in = I.tmp;
    double *Bp = I.Bp;
    float *Bp32 = mixed ? I.Bp32 : nullptr;
    unsigned short *Bs16 = mixed && corr3_split16(gc->d, gc->N4) ? I.Bs16 : nullptr;
    constexpr int LD = kMaxN + 1;
    __shared__ double Dm[kMaxN * LD];
    __shared__ double X[kMaxN * LD];
    if (st->converged) return;
    const int N = gc->N, NN2 = N * N;
    const long long NN = gc->NN;
    const int nq = (NN2 + NP - 1) / NP;
    const int i = blk / nq, q0 = (blk % nq) * NP;
    const double *src = in + (long long)i * NN;
    for (int e = threadIdx.x; e < NP * NP; e += blockDim.x) {  // zero beyond N and NN2
        const int r = e / NP, c = e % NP;
        Dm[r * LD + c] = (r < N && c < N) ? gc->Dx[r * kMaxN + c] : 0.0;
        X[r * LD + c] = (r < N && q0 + c < NN2) ? src[(long long)r * NN2 + q0 + c] : 0.0;
    }
    __syncthreads();
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int r16 = lane & 15, kq = lane >> 4;
    f64x4 acc;
    int ti, tj;
    if (plane_mfma<NP, LD, false, false>(Dm, X, wave, lane, acc, ti, tj)) {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int l = ti * 16 + kq + 4 * v, q = q0 + tj * 16 + r16;
            if (l >= N || q >= NN2) continue;
            int dig[kMaxD] = {l, q / N, q % N, 0};
            if (Bs16) { store_split16(Bs16, gc, i, dig, acc[v]); continue; }
            const long long o = packed_index(gc, i, dig);
            if (Bp32) Bp32[o] = (float)acc[v]; else Bp[o] = acc[v];
        }
    }
}

hipError_t launch_transform_game(const GameConst &hc, const StepBuffers &b, hipStream_t s)
{
    const int N = hc.N, d = hc.d;
    const int mixed = b.precision == CG_FP32_CORR;  // packed operand in binary32
    const long long nslice = hc.NN / (N * N);
    const int bpi1 = (int)(nslice * d);
    if (N <= 16)
        hipLaunchKernelGGL(k_tf_fast<16>, dim3((unsigned)(bpi1 * b.count)), dim3(256), 0, s, b.tab, bpi1, mixed);
    else
        hipLaunchKernelGGL(k_tf_fast<32>, dim3((unsigned)(bpi1 * b.count)), dim3(256), 0, s, b.tab, bpi1, mixed);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return launch_transform_rest(hc, b, s);
}

hipError_t launch_transform_rest(const GameConst &hc, const StepBuffers &b, hipStream_t s)
{
    const int N = hc.N, d = hc.d;
    const int mixed = b.precision == CG_FP32_CORR;
    const long long nslice = hc.NN / (N * N);
    if (d == 2) return hipSuccess;
    if (d == 3) {
        const int NP = N <= 16 ? 16 : 32;
        const int bpi3 = d * ((N * N + NP - 1) / NP);
        if (NP == 16)
            hipLaunchKernelGGL(k_tf_mode0<16>, dim3((unsigned)(bpi3 * b.count)), dim3(256), 0, s, b.tab, bpi3, mixed);
        else
            hipLaunchKernelGGL(k_tf_mode0<32>, dim3((unsigned)(bpi3 * b.count)), dim3(256), 0, s, b.tab, bpi3, mixed);
        return hipGetLastError();
    }
    // Q inner positions per tile, so that the dynamic LDS (D plus one or two
    // F x Q tiles) stays within 64 KiB
    const int F = (int)nslice;
    const int tiles = d == 4 ? 2 : 1;
    int Q = (8192 - kMaxN * (kMaxN + 1)) / (tiles * F);
    Q = Q > 16 ? 16 : (Q < 1 ? 1 : Q);
    const size_t shmem = sizeof(double) * ((size_t)kMaxN * (kMaxN + 1) + (size_t)tiles * F * Q);
    const int nq = (N * N + Q - 1) / Q;
    const int bpi2 = nq * d;
    hipLaunchKernelGGL(k_tf_outer, dim3((unsigned)(bpi2 * b.count)), dim3(256), shmem, s, b.tab, bpi2, mixed, Q);
    return hipGetLastError();
}

}  // namespace cg
