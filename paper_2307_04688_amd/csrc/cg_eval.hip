// cg_eval.hip -- value of an n-dimensional Chebyshev series at arbitrary
// points (the evaluation of Section 3.2 with one point per mode).
//
// For points x_q the modes 0..d-2 are contracted at once as the GEMM
//     W (npts x n_{d-1}) = KR (npts x prod_{l<d-1} n_l) * C (.. x n_{d-1}),
// where row q of KR is the Khatri-Rao product of the basis vectors
// (T_k(x_{q,l}))_k and C is the coefficient tensor with the last mode as
// columns; then f(x_q) = sum_k W[q,k] T_k(x_{q,d-1}) by Clenshaw.  The GEMM
// runs on MFMA: f64 16x16x4 (CG_FP64), f32 16x16x4 (CG_FP32) or bf16
// 16x16x32 with f32 accumulation (CG_BF16).
#include "cg_internal.h"
#include "cg_line.h"

namespace cg {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

template <typename T>
__device__ __forceinline__ T to_elem(double v);
template <>
__device__ __forceinline__ double to_elem<double>(double v) { return v; }
template <>
__device__ __forceinline__ float to_elem<float>(double v) { return (float)v; }
template <>
__device__ __forceinline__ __bf16 to_elem<__bf16>(double v) { return (__bf16)(float)v; }

// Packed operand: Bp[kidx][col], kidx = (k_0..k_{d-3}) * N4 + k_{d-2} (the
// mode d-2 padded to N4 with zeros), col = k_{d-1} padded to NC.
template <typename T>
__global__ __launch_bounds__(256) void k_pack_eval(const double *__restrict__ coef, T *__restrict__ Bp, int d,
                                                   int n0, int n1, int n2, int n3, int N4, int NC, long long K,
                                                   long long Kpad)
{
    const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= Kpad * NC) return;
    const int n[4] = {n0, n1, n2, n3};
    const int col = (int)(e % NC);
    long long kidx = e / NC;
    const bool inK = kidx < K;  // rows past K pad the bf16 K-steps of 32
    const int kl = (int)(kidx % N4);
    kidx /= N4;
    double v = 0.0;
    if (inK && kl < n[d - 2] && col < n[d - 1]) {
        long long off = col, mul = n[d - 1];
        off += (long long)kl * mul;
        mul *= n[d - 2];
        for (int l = d - 3; l >= 0; --l) {
            const int k = (int)(kidx % n[l]);
            kidx /= n[l];
            off += (long long)k * mul;
            mul *= n[l];
        }
        v = coef[off];
    }
    Bp[e] = to_elem<T>(v);
}

template <typename TE>
struct MfmaF;
// Row of accumulator element v held by lane c + 16 g: the f64 16x16x4 form
// interleaves rows (g + 4 v), the f32 forms stack them (4 g + v).
template <>
struct MfmaF<double> {
    typedef f64x4 acc_t;
    static __device__ __forceinline__ int row(int g, int v) { return g + 4 * v; }
    static __device__ __forceinline__ acc_t run(double a, double b, acc_t c)
    {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
};
template <>
struct MfmaF<float> {
    typedef f32x4 acc_t;
    static __device__ __forceinline__ int row(int g, int v) { return 4 * g + v; }
    static __device__ __forceinline__ acc_t run(float a, float b, acc_t c)
    {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
};

// FP64 / FP32 evaluation: K-steps of 4, one A and one B element per lane.
template <typename TE, typename TO, int D, int N4, int NC, int RB>
__global__ __launch_bounds__(256) void k_eval_mfma(const TE *__restrict__ Bp, const double *__restrict__ X,
                                                   TO *__restrict__ out, long long npts, int n0, int n1,
                                                   int nlast)
{
    constexpr int NCB = NC / 16;
    constexpr int ROWS_W = RB * 16;
    constexpr int ROWS_B = 4 * ROWS_W;
    constexpr int LDW = NC + 1;
    typedef typename MfmaF<TE>::acc_t acc_t;
    __shared__ double Wl[ROWS_B * LDW];

    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int r16 = lane & 15, kq = lane >> 4;
    const long long row0 = (long long)blockIdx.x * ROWS_B + wave * ROWS_W;

    // basis of mode D-2 (last contracted) and the outer-mode coordinates
    double xo[RB][2];
    double Tl[RB][N4 / 4];
#pragma unroll
    for (int rb = 0; rb < RB; ++rb) {
        long long q = row0 + rb * 16 + r16;
        q = q < npts ? q : npts - 1;
        const double *xq = X + q * D;
        xo[rb][0] = D >= 3 ? xq[0] : 0.0;
        xo[rb][1] = D >= 4 ? xq[1] : 0.0;
        const double xl = xq[D - 2];
        double tm1 = 1.0, t0 = xl;
#pragma unroll
        for (int k = 0; k < N4; ++k) {
            double tk;
            if (k == 0) tk = 1.0;
            else if (k == 1) tk = xl;
            else { tk = 2.0 * xl * t0 - tm1; tm1 = t0; t0 = tk; }
            if ((k & 3) == kq) Tl[rb][k >> 2] = tk;
        }
    }

    acc_t acc[RB][NCB];
#pragma unroll
    for (int rb = 0; rb < RB; ++rb)
#pragma unroll
        for (int c = 0; c < NCB; ++c) acc[rb][c] = acc_t{0, 0, 0, 0};

    double Ta_prev[RB], Ta[RB], Tb_prev[RB], Tb[RB];
#pragma unroll
    for (int rb = 0; rb < RB; ++rb) { Ta_prev[rb] = 0.0; Ta[rb] = 1.0; Tb_prev[rb] = 0.0; Tb[rb] = 1.0; }
    // D == 3: outer mode 0 (n0).  D == 4: modes 0 (n0, slow) and 1 (n1, fast).
    const int n_outer = (D == 2) ? 1 : (D == 3 ? n0 : n0 * n1);
    for (int oc = 0; oc < n_outer; ++oc) {
        double F[RB];
#pragma unroll
        for (int rb = 0; rb < RB; ++rb) F[rb] = (D == 2) ? 1.0 : (D == 3 ? Ta[rb] : Ta[rb] * Tb[rb]);
        const TE *Brow = Bp + (long long)oc * N4 * NC + kq * NC + r16;
#pragma unroll
        for (int t = 0; t < N4 / 4; ++t) {
            TE bf[NCB];
#pragma unroll
            for (int c = 0; c < NCB; ++c) bf[c] = Brow[t * 4 * NC + c * 16];
#pragma unroll
            for (int rb = 0; rb < RB; ++rb) {
                const TE a = to_elem<TE>(F[rb] * Tl[rb][t]);
#pragma unroll
                for (int c = 0; c < NCB; ++c) acc[rb][c] = MfmaF<TE>::run(a, bf[c], acc[rb][c]);
            }
        }
        if (D == 3) {
#pragma unroll
            for (int rb = 0; rb < RB; ++rb) {
                const double tn = (oc == 0) ? xo[rb][0] : 2.0 * xo[rb][0] * Ta[rb] - Ta_prev[rb];
                Ta_prev[rb] = Ta[rb]; Ta[rb] = tn;
            }
        } else if (D == 4) {
            const int kb = oc % n1;
            if (kb == n1 - 1) {
                const int ka = oc / n1;
#pragma unroll
                for (int rb = 0; rb < RB; ++rb) {
                    const double tn = (ka == 0) ? xo[rb][0] : 2.0 * xo[rb][0] * Ta[rb] - Ta_prev[rb];
                    Ta_prev[rb] = Ta[rb]; Ta[rb] = tn;
                    Tb_prev[rb] = 0.0; Tb[rb] = 1.0;
                }
            } else {
#pragma unroll
                for (int rb = 0; rb < RB; ++rb) {
                    const double tn = (kb == 0) ? xo[rb][1] : 2.0 * xo[rb][1] * Tb[rb] - Tb_prev[rb];
                    Tb_prev[rb] = Tb[rb]; Tb[rb] = tn;
                }
            }
        }
    }

#pragma unroll
    for (int rb = 0; rb < RB; ++rb)
#pragma unroll
        for (int c = 0; c < NCB; ++c)
#pragma unroll
            for (int v = 0; v < 4; ++v)
                Wl[(wave * ROWS_W + rb * 16 + MfmaF<TE>::row(kq, v)) * LDW + c * 16 + r16] =
                    (double)acc[rb][c][v];
    __syncthreads();

    for (int row = tid; row < ROWS_B; row += 256) {
        const long long q = (long long)blockIdx.x * ROWS_B + row;
        if (q >= npts) continue;
        double w[NC];
#pragma unroll
        for (int k = 0; k < NC; ++k) w[k] = Wl[row * LDW + k];
        out[q] = (TO)clenshaw(w, X[q * D + D - 1]);  // columns >= nlast are zero
    }
}

// BF16 evaluation: v_mfma_f32_16x16x32_bf16, lane r + 16 g supplies A[r][8g..8g+7]
// and B[8g..8g+7][r]; K-steps of 32 over the packed K (padded to 32).
template <int D, int N4, int NC, int RB>
__global__ __launch_bounds__(256) void k_eval_bf16(const __bf16 *__restrict__ Bp, const double *__restrict__ X,
                                                   float *__restrict__ out, long long npts, int n0, int n1,
                                                   int nlast, long long Kpad)
{
    constexpr int NCB = NC / 16;
    constexpr int ROWS_W = RB * 16;
    constexpr int ROWS_B = 4 * ROWS_W;
    constexpr int LDW = NC + 1;
    __shared__ double Wl[ROWS_B * LDW];

    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int r16 = lane & 15, g = lane >> 4;
    const long long row0 = (long long)blockIdx.x * ROWS_B + wave * ROWS_W;

    // per row: full basis of mode D-2 (float) and outer coordinates
    float Tl[RB][N4];
    double xo[RB][2];
#pragma unroll
    for (int rb = 0; rb < RB; ++rb) {
        long long q = row0 + rb * 16 + r16;
        q = q < npts ? q : npts - 1;
        const double *xq = X + q * D;
        xo[rb][0] = D >= 3 ? xq[0] : 0.0;
        xo[rb][1] = D >= 4 ? xq[1] : 0.0;
        const double xl = xq[D - 2];
        double tm1 = 1.0, t0 = xl;
#pragma unroll
        for (int k = 0; k < N4; ++k) {
            double tk;
            if (k == 0) tk = 1.0;
            else if (k == 1) tk = xl;
            else { tk = 2.0 * xl * t0 - tm1; tm1 = t0; t0 = tk; }
            Tl[rb][k] = (float)tk;
        }
    }

    f32x4 acc[RB][NCB];
#pragma unroll
    for (int rb = 0; rb < RB; ++rb)
#pragma unroll
        for (int c = 0; c < NCB; ++c) acc[rb][c] = f32x4{0.f, 0.f, 0.f, 0.f};

    // K index kk = oc * N4 + kl; a K-step covers 32 consecutive kk.  Outer
    // factors F(oc) are recomputed per element from per-row recurrence tables.
    const int n_outer = (D == 2) ? 1 : (D == 3 ? n0 : n0 * n1);
    const int nsteps = (int)(Kpad / 32);
    for (int st = 0; st < nsteps; ++st) {
        const long long kbase = (long long)st * 32 + 8 * g;
        bf16x8 bfr[NCB];
#pragma unroll
        for (int c = 0; c < NCB; ++c) {
#pragma unroll
            for (int e = 0; e < 8; ++e) bfr[c][e] = Bp[(kbase + e) * NC + c * 16 + r16];
        }
#pragma unroll
        for (int rb = 0; rb < RB; ++rb) {
            bf16x8 a;
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const long long kk = kbase + e;
                const int kl = (int)(kk % N4);
                const int oc = (int)(kk / N4);
                float F = 1.0f;
                if (D >= 3 && oc < n_outer) {
                    // outer factor by direct recurrence (short: n0, n1 <= 32)
                    int ka = (D == 3) ? oc : oc / n1;
                    double x0 = xo[rb][0], tp = 1.0, tc = x0, T0 = 1.0;
                    if (ka == 0) T0 = 1.0; else if (ka == 1) T0 = x0;
                    else { for (int k = 2; k <= ka; ++k) { const double tn = 2.0 * x0 * tc - tp; tp = tc; tc = tn; } T0 = tc; }
                    double Ff = T0;
                    if (D == 4) {
                        const int kb = oc % n1;
                        double x1 = xo[rb][1], sp = 1.0, sc = x1, T1 = 1.0;
                        if (kb == 0) T1 = 1.0; else if (kb == 1) T1 = x1;
                        else { for (int k = 2; k <= kb; ++k) { const double sn = 2.0 * x1 * sc - sp; sp = sc; sc = sn; } T1 = sc; }
                        Ff *= T1;
                    }
                    F = (float)Ff;
                } else if (oc >= n_outer) {
                    F = 0.0f;
                }
                float tl = 0.0f;
#pragma unroll
                for (int k = 0; k < N4; ++k)
                    if (k == kl) tl = Tl[rb][k];
                a[e] = (__bf16)(F * tl);
            }
#pragma unroll
            for (int c = 0; c < NCB; ++c)
                acc[rb][c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, bfr[c], acc[rb][c], 0, 0, 0);
        }
    }

#pragma unroll
    for (int rb = 0; rb < RB; ++rb)
#pragma unroll
        for (int c = 0; c < NCB; ++c)
#pragma unroll
            for (int v = 0; v < 4; ++v)
                Wl[(wave * ROWS_W + rb * 16 + 4 * g + v) * LDW + c * 16 + r16] = (double)acc[rb][c][v];
    __syncthreads();

    for (int row = tid; row < ROWS_B; row += 256) {
        const long long q = (long long)blockIdx.x * ROWS_B + row;
        if (q >= npts) continue;
        double w[NC];
#pragma unroll
        for (int k = 0; k < NC; ++k) w[k] = Wl[row * LDW + k];
        out[q] = (float)clenshaw(w, X[q * D + D - 1]);  // columns >= nlast are zero
    }
}

// d == 1: Clenshaw per point.
template <typename TO>
__global__ __launch_bounds__(256) void k_eval_1d(const double *__restrict__ coef, const double *__restrict__ X,
                                                 TO *__restrict__ out, long long npts, int n, int precision)
{
    const long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= npts) return;
    const double x = X[q];
    double b1 = 0.0, b2 = 0.0;
    for (int k = n - 1; k >= 1; --k) {
        double c = coef[k];
        if (precision == CG_FP32) c = (double)(float)c;
        if (precision == CG_BF16) c = (double)(float)(__bf16)(float)c;
        const double b0 = fma(2.0 * x, b1, c - b2);
        b2 = b1;
        b1 = b0;
    }
    double c0 = coef[0];
    if (precision == CG_FP32) c0 = (double)(float)c0;
    if (precision == CG_BF16) c0 = (double)(float)(__bf16)(float)c0;
    out[q] = (TO)fma(x, b1, c0 - b2);
}

static inline int round4(int n) { return (n + 3) & ~3; }

static long long eval_K(int d, const int *n, int N4)
{
    long long K = N4;
    for (int l = 0; l < d - 2; ++l) K *= n[l];
    return K;
}

size_t eval_ws_bytes(int d, const int *n, int precision)
{
    if (d < 2) return 0;
    const int N4 = round4(n[d - 2]);
    const int NC = n[d - 1] <= 16 ? 16 : 32;
    long long K = eval_K(d, n, N4);
    size_t es = precision == CG_FP64 ? 8 : (precision == CG_FP32 ? 4 : 2);
    if (precision == CG_BF16) K = (K + 31) / 32 * 32;
    return (size_t)(K * NC) * es + 256;
}

template <typename TE, typename TO, int D, int N4>
static hipError_t launch_eval_dn(const void *Bp, const double *x, TO *out, long long npts, const int *n,
                                 hipStream_t s)
{
    constexpr int NC32 = 32, NC16 = 16;
    constexpr int RB = 4;
    const int rows_b = 4 * RB * 16;
    const unsigned blocks = (unsigned)((npts + rows_b - 1) / rows_b);
    const int n0 = D >= 3 ? n[0] : 1, n1 = D >= 4 ? n[1] : 1;
    if (n[D - 1] <= 16)
        hipLaunchKernelGGL((k_eval_mfma<TE, TO, D, N4, NC16, RB>), dim3(blocks), dim3(256), 0, s,
                           (const TE *)Bp, x, out, npts, n0, n1, n[D - 1]);
    else
        hipLaunchKernelGGL((k_eval_mfma<TE, TO, D, N4, NC32, RB>), dim3(blocks), dim3(256), 0, s,
                           (const TE *)Bp, x, out, npts, n0, n1, n[D - 1]);
    return hipGetLastError();
}

template <int D, int N4>
static hipError_t launch_eval_bf16_dn(const void *Bp, const double *x, float *out, long long npts, const int *n,
                                      long long Kpad, hipStream_t s)
{
    constexpr int RB = 2;
    const int rows_b = 4 * RB * 16;
    const unsigned blocks = (unsigned)((npts + rows_b - 1) / rows_b);
    const int n0 = D >= 3 ? n[0] : 1, n1 = D >= 4 ? n[1] : 1;
    if (n[D - 1] <= 16)
        hipLaunchKernelGGL((k_eval_bf16<D, N4, 16, RB>), dim3(blocks), dim3(256), 0, s, (const __bf16 *)Bp, x, out,
                           npts, n0, n1, n[D - 1], Kpad);
    else
        hipLaunchKernelGGL((k_eval_bf16<D, N4, 32, RB>), dim3(blocks), dim3(256), 0, s, (const __bf16 *)Bp, x, out,
                           npts, n0, n1, n[D - 1], Kpad);
    return hipGetLastError();
}

#define CG_N4_SWITCH(N4v, CALL)                  \
    switch (N4v) {                               \
        case 4: { constexpr int N4c = 4; CALL; }   \
        case 8: { constexpr int N4c = 8; CALL; }   \
        case 12: { constexpr int N4c = 12; CALL; } \
        case 16: { constexpr int N4c = 16; CALL; } \
        case 20: { constexpr int N4c = 20; CALL; } \
        case 24: { constexpr int N4c = 24; CALL; } \
        case 28: { constexpr int N4c = 28; CALL; } \
        case 32: { constexpr int N4c = 32; CALL; } \
    }

template <int D>
static hipError_t launch_eval_d(const void *Bp, const double *x, void *out, long long npts, const int *n,
                                int precision, long long Kpad, hipStream_t s)
{
    const int N4 = round4(n[D - 2]);
    if (precision == CG_FP64) {
        CG_N4_SWITCH(N4, return (launch_eval_dn<double, double, D, N4c>(Bp, x, (double *)out, npts, n, s)))
    } else if (precision == CG_FP32) {
        CG_N4_SWITCH(N4, return (launch_eval_dn<float, float, D, N4c>(Bp, x, (float *)out, npts, n, s)))
    } else {
        CG_N4_SWITCH(N4, return (launch_eval_bf16_dn<D, N4c>(Bp, x, (float *)out, npts, n, Kpad, s)))
    }
    return hipErrorInvalidValue;
}

hipError_t launch_eval(int d, const int *n, const double *coef, const double *x, long long npts, void *out,
                       int precision, void *ws, size_t ws_bytes, hipStream_t s)
{
    if (npts == 0) return hipSuccess;
    if (d == 1) {
        const unsigned blocks = (unsigned)((npts + 255) / 256);
        if (precision == CG_FP64)
            hipLaunchKernelGGL(k_eval_1d<double>, dim3(blocks), dim3(256), 0, s, coef, x, (double *)out, npts, n[0],
                               precision);
        else
            hipLaunchKernelGGL(k_eval_1d<float>, dim3(blocks), dim3(256), 0, s, coef, x, (float *)out, npts, n[0],
                               precision);
        return hipGetLastError();
    }
    const int N4 = round4(n[d - 2]);
    const int NC = n[d - 1] <= 16 ? 16 : 32;
    long long K = eval_K(d, n, N4);
    long long Kpad = precision == CG_BF16 ? (K + 31) / 32 * 32 : K;
    if (ws_bytes < eval_ws_bytes(d, n, precision)) return hipErrorInvalidValue;
    const int nn[4] = {n[0], d > 1 ? n[1] : 1, d > 2 ? n[2] : 1, d > 3 ? n[3] : 1};
    const unsigned pb = (unsigned)((Kpad * NC + 255) / 256);
    if (precision == CG_FP64)
        hipLaunchKernelGGL(k_pack_eval<double>, dim3(pb), dim3(256), 0, s, coef, (double *)ws, d, nn[0], nn[1], nn[2],
                           nn[3], N4, NC, K, Kpad);
    else if (precision == CG_FP32)
        hipLaunchKernelGGL(k_pack_eval<float>, dim3(pb), dim3(256), 0, s, coef, (float *)ws, d, nn[0], nn[1], nn[2],
                           nn[3], N4, NC, K, Kpad);
    else
        hipLaunchKernelGGL(k_pack_eval<__bf16>, dim3(pb), dim3(256), 0, s, coef, (__bf16 *)ws, d, nn[0], nn[1],
                           nn[2], nn[3], N4, NC, K, Kpad);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    switch (d) {
        case 2: return launch_eval_d<2>(ws, x, out, npts, n, precision, Kpad, s);
        case 3: return launch_eval_d<3>(ws, x, out, npts, n, precision, Kpad, s);
        case 4: return launch_eval_d<4>(ws, x, out, npts, n, precision, Kpad, s);
    }
    return hipErrorInvalidValue;
}

}  // namespace cg
