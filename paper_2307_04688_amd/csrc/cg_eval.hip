// cg_eval.hip -- value of an n-dimensional Chebyshev series at arbitrary
// points (the evaluation of Section 3.2 with one point per mode).
//
// For points x_q the modes 0..d-2 are contracted at once as the GEMM
//     W (npts x n_{d-1}) = KR (npts x prod_{l<d-1} n_l) * C (.. x n_{d-1}),
// where row q of KR is the Khatri-Rao product of the basis vectors
// (T_k(x_{q,l}))_k and C is the coefficient tensor with the last mode as
// columns; then f(x_q) = sum_k W[q,k] T_k(x_{q,d-1}) by Clenshaw.  The GEMM
// runs on MFMA: f64 16x16x4 (CG_FP64), f32 16x16x4 (CG_FP32), or bf16
// 16x16x32 with f32 accumulation (CG_BF16; CG_FP32_SPLIT with both operands
// as three exact bf16 pieces of their binary32 values).
#include <type_traits>

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
                                                   long long Kpad, long long coef_stride)
{
    const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= Kpad * NC) return;
    coef += blockIdx.y * coef_stride;  // member y of a batch of tensors of one shape
    Bp += blockIdx.y * Kpad * NC;
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
// Member blockIdx.y of a batch uses packed operand Bp + y bp_stride, points
// X + x_off[y] d and outputs out + x_off[y] (npts[y] of them).
template <typename TE, typename TO, int D, int N4, int NC, int RB>
__global__ __launch_bounds__(256) void k_eval_mfma(const TE *__restrict__ Bp, const double *__restrict__ X,
                                                   TO *__restrict__ out, EvalBatch bt, int n0, int n1,
                                                   int nlast)
{
    const long long npts = bt.npts[blockIdx.y];
    if ((long long)blockIdx.x * (4 * RB * 16) >= npts) return;  // whole block beyond this member
    Bp += blockIdx.y * bt.bp_stride;
    X += bt.x_off[blockIdx.y] * D;
    out += bt.x_off[blockIdx.y];
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

// BF16 evaluation as a two-level contraction on v_mfma_f32_16x16x32_bf16
// (lane r + 16 g supplies A[r][8g..8g+7] and B[8g..8g+7][r]; D[4g+v][r] in
// element v).  The contracted index space is (o, i): o runs over mode 0 when
// d >= 3, i over the other contracted modes (mode 1 when d = 4, then mode d-2
// padded to N4).  The basis products A_q(i) = T(x_q1) T(x_q,d-2) of a chunk of
// 32 KSC inner indices (up to 18 K-steps: the whole inner index space of a
// d = 4, N = 24 series) are rounded to bf16 once and stay in registers for
// every o; the MFMAs give P_q(o, c) = sum_i A_q(i) C[o, i, c] in f32 and
// W_q(c) += T_o(x_q0) P_q(o, c), once per (chunk, o).
//
// A wave holds 32 rows (two 16-row blocks) against every column block, so
// no two waves build the same basis products, and each coefficient fragment
// it reads from LDS feeds two MFMAs.  C streams through LDS in slabs of OG
// outer values x KP K-steps of one chunk (at most 12 fragments of 1 KB; a
// chunk of KSC = 18 steps is three slabs per o), written by direct
// global-to-LDS loads into a ring of three slabs two ahead of the MFMAs,
// with one barrier per slab.  The per-row basis tables live in LDS.
//
// The same kernel gives binary32 accuracy on the bf16 MFMA (CG_FP32_SPLIT,
// three pieces): the basis products and coefficients are rounded to binary32
// and split exactly into three bf16 pieces each (at most two K-steps per
// chunk, one per slab), and every K-step runs the six piece products of
// leading order; the tables stay in binary32.
struct Bf16Geo {
    int n_o, n_b, n_l, n_c;  // outer mode, second inner mode (1 if none), mode d-2, last mode
    int K2, CH;              // inner length n_b * N4, chunks of 32 KSC
    int OG, n_og;            // outer values per slab; outer groups (n_o padded to n_og OG with zeros)
};

// K-steps per slab for a chunk of KSC steps; a chunk is KSC / KP slabs per o.
// The split form (np = 3 pieces) takes one K-step per slab: its ring then
// leaves room for two blocks per CU beside the binary32 tables (measured at
// d = 4, N = 24: 13.9 against 23.8 ms with two steps per slab).
__host__ __device__ constexpr int bf16_kp(int ksc, int np = 1) { return np > 1 ? 1 : (ksc <= 6 ? ksc : 6); }

// Packed C: fragment-contiguous, (((((o CH + ch) KSC + ks) NP + piece) NCB + c) 4 + g) 16 + col,
// 8 bf16 each, for o < n_og OG (zero beyond n_o).  NP = 1: the coefficient
// rounded to bf16; NP = 3 (split form): the coefficient rounded to binary32
// as three bf16 pieces whose sum is that binary32 value exactly.
template <int KSC, int NCB, int NP>
__global__ __launch_bounds__(256) void k_pack_bf16(const double *__restrict__ coef, __bf16 *__restrict__ Bp,
                                                   Bf16Geo gg, int N4)
{
    const long long total = (long long)gg.n_og * gg.OG * gg.CH * KSC * NP * NCB * 512;
    const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= total) return;
    const int ee = (int)(e & 7), col = (int)((e >> 3) & 15), g = (int)((e >> 7) & 3);
    long long r = e >> 9;
    const int c = (int)(r % NCB);
    r /= NCB;
    const int piece = (int)(r % NP);
    r /= NP;
    const int ks = (int)(r % KSC);
    r /= KSC;
    const int ch = (int)(r % gg.CH);
    const int o = (int)(r / gg.CH);
    const int i = (ch * KSC + ks) * 32 + 8 * g + ee;
    const int colf = c * 16 + col;
    double v = 0.0;
    if (i < gg.K2 && o < gg.n_o) {
        const int kb = i / N4, kl = i % N4;
        if (kl < gg.n_l && colf < gg.n_c)
            v = coef[(((long long)o * gg.n_b + kb) * gg.n_l + kl) * gg.n_c + colf];
    }
    float f = (float)v;
    if constexpr (NP > 1) __asm__("" : "+v"(f));  // the pieces split the binary32 value
    __bf16 h = (__bf16)f;
#pragma unroll
    for (int q = 1; q < NP; ++q) {
        if (q > piece) break;
        f -= (float)h;  // exact: what the previous pieces left
        h = (__bf16)f;
    }
    Bp[e] = h;
}

// s_waitcnt vmcnt(N) lgkmcnt(0), no wait on expcnt (gfx9 encoding:
// vmcnt[3:0], expcnt[6:4], lgkmcnt[11:8]).
template <int N>
__device__ __forceinline__ void wait_vmcnt()
{
    static_assert(N >= 0 && N < 16, "vmcnt field");
    __builtin_amdgcn_s_waitcnt(0x0070 | N);
}

template <int D, int N4, int NC, int KSC, int NP>
__global__ __launch_bounds__(256) void k_eval_bf16(const __bf16 *__restrict__ Bp, const double *__restrict__ X,
                                                   float *__restrict__ out, long long npts, Bf16Geo gg)
{
    // NP = 1: bf16 operands; NP = 3 (split form): both operands rounded to
    // binary32 and split exactly into three bf16 pieces, and the six piece
    // products of leading order (the three dropped ones are below 2^-24 of
    // the product) summed in binary32
    static_assert(NP == 1 || NP == 3, "one or three pieces");
    constexpr int NPP = NP == 3 ? 6 : 1;          // piece products per K-step
    constexpr int PD = NP == 1 ? 2 : 1;           // fragment reads run PD K-steps ahead
    constexpr int NCB = NC / 16;
    constexpr int RB = 2;                         // 16-row blocks per wave
    constexpr int ROWS_W = RB * 16;
    constexpr int ROWS_B = 4 * ROWS_W;            // 128 points per block of four waves
    constexpr int KP = bf16_kp(KSC, NP);          // K-steps per slab
    constexpr int NPART = KSC / KP;               // slabs per (chunk, o)
    static_assert(NPART * KP == KSC, "a chunk is whole slabs");
    constexpr int LDT = N4;                       // mode-l table stride (floats; 16-byte rows)
    constexpr int LDB = 33;                       // mode-1 table: n_b <= 32 values, zero up to index 32
    constexpr int MAXO = 32;                      // outer values incl. padding (bf16_geo keeps n_og OG <= 32)
    constexpr int FRAG = 512;                     // bf16 per fragment (64 lanes x 16 bytes)
    constexpr int NBUF = 3;
    constexpr int LDW = NC + 1;
    const int FR = (NPART > 1 ? 1 : gg.OG) * KP * NP * NCB;  // fragments per slab (OG = 1 when NPART > 1)
    const int n_op = gg.n_og * gg.OG;             // outer values incl. padding
    // The tables are arrays of their own, apart from the ring that the
    // direct loads write, so that reading them waits for no load in flight.
    // The mode-1 factor is stored in binary16 (|T| <= 1; rounding 2^-12,
    // far below the bf16 rounding of the product it enters).
    __shared__ __attribute__((aligned(16))) float Tl[ROWS_B * LDT];
    // (binary32 in the split form, whose products keep binary32 accuracy)
    using TbT = typename std::conditional<NP == 1, _Float16, float>::type;
    __shared__ TbT Tb[D == 4 ? ROWS_B * LDB : 1];
    __shared__ __attribute__((aligned(16))) float To[MAXO * ROWS_B];  // T_o(x_q0) as [o][row]
    extern __shared__ __attribute__((aligned(16))) __bf16 Bs[];        // NBUF slabs of FR fragments
    const int SLAB = FR * FRAG;

    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);  // scalar: slab addressing stays on the SALU
    const int r16 = lane & 15, g = lane >> 4;
    const long long q0 = (long long)blockIdx.x * ROWS_B;

    // ---- per-row basis tables by the three-term recurrence in binary32
    // (stable on [-1,1]: error ~ k 2^-24, far below the bf16 rounding of the
    // products); threads r < 128 build mode l and the outer mode of row r,
    // threads 128 + r mode 1 ----
    {
        const int r = tid & (ROWS_B - 1);
        long long q = q0 + r;
        q = q < npts ? q : npts - 1;
        const double *xq = X + q * D;
        if (tid < ROWS_B) {
            const float xl = (float)xq[D - 2];
            float tm = 1.0f, tc = xl;
            Tl[r * LDT] = 1.0f;
#pragma unroll 4
            for (int k = 1; k < N4; ++k) {
                Tl[r * LDT + k] = tc;
                const float tn = fmaf(2.0f * xl, tc, -tm);
                tm = tc;
                tc = tn;
            }
            const float xo = D >= 3 ? (float)xq[0] : 0.0f;  // d < 3: one outer value, T_0 = 1
            tm = 1.0f;
            tc = xo;
            To[r] = 1.0f;
            for (int o = 1; o < n_op; ++o) {
                To[o * ROWS_B + r] = tc;
                const float tn = fmaf(2.0f * xo, tc, -tm);
                tm = tc;
                tc = tn;
            }
        } else if (D == 4 && tid < 2 * ROWS_B) {
            const float xb = (float)xq[1];
            float tm = 1.0f, tc = xb;
            Tb[r * LDB] = (TbT)1.0f;
#pragma unroll 4
            for (int k = 1; k < LDB; ++k) {
                Tb[r * LDB + k] = (TbT)(k < gg.n_b ? tc : 0.0f);
                const float tn = fmaf(2.0f * xb, tc, -tm);
                tm = tc;
                tc = tn;
            }
        }
    }
    __syncthreads();  // tables visible; no loads in flight past this point

    // slab s = ((chunk ch, outer group og), part p), p fastest; wave w loads
    // fragments w, w + 4, ... of it, each one wave-wide 1 KB transfer (the
    // packed operand holds fewer than 2^22 fragments: 32-bit indices).  The
    // next slab to load is kept as counters (no division in the loop).
    const int nslab = gg.CH * gg.n_og * NPART;
    const __bf16 *Bl = Bp + lane * 8;
    int i_ch = 0, i_og = 0, i_p = 0, i_buf = 0;
    auto issue_next = [&]() {
        __bf16 *dst = Bs + i_buf * SLAB;
        const int base = (((i_og * gg.OG) * gg.CH + i_ch) * KSC + i_p * KP) * NP * NCB;
        if (NPART > 1) {  // FR = KP NP NCB fragments, known here: unrolled
#pragma unroll
            for (int j = 0; j < (KP * NP * NCB + 3) / 4; ++j) {
                const int f = wave + 4 * j;
                if (f < KP * NP * NCB)
                    __builtin_amdgcn_global_load_lds(
                        Bl + (base + f) * FRAG, (__attribute__((address_space(3))) void *)(dst + f * FRAG), 16, 0, 0);
            }
        } else {
            for (int f = wave; f < FR; f += 4) {
                const int oo = f / (KP * NP * NCB), rest = f - oo * (KP * NP * NCB);
                const int src = base + oo * gg.CH * KSC * NP * NCB + rest;
                __builtin_amdgcn_global_load_lds(
                    Bl + src * FRAG, (__attribute__((address_space(3))) void *)(dst + f * FRAG), 16, 0, 0);
            }
        }
        i_buf = i_buf == NBUF - 1 ? 0 : i_buf + 1;
        if (++i_p == NPART) {
            i_p = 0;
            if (++i_og == gg.n_og) {
                i_og = 0;
                ++i_ch;
            }
        }
    };

    f32x4 W[RB][NCB], P[RB][NCB];
#pragma unroll
    for (int rb = 0; rb < RB; ++rb)
#pragma unroll
        for (int c = 0; c < NCB; ++c) W[rb][c] = f32x4{0.f, 0.f, 0.f, 0.f};
    bf16x8 a[RB][KSC][NP];

    issue_next();
    if (nslab > 1) issue_next();
    const int fw = FR / 4;  // loads every wave issues per slab (some issue one more)
    int c_buf = 0;          // ring buffer of the slab being computed
    for (int ch = 0; ch < gg.CH; ++ch) {
        // basis products A_q(i) of this chunk, rounded to bf16 once; past
        // the inner length the mode-1 factor is zero (table entry, or
        // kb > 0 when there is no mode 1), so the reads need no branch
#pragma unroll
        for (int rb = 0; rb < RB; ++rb) {
            const int r = wave * ROWS_W + rb * 16 + r16;
#pragma unroll
            for (int ks = 0; ks < KSC; ++ks)
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    const int i0 = (ch * KSC + ks) * 32 + 8 * g + 4 * h;
                    const int kb = i0 / N4, kl0 = i0 - kb * N4;
                    const float4 t = *reinterpret_cast<const float4 *>(Tl + r * LDT + kl0);
                    const float tb =
                        D == 4 ? (float)Tb[r * LDB + (kb < LDB - 1 ? kb : LDB - 1)] : (kb == 0 ? 1.0f : 0.0f);
                    float pr[4] = {tb * t.x, tb * t.y, tb * t.z, tb * t.w};
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        float f = pr[u];
                        if constexpr (NP > 1) __asm__("" : "+v"(f));  // the split starts from the binary32 product
#pragma unroll
                        for (int q = 0; q < NP; ++q) {
                            const __bf16 hq = (__bf16)f;
                            a[rb][ks][q][4 * h + u] = hq;
                            f -= (float)hq;
                        }
                    }
                }
        }
        for (int og = 0; og < gg.n_og; ++og) {
#pragma unroll
            for (int p = 0; p < NPART; ++p) {
                const int s = (ch * gg.n_og + og) * NPART + p;
                // slab s complete for this wave (slab s + 1 may stay in
                // flight), then for every wave; the barrier also retires the
                // reads of slab s - 1, whose buffer the loads of slab s + 2 reuse
                if (s + 1 < nslab) {
                    switch (fw) {
                        case 0: wait_vmcnt<0>(); break;
                        case 1: wait_vmcnt<1>(); break;
                        case 2: wait_vmcnt<2>(); break;
                        default: wait_vmcnt<3>(); break;
                    }
                } else {
                    wait_vmcnt<0>();
                }
                __builtin_amdgcn_s_barrier();
                asm volatile("" ::: "memory");
                if (s + 2 < nslab) issue_next();

                const __bf16 *sb = Bs + c_buf * SLAB + lane * 8;
                c_buf = c_buf == NBUF - 1 ? 0 : c_buf + 1;
                for (int oo = 0; oo < gg.OG; ++oo) {
                    // fragment reads run PD K-steps ahead of the MFMAs that
                    // use them (an LDS read outlasts one K-step's MFMAs)
                    const __bf16 *so = sb + oo * KP * NP * NCB * FRAG;
                    bf16x8 b[PD + 1][NP][NCB];
#pragma unroll
                    for (int kk = 0; kk < PD && kk < KP; ++kk)
#pragma unroll
                        for (int q = 0; q < NP; ++q)
#pragma unroll
                            for (int c = 0; c < NCB; ++c)
                                b[kk][q][c] = *reinterpret_cast<const bf16x8 *>(so + ((kk * NP + q) * NCB + c) * FRAG);
#pragma unroll
                    for (int kk = 0; kk < KP; ++kk) {
                        if (kk + PD < KP) {
#pragma unroll
                            for (int q = 0; q < NP; ++q)
#pragma unroll
                                for (int c = 0; c < NCB; ++c)
                                    b[(kk + PD) % (PD + 1)][q][c] = *reinterpret_cast<const bf16x8 *>(
                                        so + (((kk + PD) * NP + q) * NCB + c) * FRAG);
                        }
                        // piece products (A piece, B piece), smallest first
                        constexpr int PA[6] = {2, 1, 0, 1, 0, 0}, PB[6] = {0, 1, 2, 0, 1, 0};
#pragma unroll
                        for (int pp = 0; pp < NPP; ++pp)
#pragma unroll
                            for (int c = 0; c < NCB; ++c)
#pragma unroll
                                for (int rb = 0; rb < RB; ++rb)  // each o starts from zero
                                    P[rb][c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                                        a[rb][p * KP + kk][NP == 1 ? 0 : PA[pp]],
                                        b[kk % (PD + 1)][NP == 1 ? 0 : PB[pp]][c],
                                        (p == 0 && kk == 0 && pp == 0) ? f32x4{0.f, 0.f, 0.f, 0.f} : P[rb][c], 0,
                                        0, 0);
                    }
                    // keep that order through scheduling (left alone, the
                    // scheduler sinks every read next to its MFMAs to save
                    // registers): the first PD steps' reads, then per step
                    // the reads PD ahead and the step's MFMAs
                    __builtin_amdgcn_sched_group_barrier(0x100, (KP < PD ? KP : PD) * NP * NCB, 0);
#pragma unroll
                    for (int kk = 0; kk < KP; ++kk) {
                        if (kk + PD < KP) __builtin_amdgcn_sched_group_barrier(0x100, NP * NCB, 0);
                        __builtin_amdgcn_sched_group_barrier(0x008, NPP * NCB * RB, 0);
                    }
                    if (p == NPART - 1) {  // W += T_o(x_q0) P at the accumulator rows 4g + v
                        const float *to = To + (og * gg.OG + oo) * ROWS_B + wave * ROWS_W + 4 * g;
#pragma unroll
                        for (int rb = 0; rb < RB; ++rb) {
                            const float4 t = *reinterpret_cast<const float4 *>(to + rb * 16);
#pragma unroll
                            for (int c = 0; c < NCB; ++c) {
                                W[rb][c][0] = fmaf(t.x, P[rb][c][0], W[rb][c][0]);
                                W[rb][c][1] = fmaf(t.y, P[rb][c][1], W[rb][c][1]);
                                W[rb][c][2] = fmaf(t.z, P[rb][c][2], W[rb][c][2]);
                                W[rb][c][3] = fmaf(t.w, P[rb][c][3], W[rb][c][3]);
                            }
                        }
                    }
                }
            }
        }
    }
    __syncthreads();  // every wave is done with the ring, which now holds W

    // ---- W rows to LDS, Clenshaw along the last mode ----
    float *Wl = reinterpret_cast<float *>(Bs);
#pragma unroll
    for (int rb = 0; rb < RB; ++rb)
#pragma unroll
        for (int c = 0; c < NCB; ++c)
#pragma unroll
            for (int v = 0; v < 4; ++v)
                Wl[(wave * ROWS_W + rb * 16 + 4 * g + v) * LDW + c * 16 + r16] = W[rb][c][v];
    __syncthreads();
    if (tid < ROWS_B) {
        const long long q = q0 + tid;
        if (q < npts) {
            double w[NC];
#pragma unroll
            for (int k = 0; k < NC; ++k) w[k] = (double)Wl[tid * LDW + k];
            out[q] = (float)clenshaw(w, X[q * D + D - 1]);  // columns >= n_c are zero
        }
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

// Geometry of the BF16 operand (np pieces per coefficient): outer mode,
// inner modes, chunking, slabs.
static Bf16Geo bf16_geo(int d, const int *n, int &ksc, int np)
{
    Bf16Geo gg;
    const int N4 = round4(n[d - 2]);
    gg.n_o = d >= 3 ? n[0] : 1;
    gg.n_b = d == 4 ? n[1] : 1;
    gg.n_l = n[d - 2];
    gg.n_c = n[d - 1];
    gg.K2 = gg.n_b * N4;
    const int steps = (gg.K2 + 31) / 32;
    // K-steps held in registers per chunk: fewest padded steps, counting two
    // steps of overhead (a W update) per chunk and outer value
    // (the split form holds three pieces of each basis product: at most two
    // K-steps in registers)
    const int cand[4] = {18, 6, 2, 1};
    int best = 1 << 30;
    ksc = 1;
    for (int c : cand) {
        if (np > 1 && c > 2) continue;
        const int ch = (steps + c - 1) / c;
        const int cost = ch * (c + 2);
        if (cost < best) {
            best = cost;
            ksc = c;
        }
    }
    gg.CH = (steps + ksc - 1) / ksc;
    // outer values per slab when a chunk is one slab per o: at most 12
    // fragments (three slabs and the tables leave room for two blocks per
    // CU), at most 32 outer values with the padding (the kernel's T_o
    // table), fewest padded fragments counting four of overhead (a barrier)
    // per slab
    const int kp = bf16_kp(ksc, np), f0 = kp * np * (n[d - 1] <= 16 ? 1 : 2);
    gg.OG = 1;
    if (kp == ksc) {
        best = 1 << 30;
        for (int og = 1; og * f0 <= 12; ++og) {
            if ((gg.n_o + og - 1) / og * og > 32) continue;
            const int cost = (gg.n_o + og - 1) / og * (og * f0 + 4);
            if (cost < best) {
                best = cost;
                gg.OG = og;
            }
        }
    }
    gg.n_og = (gg.n_o + gg.OG - 1) / gg.OG;
    return gg;
}

size_t eval_ws_bytes(int d, const int *n, int precision)
{
    if (d < 2) return 0;
    const int N4 = round4(n[d - 2]);
    const int NC = n[d - 1] <= 16 ? 16 : 32;
    if (precision == CG_BF16 || precision == CG_FP32_SPLIT) {
        const int np = precision == CG_BF16 ? 1 : 3;
        int ksc;
        const Bf16Geo gg = bf16_geo(d, n, ksc, np);
        return (size_t)gg.n_og * gg.OG * gg.CH * ksc * np * (NC / 16) * 512 * 2 + 256;
    }
    const long long K = eval_K(d, n, N4);
    const size_t es = precision == CG_FP64 ? 8 : 4;
    return (size_t)(K * NC) * es + 256;
}

// Row blocks of 16 points per wave: 2 for FP64 (measured: d = 4, N = 24 at
// 2^22 points 0.60 of the FP64 peak against 0.54 with 4; the d = 3 update
// points of the general form 0.76 against 0.67), 4 for FP32 (0.55 against
// 0.53).
template <typename TE, typename TO, int D, int N4>
static hipError_t launch_eval_dn(const void *Bp, const double *x, TO *out, const EvalBatch &bt, int count,
                                 const int *n, hipStream_t s)
{
    constexpr int NC32 = 32, NC16 = 16;
    constexpr int RB = sizeof(TE) == 8 ? 2 : 4;
    const int rows_b = 4 * RB * 16;
    long long mx = 0;
    for (int b = 0; b < count; ++b) mx = bt.npts[b] > mx ? bt.npts[b] : mx;
    if (mx == 0) return hipSuccess;
    const unsigned blocks = (unsigned)((mx + rows_b - 1) / rows_b);
    const int n0 = D >= 3 ? n[0] : 1, n1 = D >= 4 ? n[1] : 1;
    if (n[D - 1] <= 16)
        hipLaunchKernelGGL((k_eval_mfma<TE, TO, D, N4, NC16, RB>), dim3(blocks, (unsigned)count), dim3(256), 0, s,
                           (const TE *)Bp, x, out, bt, n0, n1, n[D - 1]);
    else
        hipLaunchKernelGGL((k_eval_mfma<TE, TO, D, N4, NC32, RB>), dim3(blocks, (unsigned)count), dim3(256), 0, s,
                           (const TE *)Bp, x, out, bt, n0, n1, n[D - 1]);
    return hipGetLastError();
}

template <int D, int N4, int NC, int KSC, int NP>
static hipError_t launch_bf16_k(const double *coef, void *ws, const double *x, float *out, long long npts,
                                const Bf16Geo &gg, hipStream_t s)
{
    constexpr int ROWS_B = 128;
    const long long total = (long long)gg.n_og * gg.OG * gg.CH * KSC * NP * (NC / 16) * 512;
    hipLaunchKernelGGL((k_pack_bf16<KSC, NC / 16, NP>), dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s,
                       coef, (__bf16 *)ws, gg, N4);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    // dynamic LDS: the ring of three slabs, which also stages the W rows
    const size_t ring = (size_t)3 * gg.OG * bf16_kp(KSC, NP) * NP * (NC / 16) * 1024;
    const size_t stage = (size_t)ROWS_B * (NC + 1) * sizeof(float);
    const size_t shm = ring > stage ? ring : stage;
    const unsigned blocks = (unsigned)((npts + ROWS_B - 1) / ROWS_B);
    if (shm > 48 * 1024) {
        e = hipFuncSetAttribute((const void *)k_eval_bf16<D, N4, NC, KSC, NP>,
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL((k_eval_bf16<D, N4, NC, KSC, NP>), dim3(blocks), dim3(256), shm, s, (const __bf16 *)ws, x,
                       out, npts, gg);
    return hipGetLastError();
}

template <int D, int N4, int NP>
static hipError_t launch_eval_bf16_dnp(const double *coef, void *ws, const double *x, float *out, long long npts,
                                       const int *n, hipStream_t s)
{
    int ksc;
    const Bf16Geo gg = bf16_geo(D, n, ksc, NP);
    if constexpr (D < 4) {  // one K-step in all (bf16_geo)
        if (n[D - 1] <= 16) return launch_bf16_k<D, N4, 16, 1, NP>(coef, ws, x, out, npts, gg, s);
        return launch_bf16_k<D, N4, 32, 1, NP>(coef, ws, x, out, npts, gg, s);
    } else if constexpr (NP > 1) {  // at most two K-steps per chunk (bf16_geo)
        if (n[D - 1] <= 16)
            return ksc == 2 ? launch_bf16_k<D, N4, 16, 2, NP>(coef, ws, x, out, npts, gg, s)
                            : launch_bf16_k<D, N4, 16, 1, NP>(coef, ws, x, out, npts, gg, s);
        return ksc == 2 ? launch_bf16_k<D, N4, 32, 2, NP>(coef, ws, x, out, npts, gg, s)
                        : launch_bf16_k<D, N4, 32, 1, NP>(coef, ws, x, out, npts, gg, s);
    } else {
        if (n[D - 1] <= 16) {
            switch (ksc) {
                case 18: return launch_bf16_k<D, N4, 16, 18, NP>(coef, ws, x, out, npts, gg, s);
                case 6: return launch_bf16_k<D, N4, 16, 6, NP>(coef, ws, x, out, npts, gg, s);
                case 2: return launch_bf16_k<D, N4, 16, 2, NP>(coef, ws, x, out, npts, gg, s);
                default: return launch_bf16_k<D, N4, 16, 1, NP>(coef, ws, x, out, npts, gg, s);
            }
        }
        switch (ksc) {
            case 18: return launch_bf16_k<D, N4, 32, 18, NP>(coef, ws, x, out, npts, gg, s);
            case 6: return launch_bf16_k<D, N4, 32, 6, NP>(coef, ws, x, out, npts, gg, s);
            case 2: return launch_bf16_k<D, N4, 32, 2, NP>(coef, ws, x, out, npts, gg, s);
            default: return launch_bf16_k<D, N4, 32, 1, NP>(coef, ws, x, out, npts, gg, s);
        }
    }
}

template <int D, int N4>
static hipError_t launch_eval_bf16_dn(const double *coef, void *ws, const double *x, float *out, long long npts,
                                      const int *n, int np, hipStream_t s)
{
    return np == 1 ? launch_eval_bf16_dnp<D, N4, 1>(coef, ws, x, out, npts, n, s)
                   : launch_eval_bf16_dnp<D, N4, 3>(coef, ws, x, out, npts, n, s);
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
static hipError_t launch_eval_d(const void *Bp, const double *x, void *out, const EvalBatch &bt, int count,
                                const int *n, int precision, hipStream_t s)
{
    const int N4 = round4(n[D - 2]);
    if (precision == CG_FP64) {
        CG_N4_SWITCH(N4, return (launch_eval_dn<double, double, D, N4c>(Bp, x, (double *)out, bt, count, n, s)))
    } else {
        CG_N4_SWITCH(N4, return (launch_eval_dn<float, float, D, N4c>(Bp, x, (float *)out, bt, count, n, s)))
    }
    return hipErrorInvalidValue;
}

template <int D>
static hipError_t launch_eval_bf16_d(const double *coef, void *ws, const double *x, void *out, long long npts,
                                     const int *n, int np, hipStream_t s)
{
    const int N4 = round4(n[D - 2]);
    CG_N4_SWITCH(N4, return (launch_eval_bf16_dn<D, N4c>(coef, ws, x, (float *)out, npts, n, np, s)))
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
    if (ws_bytes < eval_ws_bytes(d, n, precision)) return hipErrorInvalidValue;
    if (precision == CG_BF16 || precision == CG_FP32_SPLIT) {
        const int np = precision == CG_BF16 ? 1 : 3;
        switch (d) {
            case 2: return launch_eval_bf16_d<2>(coef, ws, x, out, npts, n, np, s);
            case 3: return launch_eval_bf16_d<3>(coef, ws, x, out, npts, n, np, s);
            case 4: return launch_eval_bf16_d<4>(coef, ws, x, out, npts, n, np, s);
        }
        return hipErrorInvalidValue;
    }
    const int N4 = round4(n[d - 2]);
    const int NC = n[d - 1] <= 16 ? 16 : 32;
    const long long K = eval_K(d, n, N4);
    const int nn[4] = {n[0], d > 1 ? n[1] : 1, d > 2 ? n[2] : 1, d > 3 ? n[3] : 1};
    const unsigned pb = (unsigned)((K * NC + 255) / 256);
    if (precision == CG_FP64)
        hipLaunchKernelGGL(k_pack_eval<double>, dim3(pb), dim3(256), 0, s, coef, (double *)ws, d, nn[0], nn[1], nn[2],
                           nn[3], N4, NC, K, K, 0LL);
    else
        hipLaunchKernelGGL(k_pack_eval<float>, dim3(pb), dim3(256), 0, s, coef, (float *)ws, d, nn[0], nn[1], nn[2],
                           nn[3], N4, NC, K, K, 0LL);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    EvalBatch bt = {};
    bt.npts[0] = npts;
    switch (d) {
        case 2: return launch_eval_d<2>(ws, x, out, bt, 1, n, precision, s);
        case 3: return launch_eval_d<3>(ws, x, out, bt, 1, n, precision, s);
        case 4: return launch_eval_d<4>(ws, x, out, bt, 1, n, precision, s);
    }
    return hipErrorInvalidValue;
}

size_t eval_packed_elems(int d, const int *n)
{
    const int N4 = round4(n[d - 2]);
    const int NC = n[d - 1] <= 16 ? 16 : 32;
    return (size_t)(eval_K(d, n, N4) * NC);
}

hipError_t pack_eval_f64(int d, const int *n, const double *coef, long long count, long long coef_stride,
                         double *Bp, hipStream_t s)
{
    if (d < 2 || count <= 0) return d < 2 ? hipErrorInvalidValue : hipSuccess;
    const int N4 = round4(n[d - 2]);
    const int NC = n[d - 1] <= 16 ? 16 : 32;
    const long long K = eval_K(d, n, N4);
    const int nn[4] = {n[0], n[1], d > 2 ? n[2] : 1, d > 3 ? n[3] : 1};
    const unsigned pb = (unsigned)((K * NC + 255) / 256);
    hipLaunchKernelGGL(k_pack_eval<double>, dim3(pb, (unsigned)count), dim3(256), 0, s, coef, Bp, d, nn[0], nn[1],
                       nn[2], nn[3], N4, NC, K, K, coef_stride);
    return hipGetLastError();
}

hipError_t eval_f64_batch(int d, const int *n, const double *Bp, const double *x, double *out, const EvalBatch &bt,
                          int count, hipStream_t s)
{
    if (count < 1 || count > kMaxD) return hipErrorInvalidValue;
    switch (d) {
        case 2: return launch_eval_d<2>(Bp, x, out, bt, count, n, CG_FP64, s);
        case 3: return launch_eval_d<3>(Bp, x, out, bt, count, n, CG_FP64, s);
        case 4: return launch_eval_d<4>(Bp, x, out, bt, count, n, CG_FP64, s);
    }
    return hipErrorInvalidValue;
}

}  // namespace cg
