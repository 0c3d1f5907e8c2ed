// cg_mixed.hip -- contraction of the value-iteration step at binary32
// accuracy on MFMA (binary32 MFMA, or for d = 3 from N4 = 20 on bf16 MFMA on
// exactly split binary32 operands) with an FP64 correction (precision
// CG_FP32_CORR).
//
// For player i and node j with other-mode coordinates x_l = xbar_l + Delta_l
// (xbar_l the node, Delta_l = 2 h b_l / p_max the Euler shift), the line
// coefficients w[j][k_i] = sum_K KR_K(x) c_i[K] split exactly into
//   w = E0 + sum_l Delta_l E1_l + R,
//   E0  = sum_K KR_K(xbar) c_i[K]          (V_i transformed along mode i only),
//   E1_l = sum_K d/dx_l KR_K(xbar) c_i[K]  (the same, differentiated along l),
//   R   = sum_K A2_K c_i[K],  A2 = KR(x) - KR(xbar) - sum_l Delta_l d/dx_l KR(xbar).
// E0 and E1 are small FP64 mode products of V (no point evaluation), computed
// once per iteration; only the second-order remainder R, of relative size
// ~Delta^2, runs at binary32 accuracy (inputs rounded to binary32, products
// accumulated in binary32, then added into FP64).
//
// Two kernels contract R.  d = 3 (k_contract_corr3): the remainder splits
// into one product per K element plus two one-mode contractions against
// nodal tensors, the products in split bfloat16 form from N4 = 20 on (see
// the kernel).  d = 2, 4 (k_contract_corr): A2 is
// built per K element from per-mode quantities: with T = T_k(x),
// Tb = T_k(xbar), P = T_k'(xbar) Delta (first-order increment) and
// R1 = T - Tb - P, a product over a mode set S extends by a mode c as
//   Rem_{S+c} = Rem_S T_c + Lin_S R1_c + FO_S P_c,
//   FO_{S+c}  = FO_S Tb_c + Pb_S P_c,   Pb_{S+c} = Pb_S Tb_c,
//   Lin_S = Pb_S + FO_S,
// where Pb_S is the product of Tb and FO_S its first-order part, so each
// K element costs three multiply-adds once the outer modes are combined.
#include "cg_line.h"
#include "cg_tf.h"

namespace cg {

// E[i][slot][jm][col] (jm enumerates the modes other than i in increasing
// order, col = k_i): slot 0 = G_i = V_i transformed (DCT-I) along mode i only,
// at the nodes of the other modes; slot 1 + s = G_i differentiated at the
// nodes along om_s, the s-th mode other than i.  One block per plane (mode
// l = om_s by mode i, the remaining modes fixed): the plane of V_i goes to
// LDS, G = V Dx^T along mode i, then Dd G along l; the s = 0 planes also
// write slot 0.
template <int NP>
__device__ __forceinline__ void taylor_block(const Inst *__restrict__ tab, int bpi, int bid, double *sm)
{
    const InstView I = inst_view(tab, bid / bpi);
    const int blk = bid % bpi;
    const GameConst *__restrict__ gc = I.gc;
    const GameStatus *st = I.st;
    double *E = I.E;
    constexpr int LD = kMaxN + 1;
    double *Dx = sm, *Dd = sm + kMaxN * LD, *X = sm + 2 * kMaxN * LD, *Gp = sm + 3 * kMaxN * LD;
    if (st->converged) return;
    const int N = gc->N, d = gc->d, NC = gc->NC;
    const long long NN = gc->NN;
    const int NM = (int)(NN / N);
    int nf = 1;
    for (int q = 0; q < d - 2; ++q) nf *= N;
    const int i = blk / ((d - 1) * nf);
    const int s = (blk / nf) % (d - 1);
    const int f = blk % nf;
    int om[kMaxD];
    for (int t = 0; t < d - 1; ++t) om[t] = t < i ? t : t + 1;
    const int l = om[s];
    // digits of the fixed modes (the other modes except l, increasing order) from f
    int dig[kMaxD];
    {
        int rem = f;
        for (int t = d - 2; t >= 0; --t) {
            if (t == s) continue;
            dig[om[t]] = rem % N;
            rem /= N;
        }
    }
    long long stride[kMaxD];
    stride[d - 1] = 1;
    for (int q = d - 2; q >= 0; --q) stride[q] = stride[q + 1] * N;
    long long base = 0;
    for (int q = 0; q < d; ++q)
        if (q != i && q != l) base += dig[q] * stride[q];
    const double *Vi = I.V + (long long)st->cur * d * NN + (long long)i * NN;
    for (int e = threadIdx.x; e < NP * NP; e += blockDim.x) {  // zero beyond N
        const int r = e / NP, c = e % NP;  // r: node along l, c: node along i
        const bool in = r < N && c < N;
        Dx[r * LD + c] = in ? gc->Dx[r * kMaxN + c] : 0.0;
        Dd[r * LD + c] = in ? gc->Dd[r * kMaxN + c] : 0.0;
        X[r * LD + c] = in ? Vi[base + r * stride[l] + c * stride[i]] : 0.0;
    }
    __syncthreads();
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int r16 = lane & 15, kq = lane >> 4;
    f64x4 acc;
    int ti, tj;
    // G[r][ki] = sum_j X[r][j] Dx[ki][j]
    if (plane_mfma<NP, LD, false, true>(X, Dx, wave, lane, acc, ti, tj)) {
#pragma unroll
        for (int v = 0; v < 4; ++v) Gp[(ti * 16 + kq + 4 * v) * LD + tj * 16 + r16] = acc[v];
    }
    __syncthreads();
    // E_l[r][ki] = sum_k Dd[r][k] G[k][ki]
    double *Ei = E + (long long)i * d * NM * NC;
    if (plane_mfma<NP, LD, false, false>(Dd, Gp, wave, lane, acc, ti, tj)) {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int r = ti * 16 + kq + 4 * v, ki = tj * 16 + r16;
            if (r >= N || ki >= N) continue;
            int jm = 0;
            for (int t = 0; t < d - 1; ++t) jm = jm * N + (t == s ? r : dig[om[t]]);
            Ei[((long long)(1 + s) * NM + jm) * NC + ki] = acc[v];
            if (s == 0) Ei[(long long)jm * NC + ki] = Gp[r * LD + ki];
        }
    }
    if (d != 3) return;
    // d = 3: F_l = Dx G, the coefficient tensor with modes l and i transformed
    // and the third mode (digit f) at its nodes, in binary32 for the
    // one-mode remainder terms of k_contract_corr3, one N4 x NC slab per
    // (slot s, digit f) stored in MFMA fragment order: element (r, ki) goes to
    // lane (r mod 4) 16 + (ki mod 16), entry (r / 4) (NC / 16) + ki / 16 of
    // that lane's corr3_chunk floats (r < N4, ki < NC; the padding comes out
    // zero from the zero-padded operands).
    const int CH = corr3_chunk(gc->N4, NC), NCB = NC / 16;
    float *E2 = reinterpret_cast<float *>(E + (long long)d * d * NM * NC) + (long long)i * 2 * N * 64 * CH;
    if (plane_mfma<NP, LD, false, false>(Dx, Gp, wave, lane, acc, ti, tj)) {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int r = ti * 16 + kq + 4 * v, ki = tj * 16 + r16;
            if (r < gc->N4 && ki < NC)
                E2[(((long long)s * N + f) * 64 + (r & 3) * 16 + (ki & 15)) * CH + (r >> 2) * NCB + (ki >> 4)] =
                    (float)acc[v];
        }
    }
}

// The first transform pass and the Taylor tensors in one launch: both read
// only V^{[r]} and each alone fills few CUs (d N slices; d (d-1) N^(d-2)
// planes).  Blocks [0, count bpi_tf) run the transform pass, the rest the
// Taylor planes.
template <int NP>
__global__ __launch_bounds__(256) void k_tf_taylor(const Inst *__restrict__ tab, int bpi_tf, int bpi_ty, int n_tf)
{
    __shared__ double sm[4 * kMaxN * (kMaxN + 1)];
    if ((int)blockIdx.x < n_tf)
        tf_fast_block<NP>(tab, bpi_tf, 1, blockIdx.x, sm);
    else
        taylor_block<NP>(tab, bpi_ty, blockIdx.x - n_tf, sm);
}

hipError_t launch_tf_taylor(const GameConst &hc, const StepBuffers &b, hipStream_t s)
{
    int nf = 1;
    for (int q = 0; q < hc.d - 2; ++q) nf *= hc.N;
    const int bpi_ty = hc.d * (hc.d - 1) * nf;
    const int bpi_tf = (int)(hc.NN / ((long long)hc.N * hc.N)) * hc.d;
    const int n_tf = bpi_tf * b.count;
    const unsigned grid = (unsigned)(n_tf + bpi_ty * b.count);
    if (hc.N <= 16)
        hipLaunchKernelGGL(k_tf_taylor<16>, dim3(grid), dim3(256), 0, s, b.tab, bpi_tf, bpi_ty, n_tf);
    else
        hipLaunchKernelGGL(k_tf_taylor<32>, dim3(grid), dim3(256), 0, s, b.tab, bpi_tf, bpi_ty, n_tf);
    return hipGetLastError();
}

// Per-mode basis quantities at one row: T_k(x), T_k(xbar), T_k'(xbar) by
// three-term recurrences, advanced one k at a time.
struct ModeRec {
    double x, xb, dl;            // shifted coordinate, node, Delta
    double t0, t1, b0, b1, p0, p1;  // T_{k-1}, T_k at x; same at xbar; T'_{k-1}, T'_k at xbar
    __device__ void init(double x_, double xb_)
    {
        x = x_; xb = xb_; dl = x_ - xb_;
        t0 = 0.0; t1 = 1.0; b0 = 0.0; b1 = 1.0; p0 = 0.0; p1 = 0.0;  // k = 0
    }
    // quantities for the current k: T, Tb, P = T' Delta, R1 = T - Tb - P
    __device__ void get(double &T, double &Tb, double &P, double &R1) const
    {
        T = t1; Tb = b1; P = p1 * dl; R1 = (t1 - b1) - P;
    }
    __device__ void advance(int k)  // from k to k + 1
    {
        double tn, bn, pn;
        if (k == 0) { tn = x; bn = xb; pn = 1.0; }
        else {
            tn = 2.0 * x * t1 - t0;
            bn = 2.0 * xb * b1 - b0;
            pn = 2.0 * b1 + 2.0 * xb * p1 - p0;
        }
        t0 = t1; t1 = tn; b0 = b1; b1 = bn; p0 = p1; p1 = pn;
    }
};

// The same quantities for k = k0, k0 + 4, k0 + 8, ... (k0 in 0..3), by the
// stride-4 recurrences T_{k+4} = 2 T_4 T_k - T_{k-4} (from T_m T_n =
// (T_{m+n} + T_{|m-n|}) / 2) and its derivative, started from T_{k0} and
// T_{k0-4} = T_{4-k0}: a lane that needs every fourth k steps N/4 times.
struct ModeRec4 {
    double dl, t4, b4, p4;
    double t0, t1, b0, b1, p0, p1;  // k - 4 and k: at x, at xbar, derivative at xbar
    __device__ void init(double x, double xb, int k0)
    {
        dl = x - xb;
        double T[5], B[5], P[5];
        T[0] = 1.0; T[1] = x; B[0] = 1.0; B[1] = xb; P[0] = 0.0; P[1] = 1.0;
#pragma unroll
        for (int k = 1; k < 4; ++k) {
            T[k + 1] = 2.0 * x * T[k] - T[k - 1];
            B[k + 1] = 2.0 * xb * B[k] - B[k - 1];
            P[k + 1] = 2.0 * B[k] + 2.0 * xb * P[k] - P[k - 1];
        }
        t4 = T[4]; b4 = B[4]; p4 = P[4];
        // select without indexing the arrays by a lane-dependent value
        t1 = T[0]; b1 = B[0]; p1 = P[0]; t0 = T[4]; b0 = B[4]; p0 = P[4];
#pragma unroll
        for (int m = 1; m < 4; ++m)
            if (k0 == m) { t1 = T[m]; b1 = B[m]; p1 = P[m]; t0 = T[4 - m]; b0 = B[4 - m]; p0 = P[4 - m]; }
    }
    __device__ void get(double &T, double &Tb, double &P, double &R1) const
    {
        T = t1; Tb = b1; P = p1 * dl; R1 = (t1 - b1) - P;
    }
    __device__ void advance4()
    {
        const double tn = 2.0 * t4 * t1 - t0;
        const double bn = 2.0 * b4 * b1 - b0;
        const double pn = 2.0 * p4 * b1 + 2.0 * b4 * p1 - p0;
        t0 = t1; t1 = tn; b0 = b1; b1 = bn; p0 = p1; p1 = pn;
    }
};

// T_k(x) alone for k = k0, k0 + 4, ... (the node values come from a table).
struct ModeT4 {
    double t4, t0, t1;  // T_4; T_{k-4}, T_k
    __device__ void init(double x, int k0)
    {
        double T[5];
        T[0] = 1.0; T[1] = x;
#pragma unroll
        for (int k = 1; k < 4; ++k) T[k + 1] = 2.0 * x * T[k] - T[k - 1];
        t4 = T[4];
        t1 = T[0]; t0 = T[4];
#pragma unroll
        for (int m = 1; m < 4; ++m)
            if (k0 == m) { t1 = T[m]; t0 = T[4 - m]; }
    }
    __device__ void advance4()
    {
        const double tn = 2.0 * t4 * t1 - t0;
        t0 = t1; t1 = tn;
    }
};

template <int D, int N4, int NC, int RB, int OCB>
__global__ __launch_bounds__(256) void k_contract_corr(const Inst *__restrict__ tab, int bpi,
                                                       int blocks_per_player)
{
    const InstView I = inst_view(tab, blockIdx.x / bpi);
    const int blk = blockIdx.x % bpi;
    const GameConst *__restrict__ gc = I.gc;
    const GameStatus *st = I.st;
    const double *__restrict__ Ubuf = I.U;
    const float *__restrict__ Bp32 = I.Bp32;
    const double *__restrict__ E = I.E;
    double *__restrict__ Wout = I.W;
    constexpr int NCB = NC / 16;
    constexpr int ROWS_W = RB * 16;
    constexpr int ROWS_B = 4 * ROWS_W;
    constexpr int LDB = NC == 32 ? 48 : 16;     // slab rows (floats): kq groups on disjoint banks
    constexpr int SLAB = OCB * N4 * LDB;        // OCB outer values per slab
    constexpr int OC_E4 = N4 * NC / 4;          // float4 elements per outer value
    constexpr int SLAB_E4 = OCB * OC_E4;
    constexpr int PF = (SLAB_E4 + 255) / 256;
    __shared__ float lds[2 * SLAB];
    __shared__ double dls[ROWS_B * (D - 1)];    // Delta of every row, for the epilogue

    if (st->converged) return;
    const int cur = st->cur;
    const int NN = (int)gc->NN;
    const int N = gc->N;
    const double *Uold = Ubuf + (long long)cur * D * NN;

    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int r16 = lane & 15, kq = lane >> 4;
    const int player = blk / blocks_per_player;
    const int tile = blk % blocks_per_player;
    const int row0 = tile * ROWS_B + wave * ROWS_W;

    int om[D - 1];
#pragma unroll
    for (int t = 0; t < D - 1; ++t) om[t] = t < player ? t : t + 1;

    // ---- per row: node, shift, inner-mode quantities, outer-mode recurrences ----
    float Tc[RB][N4 / 4], Rc[RB][N4 / 4], Pc[RB][N4 / 4];
    ModeRec ra[RB], rb_[RB];
    ModeRec4 ra4[RB];  // d = 3: the outer mode, this lane's values oc = 4 w + kq
#pragma unroll
    for (int rb = 0; rb < RB; ++rb) {
        const int j = min(row0 + rb * 16 + r16, NN - 1);
        double p[D], ub[D], b[D];
        node_state<D>(gc, Uold, j, p, ub, b);
        int dig[D];
        {
            int rem = j;
#pragma unroll
            for (int l = D - 1; l >= 0; --l) { dig[l] = rem % N; rem /= N; }
        }
        double xs[D - 1], xb[D - 1];
#pragma unroll
        for (int t = 0; t < D - 1; ++t) {
            double y = 0.0, xbar = 0.0;
#pragma unroll
            for (int l = 0; l < D; ++l)
                if (l == om[t]) { y = fma(gc->h, b[l], p[l]); xbar = gc->xnode[dig[l]]; }
            xs[t] = 2.0 * y / gc->pmax - 1.0;
            xb[t] = xbar;
            if (kq == 0) dls[(wave * ROWS_W + rb * 16 + r16) * (D - 1) + t] = xs[t] - xbar;
        }
        ModeRec4 rc;  // this lane's k = 4 t + kq
        rc.init(xs[D - 2], xb[D - 2], kq);
#pragma unroll
        for (int t = 0; t < N4 / 4; ++t) {
            double T, Tb, P, R1;
            rc.get(T, Tb, P, R1);
            Tc[rb][t] = (float)T;
            Rc[rb][t] = (float)R1;
            Pc[rb][t] = (float)P;
            rc.advance4();
        }
        if (D == 3) ra4[rb].init(xs[0], xb[0], kq);
        if (D >= 4) ra[rb].init(xs[0], xb[0]);
        if (D >= 4) rb_[rb].init(xs[1], xb[1]);
    }

    f32x4 acc[RB][NCB];
    double acc64[RB][NCB][4];
#pragma unroll
    for (int rb = 0; rb < RB; ++rb)
#pragma unroll
        for (int c = 0; c < NCB; ++c) {
            acc[rb][c] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int v = 0; v < 4; ++v) acc64[rb][c][v] = 0.0;
        }

    const float4 *Bg = reinterpret_cast<const float4 *>(Bp32 + (long long)player * gc->K * NC);
    const int n_outer = (D == 2) ? 1 : (D == 3 ? N : N * N);
    float4 pf[PF];
    auto load_slab = [&](int sb) {  // outer values past the last one read as zero
#pragma unroll
        for (int q = 0; q < PF; ++q) {
            const int e4 = tid + q * 256;
            if (e4 < SLAB_E4)
                pf[q] = sb * OCB + e4 / OC_E4 < n_outer ? Bg[(long long)sb * SLAB_E4 + e4]
                                                       : make_float4(0.f, 0.f, 0.f, 0.f);
        }
    };
    auto store_slab = [&](float *buf) {
#pragma unroll
        for (int q = 0; q < PF; ++q) {
            const int e4 = tid + q * 256;
            if (e4 < SLAB_E4) {
                const int e = 4 * e4, r = e / NC, c = e % NC;
                float *dst = buf + r * LDB + c;
                dst[0] = pf[q].x; dst[1] = pf[q].y; dst[2] = pf[q].z; dst[3] = pf[q].w;
            }
        }
    };

    float myRem[RB], myLin[RB], myFO[RB];
    const int n_slabs = (n_outer + OCB - 1) / OCB;
    load_slab(0);
    store_slab(lds);
    __syncthreads();
    for (int sb = 0; sb < n_slabs; ++sb) {
        const bool more = sb + 1 < n_slabs;
        if (more) load_slab(sb + 1);
#pragma unroll
        for (int ocl = 0; ocl < OCB; ++ocl) {
        const int oc = sb * OCB + ocl;
        const float *cb = lds + (sb & 1) * SLAB + ocl * N4 * LDB;
        // outer-mode factors of the remainder recursion
        float fRem[RB], fLin[RB], fFO[RB];
        if (D == 3) {
            // the lane with kq = oc mod 4 holds them (computed once per four outer values)
            if ((oc & 3) == 0) {
#pragma unroll
                for (int rb = 0; rb < RB; ++rb) {
                    if (oc > 0) ra4[rb].advance4();
                    double Ta, Tba, Pa, R1a;
                    ra4[rb].get(Ta, Tba, Pa, R1a);
                    myRem[rb] = (float)R1a;
                    myLin[rb] = (float)(Tba + Pa);
                    myFO[rb] = (float)Pa;
                }
            }
            const int src = r16 + 16 * (oc & 3);
#pragma unroll
            for (int rb = 0; rb < RB; ++rb) {
                fRem[rb] = __shfl(myRem[rb], src);
                fLin[rb] = __shfl(myLin[rb], src);
                fFO[rb] = __shfl(myFO[rb], src);
            }
        }
#pragma unroll
        for (int rb = 0; rb < RB; ++rb) {
            if (D == 3) {
            } else if (D == 2) {
                fRem[rb] = 0.f; fLin[rb] = 1.f; fFO[rb] = 0.f;
            } else {
                double Ta, Tba, Pa, R1a;
                ra[rb].get(Ta, Tba, Pa, R1a);
                double Rem = R1a, FO = Pa, Pb = Tba;
                if (D == 4) {
                    double Tb, Tbb, Pb2, R1b;
                    rb_[rb].get(Tb, Tbb, Pb2, R1b);
                    const double Lin = Pb + FO;
                    Rem = Rem * Tb + Lin * R1b + FO * Pb2;
                    FO = FO * Tbb + Pb * Pb2;
                    Pb = Pb * Tbb;
                }
                fRem[rb] = (float)Rem;
                fLin[rb] = (float)(Pb + FO);
                fFO[rb] = (float)FO;
            }
        }
        // all B fragments of this outer value first, so the LDS latency is paid once
        float bf[N4 / 4][NCB];
#pragma unroll
        for (int t = 0; t < N4 / 4; ++t)
#pragma unroll
            for (int c = 0; c < NCB; ++c) bf[t][c] = cb[(4 * t + kq) * LDB + c * 16 + r16];
        // keep the reads ahead of the MFMAs (the scheduler would otherwise sink
        // each read to just before its MFMA and expose its latency); measured
        // faster at d = 3 only
        if constexpr (D == 3) __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int t = 0; t < N4 / 4; ++t) {
#pragma unroll
            for (int rb = 0; rb < RB; ++rb) {
                const float a = fmaf(fRem[rb], Tc[rb][t], fmaf(fLin[rb], Rc[rb][t], fFO[rb] * Pc[rb][t]));
#pragma unroll
                for (int c = 0; c < NCB; ++c)
                    acc[rb][c] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, bf[t][c], acc[rb][c], 0, 0, 0);
            }
        }
        // advance the outer-mode recurrences (d = 3: at the next window)
        if (D == 4) {
            const int kb = oc % N;
            if (kb == N - 1) {
                const int ka = oc / N;
#pragma unroll
                for (int rb = 0; rb < RB; ++rb) {
                    ra[rb].advance(ka);
                    rb_[rb].init(rb_[rb].x, rb_[rb].xb);
                }
            } else {
#pragma unroll
                for (int rb = 0; rb < RB; ++rb) rb_[rb].advance(kb);
            }
        }
        }
        // binary32 partial sums of this slab (OCB * N4 K-rows) into FP64
#pragma unroll
        for (int rb = 0; rb < RB; ++rb)
#pragma unroll
            for (int c = 0; c < NCB; ++c) {
#pragma unroll
                for (int v = 0; v < 4; ++v) acc64[rb][c][v] += (double)acc[rb][c][v];
                acc[rb][c] = f32x4{0.f, 0.f, 0.f, 0.f};
            }
        if (more) store_slab(lds + ((sb + 1) & 1) * SLAB);
        __syncthreads();
    }

    // ---- epilogue: element v of lane c + 16 kq is row 4 kq + v (f32 layout) ----
    const int NM = NN / N;
    int stride_i = 1;
    for (int l = player + 1; l < D; ++l) stride_i *= N;
    const double *Ei = E + (long long)player * D * NM * NC;
    double *Wp = Wout + (long long)player * NN * NC;
#pragma unroll
    for (int rb = 0; rb < RB; ++rb)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int rl = rb * 16 + 4 * kq + v;
            const int j = row0 + rl;
            if (j >= NN) continue;
            // node index without mode i
            const int hi = j / (stride_i * N), lo = j % stride_i;
            const int jm = hi * stride_i + lo;
            const double *dl = dls + (wave * ROWS_W + rl) * (D - 1);
#pragma unroll
            for (int c = 0; c < NCB; ++c) {
                const int col = c * 16 + r16;
                double w = acc64[rb][c][v] + Ei[(long long)jm * NC + col];
#pragma unroll
                for (int t = 0; t < D - 1; ++t) w = fma(dl[t], Ei[((long long)(1 + t) * NM + jm) * NC + col], w);
                Wp[(long long)j * NC + col] = w;
            }
        }
}

// d = 3 form of the remainder contraction.  With o < n the two modes other
// than i and, per mode, T = T_k(x), Tb = T_k(xbar), P = T_k'(xbar) Delta,
// R1 = T - Tb - P and D = T - Tb = P + R1, the Khatri-Rao element splits
// exactly as
//   T_o T_n = Tb_o Tb_n + (P_o Tb_n + Tb_o P_n) + (R1_o Tb_n + Tb_o R1_n) + D_o D_n.
// The first two groups are E0 and the E1 terms (FP64, epilogue).  In the third
// group one mode sits at its node, so it contracts against the coefficient
// tensor with that mode at the nodes: sum_o R1_o Co[jn][o] + sum_n R1_n Cn[jo][n]
// (E2, written by the Taylor launch, one N4 x NC slab per line), 2 N4 K-rows.
// The last group is the main binary32 GEMM, A = D_o D_n: one product per A
// element (the outer factor D_o of a row comes from an LDS table), against
// three for the general recursion above.
//
// Split form (SPLIT, corr3_split16): the main GEMM runs in two levels on
// v_mfma_f32_16x16x32_bf16.  Per outer value k_o, P[r][k_i] = sum_kn D_n[r][kn]
// C[k_o][kn][k_i] with both operands as three bfloat16 pieces (D_n split once
// per row, C split by the transform) and the six piece products of leading
// order (hi hi, hi mid, mid hi, hi lo, mid mid, lo hi; the three dropped
// ones are below 2^-24 of the product), accumulated in binary32; then
// acc += D_o[r][k_o] P on the VALU.  The K index of the MFMA runs over
// kn = 4 e + g (lane group g, element e), the layout of the stride-4 basis
// recurrences, padded to 32 with zeros.
//
// Rows: the nodes of player i ordered by line, r = (jo N + jn) N + ji, so the
// 16 rows of an MFMA block share (jo, jn) when N is a multiple of 16; a block
// that straddles lines runs the E2 terms once per line, the A rows of the
// other lines masked to zero.  binary32 partial sums enter FP64 every FOLD
// slabs (FOLD OCB N4 K-rows); in the split form the whole remainder (one-mode
// terms and every outer value) is summed in binary32 and enters FP64 in the
// epilogue.
// Slab sb (OCB outer values) of the packed binary32 coefficients into
// registers: float4 element e4 = tid + NTHR q of the slab.  Outer values past
// the last one (slabs padded to whole groups) read the last one's
// coefficients (their D_o table entries are zero); threads past the slab
// read a valid element and do not store it.
template <int PF, int SLAB_E4, int OC_E4, int OCB, int NTHR>
__device__ __forceinline__ void corr3_load(f32x4 (&pf)[PF], const f32x4 *__restrict__ Bg, int sb, int n_outer,
                                           int tid)
{
#pragma unroll
    for (int q = 0; q < PF; ++q) {
        const int e4 = min(tid + q * NTHR, SLAB_E4 - 1);
        const int oc = min(sb * OCB + e4 / OC_E4, n_outer - 1);
        pf[q] = Bg[(long long)oc * OC_E4 + e4 % OC_E4];
    }
}
template <int PF, int SLAB_E4, int NTHR>
__device__ __forceinline__ void corr3_store_flat(const f32x4 (&pf)[PF], float *buf, int tid)
{
#pragma unroll
    for (int q = 0; q < PF; ++q) {
        const int e4 = tid + q * NTHR;
        if (SLAB_E4 % NTHR == 0 || e4 < SLAB_E4) reinterpret_cast<f32x4 *>(buf)[e4] = pf[q];
    }
}
template <int PF, int SLAB_E4, int NC, int LDB, int NTHR>
__device__ __forceinline__ void corr3_store(const f32x4 (&pf)[PF], float *buf, int tid)
{
#pragma unroll
    for (int q = 0; q < PF; ++q) {
        const int e4 = tid + q * NTHR;
        if (e4 < SLAB_E4) {
            const int e = 4 * e4;
            *reinterpret_cast<f32x4 *>(buf + (e / NC) * LDB + e % NC) = pf[q];
        }
    }
}

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

template <int N4, int NC, int RB, int OCB, int FOLD, int WPB, int NX, bool SPLIT>
__global__ __launch_bounds__(64 * WPB) __attribute__((amdgpu_waves_per_eu(RB == 1 ? 3 : (SPLIT && RB == 2 ? 2 : 1))))
void k_contract_corr3(
    const Inst *__restrict__ tab, int bpi, int blocks_per_player)
{
    // NX = N when N is known at compile time (N = N4, every shape of the
    // benchmark workloads), 0 for the general case.  With NX a multiple of 16
    // the 16 rows of an MFMA block lie on one line.
    constexpr int D = 3;
    constexpr bool ONE_LINE = NX > 0 && NX % 16 == 0;
    const InstView I = inst_view(tab, blockIdx.x / bpi);
    const int blk = blockIdx.x % bpi;
    const GameConst *__restrict__ gc = I.gc;
    const GameStatus *st = I.st;
    constexpr int NCB = NC / 16;
    constexpr int NT = N4 / 4;
    constexpr int CH = corr3_chunk(N4, NC);      // floats per lane of a nodal slab
    constexpr int ROWS_W = RB * 16;
    constexpr int ROWS_B = WPB * ROWS_W;         // WPB waves share every coefficient slab
    constexpr int NTHR = 64 * WPB;
    constexpr int LDB = NC == 32 ? 48 : 16;      // slab rows (floats): kq groups on disjoint banks
    // float4 elements per outer value: binary32 N4 x NC, or (split form) 3
    // pieces x NCB fragments of 64 lanes x 16 bytes, copied as stored
    constexpr int OC_E4 = SPLIT ? 3 * NCB * 64 : N4 * NC / 4;
    constexpr int SLAB = SPLIT ? OCB * OC_E4 * 4 : OCB * N4 * LDB;  // floats; OCB outer values per slab
    constexpr int SLAB_E4 = OCB * OC_E4;
    constexpr int PF = (SLAB_E4 + NTHR - 1) / NTHR;
    constexpr int LDO = N4 + 1;                  // row stride of the D_o table [row][k_o]
    constexpr int LDT = ROWS_B;                  // split form: the table transposed, [k_o][row]
    __shared__ __attribute__((aligned(16))) float lds[2 * SLAB];
    __shared__ __attribute__((aligned(16))) float dO[SPLIT ? N4 * LDT : ROWS_B * LDO];
    __shared__ double dls[ROWS_B * 2];           // Delta_o, Delta_n of every row, for the epilogue

    if (st->converged) return;
    const int cur = st->cur;
    const int NN = (int)gc->NN;
    const int N = NX > 0 ? NX : gc->N;
    const int NM = NN / N;  // nodes of the other modes (lines)
    const double *Uold = I.U + (long long)cur * D * NN;

    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int r16 = lane & 15, kq = lane >> 4;
    const int player = blk / blocks_per_player;
    const int tile = blk % blocks_per_player;
    const int row0 = tile * ROWS_B + wave * ROWS_W;
    const int om0 = player == 0 ? 1 : 0, om1 = player == 2 ? 1 : 2;
    const int st_i = player == 0 ? N * N : (player == 1 ? N : 1);    // node stride of mode i
    const int st_o = om0 == 0 ? N * N : N, st_n = om1 == 1 ? N : 1;  // of modes o and n
    // a / N for 0 <= a < 2^21: exact division when N is a constant, else in
    // binary32 ((a + 1/2) / N lies at least 1/(2N) from an integer, far beyond
    // the rounding of the product)
    const float invN = 1.0f / (float)N;
    auto divN = [&](int a) { return NX > 0 ? a / NX : (int)(((float)a + 0.5f) * invN); };

    // ---- the first coefficient slab and the nodal tensors of each row block's
    //      first line (lane-contiguous float4 loads), issued first so that
    //      their latency overlaps the per-row work ----
    const f32x4 *Bg = SPLIT ? reinterpret_cast<const f32x4 *>(I.Bs16 + player * split16_player(N, NC))
                            : reinterpret_cast<const f32x4 *>(I.Bp32 + (long long)player * gc->K * NC);
    const int n_outer = N;
    f32x4 pf0[PF];
    corr3_load<PF, SLAB_E4, OC_E4, OCB, NTHR>(pf0, Bg, 0, n_outer, tid);
    const float *E2 = reinterpret_cast<const float *>(I.E + (long long)D * D * NM * NC) +
                      (long long)player * 2 * N * 64 * CH;
    f32x4 nbo[RB][CH / 4], nbn[RB][CH / 4];
#pragma unroll
    for (int rb = 0; rb < RB; ++rb) {
        const int L = divN(min(row0 + rb * 16, NN - 1));
        const int jo = divN(L), jn = L - jo * N;
        const f32x4 *Bo = reinterpret_cast<const f32x4 *>(E2 + ((long long)jn * 64 + lane) * CH);        // Co[jn]
        const f32x4 *Bn = reinterpret_cast<const f32x4 *>(E2 + (((long long)N + jo) * 64 + lane) * CH); // Cn[jo]
#pragma unroll
        for (int q = 0; q < CH / 4; ++q) {
            nbo[rb][q] = Bo[q];
            nbn[rb][q] = Bn[q];
        }
    }

    // ---- per row: node, shift, D_n, R1_n, R1_o (this lane's k = 4 t + kq), D_o (table) ----
    float Dn[RB][NT], R1n[RB][NT], R1o[RB][NT];
#pragma unroll
    for (int rb = 0; rb < RB; ++rb) {
        const int r = min(row0 + rb * 16 + r16, NN - 1);
        const int L = divN(r), ji = r - L * N;
        const int jo = divN(L), jn = L - jo * N;
        const int j = ji * st_i + jo * st_o + jn * st_n;
        // T_k and T_k' at the node from the table (this lane's k = 4 t + kq,
        // zero past N), loaded before the node state so that the two round
        // trips overlap
        const double2 *tbo = reinterpret_cast<const double2 *>(gc->TnP) + jo * kMaxN + kq;
        const double2 *tbn = reinterpret_cast<const double2 *>(gc->TnP) + jn * kMaxN + kq;
        double2 bo[NT], bn[NT];
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            bn[t] = tbn[4 * t];
            bo[t] = tbo[4 * t];
        }
        double p[D], ub[D], b[D];
        node_state<D>(gc, Uold, j, p, ub, b);
        double xo = 0.0, xn = 0.0;
#pragma unroll
        for (int l = 0; l < D; ++l) {
            const double y = 2.0 * fma(gc->h, b[l], p[l]) / gc->pmax - 1.0;
            if (l == om0) xo = y;
            if (l == om1) xn = y;
        }
        const double xbo = gc->xnode[jo], xbn = gc->xnode[jn];
        const int rl = wave * ROWS_W + rb * 16 + r16;
        if (kq == 0) {
            dls[rl * 2 + 0] = xo - xbo;
            dls[rl * 2 + 1] = xn - xbn;
        }
        // T_k at the shifted point by recurrence
        ModeT4 mo, mn;
        mo.init(xo, kq);
        mn.init(xn, kq);
        const double dlo = xo - xbo, dln = xn - xbn;
        float *dOl = SPLIT ? dO + kq * LDT + rl : dO + rl * LDO + kq;
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            const int k = 4 * t + kq;
            const double Dnk = mn.t1 - bn[t].x;   // D = T - Tb
            Dn[rb][t] = (float)Dnk;
            R1n[rb][t] = (float)(Dnk - bn[t].y * dln);  // R1 = D - T'(xbar) Delta
            mn.advance4();
            const double Dok = mo.t1 - bo[t].x;
            R1o[rb][t] = (float)(Dok - bo[t].y * dlo);
            const float dov = k < N ? (float)Dok : 0.f;  // outer values past N: zero rows
            dOl[SPLIT ? 4 * t * LDT : 4 * t] = dov;
            mo.advance4();
        }
    }

    // binary32 form: acc holds one group of outer values, acc64 the FP64
    // sum; split form: acc holds the whole remainder in binary32 (the one-mode
    // terms, then every outer value) and acc64 is unused
    f32x4 acc[RB][NCB];
    double acc64[RB][NCB][4];
#pragma unroll
    for (int rb = 0; rb < RB; ++rb)
#pragma unroll
        for (int c = 0; c < NCB; ++c) {
            acc[rb][c] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int v = 0; v < 4; ++v) acc64[rb][c][v] = 0.0;
        }

    // FOLD slabs per group (FOLD OCB = 4 outer values; the last group is
    // padded with zero rows of A): the first MFMA of a group starts from a
    // zero accumulator and the group's binary32 sums then enter FP64, with no
    // branch inside the group; slab sb sits in LDS buffer sb mod 2.
    static_assert(OCB * FOLD == 4, "four outer values per group");
    const int n_groups = (n_outer + OCB * FOLD - 1) / (OCB * FOLD);
    const int n_slabs = n_groups * FOLD;
    if constexpr (SPLIT)
        corr3_store_flat<PF, SLAB_E4, NTHR>(pf0, lds, tid);
    else
        corr3_store<PF, SLAB_E4, NC, LDB, NTHR>(pf0, lds, tid);
    __syncthreads();  // also publishes the D_o table

    // ---- one-mode remainder terms against the nodal tensors of each line
    //      (before the main loop: R1_n, R1_o are dead afterwards) ----
#pragma unroll
    for (int rb = 0; rb < RB; ++rb) {
        const int rbase = row0 + rb * 16;
        if (rbase >= NN) continue;
        const int myr = rbase + r16;
        const int Lfirst = divN(rbase), Llast = ONE_LINE ? Lfirst : divN(min(rbase + 15, NN - 1));
        for (int L = Lfirst; L <= Llast; ++L) {
            const bool in = ONE_LINE || (myr < NN && divN(myr) == L);
            if (L != Lfirst) {  // further lines of a block that straddles lines: their slabs
                const int jo = divN(L), jn = L - jo * N;
                const f32x4 *Bo = reinterpret_cast<const f32x4 *>(E2 + ((long long)jn * 64 + lane) * CH);
                const f32x4 *Bn = reinterpret_cast<const f32x4 *>(E2 + (((long long)N + jo) * 64 + lane) * CH);
#pragma unroll
                for (int q = 0; q < CH / 4; ++q) {
                    nbo[rb][q] = Bo[q];
                    nbn[rb][q] = Bn[q];
                }
            }
            f32x4 na[NCB];
#pragma unroll
            for (int t = 0; t < NT; ++t) {
                const float ao = in ? R1o[rb][t] : 0.f, an = in ? R1n[rb][t] : 0.f;
#pragma unroll
                for (int c = 0; c < NCB; ++c) {
                    const int e = t * NCB + c;  // entry of the lane's chunk
                    const f32x4 cin = t == 0 ? f32x4{0.f, 0.f, 0.f, 0.f} : na[c];
                    na[c] = __builtin_amdgcn_mfma_f32_16x16x4f32(ao, nbo[rb][e >> 2][e & 3], cin, 0, 0, 0);
                    na[c] = __builtin_amdgcn_mfma_f32_16x16x4f32(an, nbn[rb][e >> 2][e & 3], na[c], 0, 0, 0);
                }
            }
#pragma unroll
            for (int c = 0; c < NCB; ++c)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    if constexpr (SPLIT)
                        acc[rb][c][v] += na[c][v];
                    else
                        acc64[rb][c][v] += (double)na[c][v];
                }
        }
    }

    // split form: D_n of each row as three bfloat16 pieces, element e = k / 4
    // of lane group kq (k = 4 e + kq), zero past N4
    bf16x8 a16[RB][3];
    if constexpr (SPLIT) {
#pragma unroll
        for (int rb = 0; rb < RB; ++rb)
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                float r = e < NT ? Dn[rb][e] : 0.f;
                // the pieces split the binary32 value (an opaque copy keeps the
                // compiler from rounding the FP64 value to bf16 directly, a
                // longer sequence)
                __asm__("" : "+v"(r));
#pragma unroll
                for (int p = 0; p < 3; ++p) {
                    const __bf16 h = (__bf16)r;
                    a16[rb][p][e] = h;
                    r -= (float)h;
                }
            }
    }

    // one group of four outer values; the split form keeps the group loop
    // rolled (a known trip count would otherwise unroll it whole and hoist
    // every slab load)
    auto run_group = [&](const int g) __attribute__((always_inline)) {
#pragma unroll
        for (int q = 0; q < FOLD; ++q) {
            const int sb = g * FOLD + q;
            const bool more = sb + 1 < n_slabs;
            f32x4 pf[PF];
            // (the last slab loads a valid, unused slab: pf stays unconditionally defined)
            corr3_load<PF, SLAB_E4, OC_E4, OCB, NTHR>(pf, Bg, more ? sb + 1 : sb, n_outer, tid);
            if constexpr (SPLIT) {
#pragma unroll
                for (int ocl = 0; ocl < OCB; ++ocl) {
                    const int oc = sb * OCB + ocl;
                    const f32x4 *fb = reinterpret_cast<const f32x4 *>(lds + (sb & 1) * SLAB) + ocl * OC_E4 + lane;
                    bf16x8 b16[3][NCB];
#pragma unroll
                    for (int p = 0; p < 3; ++p)
#pragma unroll
                        for (int c = 0; c < NCB; ++c) b16[p][c] = __builtin_bit_cast(bf16x8, fb[(p * NCB + c) * 64]);
                    f32x4 fo4[RB];  // D_o of output rows 4 kq + v
#pragma unroll
                    for (int rb = 0; rb < RB; ++rb)
                        fo4[rb] = *reinterpret_cast<const f32x4 *>(dO + oc * LDT + wave * ROWS_W + rb * 16 + 4 * kq);
                    __builtin_amdgcn_sched_barrier(0);
                    // piece products (A piece, B piece), smallest first
                    constexpr int PA[6] = {2, 1, 0, 1, 0, 0}, PB[6] = {0, 1, 2, 0, 1, 0};
                    f32x4 P[RB][NCB];
#pragma unroll
                    for (int pp = 0; pp < 6; ++pp)
#pragma unroll
                        for (int rb = 0; rb < RB; ++rb)
#pragma unroll
                            for (int c = 0; c < NCB; ++c)
                                P[rb][c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                                    a16[rb][PA[pp]], b16[PB[pp]][c],
                                    pp == 0 ? f32x4{0.f, 0.f, 0.f, 0.f} : P[rb][c], 0, 0, 0);
#pragma unroll
                    for (int rb = 0; rb < RB; ++rb)
#pragma unroll
                        for (int c = 0; c < NCB; ++c)
#pragma unroll
                            for (int v = 0; v < 4; ++v) acc[rb][c][v] = fmaf(fo4[rb][v], P[rb][c][v], acc[rb][c][v]);
                }
            } else {
#pragma unroll
                for (int ocl = 0; ocl < OCB; ++ocl) {
                    const int oc = sb * OCB + ocl;
                    const float *cb = lds + (sb & 1) * SLAB + ocl * N4 * LDB;
                    float bf[NT][NCB];
#pragma unroll
                    for (int t = 0; t < NT; ++t)
#pragma unroll
                        for (int c = 0; c < NCB; ++c) bf[t][c] = cb[(4 * t + kq) * LDB + c * 16 + r16];
                    float fo[RB];
#pragma unroll
                    for (int rb = 0; rb < RB; ++rb) fo[rb] = dO[(wave * ROWS_W + rb * 16 + r16) * LDO + oc];
                    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                    for (int t = 0; t < NT; ++t) {
#pragma unroll
                        for (int rb = 0; rb < RB; ++rb) {
                            const float a = fo[rb] * Dn[rb][t];
#pragma unroll
                            for (int c = 0; c < NCB; ++c) {
                                const f32x4 cin = (q == 0 && ocl == 0 && t == 0) ? f32x4{0.f, 0.f, 0.f, 0.f}
                                                                                 : acc[rb][c];
                                acc[rb][c] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, bf[t][c], cin, 0, 0, 0);
                            }
                        }
                    }
                }
            }
            if (more) {
                if constexpr (SPLIT)
                    corr3_store_flat<PF, SLAB_E4, NTHR>(pf, lds + ((sb + 1) & 1) * SLAB, tid);
                else
                    corr3_store<PF, SLAB_E4, NC, LDB, NTHR>(pf, lds + ((sb + 1) & 1) * SLAB, tid);
            }
            __syncthreads();
        }
        if constexpr (!SPLIT) {
#pragma unroll
            for (int rb = 0; rb < RB; ++rb)
#pragma unroll
                for (int c = 0; c < NCB; ++c)
#pragma unroll
                    for (int v = 0; v < 4; ++v) acc64[rb][c][v] += (double)acc[rb][c][v];
        }
    };
    if constexpr (SPLIT) {
        // the split form sums every outer value in binary32 (the 6 x 32 piece
        // products of one outer value already are) and enters FP64 in the
        // epilogue
#pragma unroll 1
        for (int g = 0; g < n_groups; ++g) run_group(g);
    } else {
        for (int g = 0; g < n_groups; ++g) run_group(g);
    }

    // ---- epilogue: element v of lane c + 16 kq is row 4 kq + v (f32 layout);
    //      W = remainder + E0 + Delta_o E1_o + Delta_n E1_n ----
    const double *Ei = I.E + (long long)player * D * NM * NC;
    double *Wp = I.W + (long long)player * NN * NC;
#pragma unroll
    for (int rb = 0; rb < RB; ++rb) {
        double e0[NCB], e1o[NCB], e1n[NCB];
        if constexpr (ONE_LINE) {  // one line per block of 16 rows: its E tensors once per column
            const int L = divN(min(row0 + rb * 16, NN - 1));
#pragma unroll
            for (int c = 0; c < NCB; ++c) {
                const int col = c * 16 + r16;
                e0[c] = Ei[(long long)L * NC + col];
                e1o[c] = Ei[((long long)NM + L) * NC + col];
                e1n[c] = Ei[((long long)2 * NM + L) * NC + col];
            }
        }
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int rl = rb * 16 + 4 * kq + v;
            const int r = row0 + rl;
            if (r >= NN) continue;
            const int L = divN(r), ji = r - L * N;
            const int jo = divN(L), jn = L - jo * N;
            const int j = ji * st_i + jo * st_o + jn * st_n;
            const double dlo = dls[(wave * ROWS_W + rl) * 2 + 0], dln = dls[(wave * ROWS_W + rl) * 2 + 1];
#pragma unroll
            for (int c = 0; c < NCB; ++c) {
                const int col = c * 16 + r16;
                if constexpr (!ONE_LINE) {
                    e0[c] = Ei[(long long)L * NC + col];
                    e1o[c] = Ei[((long long)NM + L) * NC + col];
                    e1n[c] = Ei[((long long)2 * NM + L) * NC + col];
                }
                double w = (SPLIT ? (double)acc[rb][c][v] : acc64[rb][c][v]) + e0[c];
                w = fma(dlo, e1o[c], w);
                w = fma(dln, e1n[c], w);
                Wp[(long long)j * NC + col] = w;
            }
        }
    }
}

// Waves per block of the d = 3 mixed contraction (they share every
// coefficient slab staged in LDS).
constexpr int kCorr3Waves = 4;

template <int N4, int RB, int NX>
static hipError_t launch_corr3_nrx(const GameConst &hc, const StepBuffers &b, hipStream_t s)
{
    constexpr int NC = N4 <= 16 ? 16 : 32;
    constexpr int W = kCorr3Waves;
    constexpr bool SPLIT = corr3_split16(3, N4);
    const int NN = (int)hc.NN;
    const int bpp = (NN + W * RB * 16 - 1) / (W * RB * 16);
    const int bpi = bpp * 3;
    if (b.ocb == 2)
        hipLaunchKernelGGL((k_contract_corr3<N4, NC, RB, 2, 2, W, NX, SPLIT>), dim3((unsigned)(bpi * b.count)),
                           dim3(64 * W), 0, s, b.tab, bpi, bpp);
    else
        hipLaunchKernelGGL((k_contract_corr3<N4, NC, RB, 1, 4, W, NX, SPLIT>), dim3((unsigned)(bpi * b.count)),
                           dim3(64 * W), 0, s, b.tab, bpi, bpp);
    return hipGetLastError();
}

template <int N4, int RB>
static hipError_t launch_corr3_nr(const GameConst &hc, const StepBuffers &b, hipStream_t s)
{
    return hc.N == N4 ? launch_corr3_nrx<N4, RB, N4>(hc, b, s) : launch_corr3_nrx<N4, RB, 0>(hc, b, s);
}

template <int N4>
static hipError_t launch_corr3_n(const GameConst &hc, const StepBuffers &b, hipStream_t s)
{
    switch (b.rb) {
        case 1: return launch_corr3_nr<N4, 1>(hc, b, s);
        case 4: return launch_corr3_nr<N4, 4>(hc, b, s);
        default: return launch_corr3_nr<N4, 2>(hc, b, s);
    }
}

template <int D, int N4, int RB>
static hipError_t launch_corr_dnr(const GameConst &hc, const StepBuffers &b, hipStream_t s)
{
    constexpr int NC = N4 <= 16 ? 16 : 32;
    const int NN = (int)hc.NN;
    const int bpp = (NN + 4 * RB * 16 - 1) / (4 * RB * 16);
    const int bpi = bpp * D;
    if (D >= 3 && b.ocb == 2)
        hipLaunchKernelGGL((k_contract_corr<D, N4, NC, RB, D >= 3 ? 2 : 1>), dim3((unsigned)(bpi * b.count)),
                           dim3(256), 0, s, b.tab, bpi, bpp);
    else
        hipLaunchKernelGGL((k_contract_corr<D, N4, NC, RB, 1>), dim3((unsigned)(bpi * b.count)), dim3(256), 0, s,
                           b.tab, bpi, bpp);
    return hipGetLastError();
}

template <int D, int N4>
static hipError_t launch_corr_dn(const GameConst &hc, const StepBuffers &b, hipStream_t s)
{
    switch (b.rb) {
        case 1: return launch_corr_dnr<D, N4, 1>(hc, b, s);
        case 4: return launch_corr_dnr<D, N4, 4>(hc, b, s);
        default: return launch_corr_dnr<D, N4, 2>(hc, b, s);
    }
}

template <int D>
static hipError_t launch_corr_d(const GameConst &hc, const StepBuffers &b, hipStream_t s)
{
    switch (hc.N4) {
        case 4: return launch_corr_dn<D, 4>(hc, b, s);
        case 8: return launch_corr_dn<D, 8>(hc, b, s);
        case 12: return launch_corr_dn<D, 12>(hc, b, s);
        case 16: return launch_corr_dn<D, 16>(hc, b, s);
        case 20: return launch_corr_dn<D, 20>(hc, b, s);
        case 24: return launch_corr_dn<D, 24>(hc, b, s);
        case 28: return launch_corr_dn<D, 28>(hc, b, s);
        case 32: return launch_corr_dn<D, 32>(hc, b, s);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_contract_corr(const GameConst &hc, const StepBuffers &b, hipStream_t s)
{
    if (hc.d == 3) {
        switch (hc.N4) {
            case 4: return launch_corr3_n<4>(hc, b, s);
            case 8: return launch_corr3_n<8>(hc, b, s);
            case 12: return launch_corr3_n<12>(hc, b, s);
            case 16: return launch_corr3_n<16>(hc, b, s);
            case 20: return launch_corr3_n<20>(hc, b, s);
            case 24: return launch_corr3_n<24>(hc, b, s);
            case 28: return launch_corr3_n<28>(hc, b, s);
            case 32: return launch_corr3_n<32>(hc, b, s);
        }
        return hipErrorInvalidValue;
    }
    switch (hc.d) {
        case 2: return launch_corr_d<2>(hc, b, s);
        case 4: return launch_corr_d<4>(hc, b, s);
    }
    return hipErrorInvalidValue;
}

}  // namespace cg
