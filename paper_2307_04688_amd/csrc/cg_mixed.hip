// cg_mixed.hip -- contraction of the value-iteration step with binary32 MFMA
// and an FP64 correction (precision CG_FP32_CORR).
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
// ~Delta^2, runs on binary32 MFMA (inputs rounded to binary32, products
// accumulated in binary32 over the K-rows of one LDS slab -- N4 or 2 N4 --
// then added into FP64).
//
// A2 is built per K element from per-mode quantities: with T = T_k(x),
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
    switch (hc.d) {
        case 2: return launch_corr_d<2>(hc, b, s);
        case 3: return launch_corr_d<3>(hc, b, s);
        case 4: return launch_corr_d<4>(hc, b, s);
    }
    return hipErrorInvalidValue;
}

}  // namespace cg
