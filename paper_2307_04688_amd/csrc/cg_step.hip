// cg_step.hip -- one iteration r -> r+1 of the value iteration (Steps 1-4 of
// Section 2.1, implemented as in Section 3.4) for every player and node.
//
// Structure of the work.  For player i and node j the N_u update points
// p_j + h g(p_j, [u_m, u_{-i}]) share every coordinate except the i-th, which
// is affine in u_m.  So V_i restricted to that line is a 1-D Chebyshev series
// whose coefficients are
//     w_i[j, k_i] = sum_{k_{-i}} c_i[k] prod_{l != i} T_{k_l}(x_l(j)),
// one contraction of the d-1 other modes at one point.  Over all nodes of a
// player this is the GEMM
//     W_i (N^d x N) = KR_i (N^d x N^(d-1)) * C_i (N^(d-1) x N),
// where row j of KR_i is the Khatri-Rao product of the basis vectors
// (T_k(x_l(j)))_k of the other modes and C_i is the coefficient tensor
// unfolded with mode i as columns.  The GEMM runs on MFMA (f64 16x16x4);
// KR_i is generated in registers from per-row recurrences, C_i is read from
// a packed copy in L2.  The rest of the step (line samples, u-fit, argmax,
// residual) is per-row FP64 VALU work with long dependency chains; it runs
// in a second kernel at its own occupancy, reading W_i back from L2/MALL, so
// that its registers do not limit the waves of the MFMA kernel.
#include "cg_line.h"

namespace cg {

// ---------------------------------------------------------------------------
// Contraction kernel, FP64: W_i = KR_i * C_i for one tile of rows.  Block = 4
// waves; wave w owns RB row blocks of 16 nodes of one player.  Lane layout
// of v_mfma_f64_16x16x4f64: A[r][k] and B[k][c] come from lane r + 16 k
// (resp. c + 16 k); D[g + 4 v][c] sits in lane c + 16 g, element v (rows
// interleaved by 4, unlike the f32 forms).
//
// The packed operand of the player (K x NC) streams through LDS in slabs of
// OCB * N4 rows (OCB values of the outer modes), double-buffered: the block
// loads slab s+1 into registers while its waves run the MFMAs of slab s.  The
// result rows go to W[i][j][0..NC) (L2/MALL-resident) for the line kernel.
template <int D, int N4, int NC, int RB, int OCB>
__global__ __launch_bounds__(256) void k_contract_f64(const Inst *__restrict__ tab, int bpi, int blocks_per_player)
{
    const InstView I = inst_view(tab, blockIdx.x / bpi);
    const int blk = blockIdx.x % bpi;
    const GameConst *__restrict__ gc = I.gc;
    const GameStatus *st = I.st;
    const double *__restrict__ Ubuf = I.U;
    const double *__restrict__ Bp = I.Bp;
    double *__restrict__ Wout = I.W;
    constexpr int NCB = NC / 16;
    constexpr int ROWS_W = RB * 16;
    constexpr int ROWS_B = 4 * ROWS_W;
    constexpr int LDB = NC == 32 ? 48 : 16;       // slab rows: kq groups on disjoint banks
    constexpr int SLAB = OCB * N4 * LDB;
    constexpr int OC_E2 = N4 * NC / 2;            // double2 elements per outer value
    constexpr int SLAB_E2 = OCB * OC_E2;          // double2 elements per slab
    constexpr int PF = (SLAB_E2 + 255) / 256;     // double2 prefetch registers per thread
    __shared__ double lds[2 * SLAB];

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

    int om[D - 1];  // other modes in increasing order
#pragma unroll
    for (int t = 0; t < D - 1; ++t) om[t] = t < player ? t : t + 1;

    // ---- shifted coordinates and basis values of each row ----
    double xo[RB][D - 1];
    double Tl[RB][N4 / 4];
#pragma unroll
    for (int rb = 0; rb < RB; ++rb) {
        const int j = min(row0 + rb * 16 + r16, NN - 1);
        double p[D], ub[D], b[D];
        node_state<D>(gc, Uold, j, p, ub, b);
#pragma unroll
        for (int t = 0; t < D - 1; ++t) {
            double y = 0.0;
#pragma unroll
            for (int l = 0; l < D; ++l)
                if (l == om[t]) y = fma(gc->h, b[l], p[l]);
            xo[rb][t] = 2.0 * y / gc->pmax - 1.0;
        }
        const double xl = xo[rb][D - 2];
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

    f64x4 acc[RB][NCB];
#pragma unroll
    for (int rb = 0; rb < RB; ++rb)
#pragma unroll
        for (int c = 0; c < NCB; ++c) acc[rb][c] = f64x4{0.0, 0.0, 0.0, 0.0};

    const double2 *Bg = reinterpret_cast<const double2 *>(Bp + (long long)player * gc->K * NC);
    const int n_outer = (D == 2) ? 1 : (D == 3 ? N : N * N);
    double2 pf[PF];
    auto load_slab = [&](int sb) {  // outer values past the last one read as zero
#pragma unroll
        for (int q = 0; q < PF; ++q) {
            const int e2 = tid + q * 256;
            if (e2 < SLAB_E2)
                pf[q] = sb * OCB + e2 / OC_E2 < n_outer ? Bg[(long long)sb * SLAB_E2 + e2] : double2{0.0, 0.0};
        }
    };
    auto store_slab = [&](double *buf) {
#pragma unroll
        for (int q = 0; q < PF; ++q) {
            const int e2 = tid + q * 256;
            if (e2 < SLAB_E2) {
                const int e = 2 * e2, r = e / NC, c = e % NC;
                buf[r * LDB + c] = pf[q].x;
                buf[r * LDB + c + 1] = pf[q].y;
            }
        }
    };

    double Ta_prev[RB], Ta[RB], Tb_prev[RB], Tb[RB];
#pragma unroll
    for (int rb = 0; rb < RB; ++rb) { Ta_prev[rb] = 0.0; Ta[rb] = 1.0; Tb_prev[rb] = 0.0; Tb[rb] = 1.0; }
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
        const double *cb = lds + (sb & 1) * SLAB + ocl * N4 * LDB;
        double F[RB];
#pragma unroll
        for (int rb = 0; rb < RB; ++rb) F[rb] = (D == 2) ? 1.0 : (D == 3 ? Ta[rb] : Ta[rb] * Tb[rb]);
        // B fragments one K-step ahead of the MFMAs that use them
        double bf[2][NCB];
#pragma unroll
        for (int c = 0; c < NCB; ++c) bf[0][c] = cb[kq * LDB + c * 16 + r16];
#pragma unroll
        for (int t = 0; t < N4 / 4; ++t) {
            if (t + 1 < N4 / 4) {
#pragma unroll
                for (int c = 0; c < NCB; ++c) bf[(t + 1) & 1][c] = cb[(4 * (t + 1) + kq) * LDB + c * 16 + r16];
            }
#pragma unroll
            for (int rb = 0; rb < RB; ++rb) {
                const double a = F[rb] * Tl[rb][t];
#pragma unroll
                for (int c = 0; c < NCB; ++c)
                    acc[rb][c] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, bf[t & 1][c], acc[rb][c], 0, 0, 0);
            }
        }
        // advance the outer-mode recurrences T_{k+1} = 2 x T_k - T_{k-1}
        if (D == 3) {
#pragma unroll
            for (int rb = 0; rb < RB; ++rb) {
                const double tn = (oc == 0) ? xo[rb][0] : 2.0 * xo[rb][0] * Ta[rb] - Ta_prev[rb];
                Ta_prev[rb] = Ta[rb]; Ta[rb] = tn;
            }
        } else if (D == 4) {
            const int kb = oc % N;
            if (kb == N - 1) {
                const int ka = oc / N;
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
        if (more) store_slab(lds + ((sb + 1) & 1) * SLAB);
        __syncthreads();
    }

    // ---- rows to W: element v of lane c + 16 kq is row kq + 4 v ----
    double *Wp = Wout + (long long)player * NN * NC;
#pragma unroll
    for (int rb = 0; rb < RB; ++rb)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int j = row0 + rb * 16 + kq + 4 * v;
            if (j < NN) {
#pragma unroll
                for (int c = 0; c < NCB; ++c) Wp[(long long)j * NC + c * 16 + r16] = acc[rb][c][v];
            }
        }
}

// End of a step: record its residual r, test convergence and finiteness,
// flip the state buffers.
__device__ void finish_step(const GameConst *__restrict__ gc, GameStatus *st, int cur, double r)
{
    st->steps_done += 1;
    st->total_steps += 1;
    st->last_res = r;
    if (!(r <= 1.7976931348623157e308)) {
        st->nonfinite = 1;
        st->converged = 1;
    } else if (gc->tol > 0.0 && r < gc->tol) {
        st->converged = 1;
    }
    st->cur = 1 - cur;
}

// ---------------------------------------------------------------------------
// Line kernel: Steps 2-4 at every (player, node) from the line coefficients
// W[i][j][0..NC): fit in u, argmax, new value and control, residual.
// COMPOSE (control nodes >= N): one thread per row computes the fit
// coefficients directly (line_compose).  Otherwise two threads share a row:
// each samples half of the control nodes, and the partial fits are summed
// through LDS.
template <int D, int N4, int NC, bool COMPOSE>
__global__ __launch_bounds__(COMPOSE ? 64 : 256) void k_line_f64(const Inst *__restrict__ tab, int bpi,
                                                                  int blocks_per_player)
{
    const InstView I = inst_view(tab, blockIdx.x / bpi);
    const int blk = blockIdx.x % bpi;
    const GameConst *__restrict__ gc = I.gc;
    GameStatus *st = I.st;
    double *Vbuf = I.V, *Ubuf = I.U;
    const double *__restrict__ Win = I.W;
    // one wave per block when a thread owns a row: the few waves of a step
    // spread evenly over the SIMDs
    constexpr int TPR = COMPOSE ? 1 : 2;
    constexpr int BT = COMPOSE ? 64 : 256;
    constexpr int ROWS_B = BT / TPR;
    constexpr int NWB = BT / 64;
    __shared__ double Qx[COMPOSE ? 1 : N4 * ROWS_B];
    __shared__ double red[NWB];

    if (st->converged) return;
    const int cur = st->cur;
    const int NN = (int)gc->NN;
    const double *Vold = Vbuf + (long long)cur * D * NN;
    const double *Uold = Ubuf + (long long)cur * D * NN;
    double *Vnew = Vbuf + (long long)(1 - cur) * D * NN;
    double *Unew = Ubuf + (long long)(1 - cur) * D * NN;

    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int player = blk / blocks_per_player;
    const int tile = blk % blocks_per_player;
    const int row = tid % ROWS_B;
    const int part = tid / ROWS_B;
    const int j = tile * ROWS_B + row;
    const int jc = j < NN ? j : NN - 1;

    double w[N4];
    const double2 *wr = reinterpret_cast<const double2 *>(Win + ((long long)player * NN + jc) * NC);
#pragma unroll
    for (int k = 0; k < N4 / 2; ++k) {
        const double2 t = wr[k];
        w[2 * k] = t.x;
        w[2 * k + 1] = t.y;
    }
    double p[D], ub[D], b[D];
    node_state<D>(gc, Uold, jc, p, ub, b);
    double q[N4];
    const double s0 = 2.0 * ub[player] / gc->umax - 1.0;  // Newton's start: the current control
    bool direct = false;
    double vd = 0.0, sd = 0.0;
    if constexpr (COMPOSE) {
        // certified concave lines skip the series in s
        direct = line_argmax_direct<D, N4>(gc, player, p, ub, b, w, s0, vd, sd);
        if (!direct) line_compose<D, N4>(gc, player, p, ub, b, w, q);
    } else {
        line_fit_regs<D, N4, N4>(gc, player, p, ub, b, w, part, 2, q);
        if (part == 1) {
#pragma unroll
            for (int l = 0; l < N4; ++l) Qx[l * ROWS_B + row] = q[l];
        }
        __syncthreads();
        if (part == 0) {
#pragma unroll
            for (int l = 0; l < N4; ++l) q[l] += Qx[l * ROWS_B + row];
        }
    }
    double resmax = 0.0;
    if (part == 0 && j < NN) {
        double s = sd;
        const double vn = direct ? vd : line_argmax(q, gc->Nu, s0, s);
        const double un = 0.5 * gc->umax * (s + 1.0);
        const long long o = (long long)player * NN + j;
        Vnew[o] = vn;
        Unew[o] = un;
        resmax = fabs(vn - Vold[o]);  // a NaN stays NaN and wins the bitwise max below
    }
    unsigned long long bits = __double_as_longlong(resmax);
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        const unsigned long long o = __shfl_xor(bits, off);
        bits = o > bits ? o : bits;
    }
    if (lane == 0) red[wave] = __longlong_as_double(bits);
    __syncthreads();
    if (tid == 0) {  // this block's maximum; k_finish reduces them (no same-address atomics)
        unsigned long long m = 0;
        for (int w2 = 0; w2 < NWB; ++w2) {
            const unsigned long long x = __double_as_longlong(red[w2]);
            m = x > m ? x : m;
        }
        I.blk[blk] = __longlong_as_double(m);
    }
}

// End of an iteration, one block per instance: the residual is the bitwise
// maximum of the line kernel's per-block maxima (non-negative doubles order as
// their bit patterns, and a NaN's bits exceed every finite value's), then the
// status bookkeeping.
__global__ __launch_bounds__(256) void k_finish(const Inst *__restrict__ tab, int nblk)
{
    const InstView I = inst_view(tab, blockIdx.x);
    GameStatus *st = I.st;
    __shared__ unsigned long long red[4];
    if (st->converged) return;
    const int tid = threadIdx.x;
    unsigned long long m = 0;
#pragma unroll 8
    for (int k = tid; k < nblk; k += 256) {  // eight loads in flight per thread
        const unsigned long long x = __double_as_longlong(I.blk[k]);
        m = x > m ? x : m;
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        const unsigned long long o = __shfl_xor(m, off);
        m = o > m ? o : m;
    }
    if ((tid & 63) == 0) red[tid >> 6] = m;
    __syncthreads();
    if (tid == 0) {
        m = red[0];
#pragma unroll
        for (int w = 1; w < 4; ++w) m = red[w] > m ? red[w] : m;
        finish_step(I.gc, st, st->cur, __longlong_as_double(m));
    }
}

template <int D, int N4, int RB>
static hipError_t launch_contract_dnr(const GameConst &hc, const StepBuffers &b, hipStream_t s)
{
    constexpr int NC = N4 <= 16 ? 16 : 32;
    const int NN = (int)hc.NN;
    const int bpp = (NN + 4 * RB * 16 - 1) / (4 * RB * 16);
    const int bpi = bpp * D;
    if (D >= 3 && b.ocb == 2)
        hipLaunchKernelGGL((k_contract_f64<D, N4, NC, RB, D >= 3 ? 2 : 1>), dim3((unsigned)(bpi * b.count)), dim3(256),
                           0, s, b.tab, bpi, bpp);
    else
        hipLaunchKernelGGL((k_contract_f64<D, N4, NC, RB, 1>), dim3((unsigned)(bpi * b.count)), dim3(256), 0, s,
                           b.tab, bpi, bpp);
    return hipGetLastError();
}

template <int D, int N4>
static hipError_t launch_step_dn(const GameConst &hc, const StepBuffers &b, hipStream_t s)
{
    constexpr int NC = N4 <= 16 ? 16 : 32;
    const int NN = (int)hc.NN;
    hipError_t e;
    if (b.ev_begin) {
        e = hipEventRecord(b.ev_begin, s);
        if (e != hipSuccess) return e;
    }
    if (b.precision == CG_FP32_CORR) {
        e = launch_contract_corr(hc, b, s);
    } else {
        switch (b.rb) {
            case 1: e = launch_contract_dnr<D, N4, 1>(hc, b, s); break;
            case 4: e = launch_contract_dnr<D, N4, 4>(hc, b, s); break;
            default: e = launch_contract_dnr<D, N4, 2>(hc, b, s); break;
        }
    }
    if (e != hipSuccess) return e;
    if (b.ev_end) {
        e = hipEventRecord(b.ev_end, s);
        if (e != hipSuccess) return e;
    }
    if (hc.Nu >= hc.N) {  // the fit in u is exact: compose the series directly
        const int lpp = (NN + 63) / 64;
        const int bpi = lpp * D;
        hipLaunchKernelGGL((k_line_f64<D, N4, NC, true>), dim3((unsigned)(bpi * b.count)), dim3(64), 0, s, b.tab,
                           bpi, lpp);
        e = hipGetLastError();
        if (e == hipSuccess) hipLaunchKernelGGL(k_finish, dim3((unsigned)b.count), dim3(256), 0, s, b.tab, bpi);
    } else {
        const int lpp = (NN + 127) / 128;
        const int bpi = lpp * D;
        hipLaunchKernelGGL((k_line_f64<D, N4, NC, false>), dim3((unsigned)(bpi * b.count)), dim3(256), 0, s, b.tab,
                           bpi, lpp);
        e = hipGetLastError();
        if (e == hipSuccess) hipLaunchKernelGGL(k_finish, dim3((unsigned)b.count), dim3(256), 0, s, b.tab, bpi);
    }
    return hipGetLastError();
}

template <int D>
static hipError_t launch_step_d(const GameConst &hc, const StepBuffers &b, hipStream_t s)
{
    switch (hc.N4) {
        case 4: return launch_step_dn<D, 4>(hc, b, s);
        case 8: return launch_step_dn<D, 8>(hc, b, s);
        case 12: return launch_step_dn<D, 12>(hc, b, s);
        case 16: return launch_step_dn<D, 16>(hc, b, s);
        case 20: return launch_step_dn<D, 20>(hc, b, s);
        case 24: return launch_step_dn<D, 24>(hc, b, s);
        case 28: return launch_step_dn<D, 28>(hc, b, s);
        case 32: return launch_step_dn<D, 32>(hc, b, s);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_step(const GameConst &hc, const StepBuffers &b, hipStream_t s)
{
    // 1. coefficients of every V_i (Algorithm Cnv) into the packed operand;
    //    the mixed path computes its Taylor tensors in the first pass's launch
    hipError_t e = b.precision == CG_FP32_CORR ? launch_tf_taylor(hc, b, s) : launch_transform_game(hc, b, s);
    if (e == hipSuccess && b.precision == CG_FP32_CORR) e = launch_transform_rest(hc, b, s);
    if (e != hipSuccess) return e;
    // 2. contraction (MFMA), then line fit + argmax + residual + bookkeeping
    switch (hc.d) {
        case 2: e = launch_step_d<2>(hc, b, s); break;
        case 3: e = launch_step_d<3>(hc, b, s); break;
        case 4: e = launch_step_d<4>(hc, b, s); break;
        default: return hipErrorInvalidValue;
    }
    return e;
}

}  // namespace cg
