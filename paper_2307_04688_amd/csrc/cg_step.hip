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
// residual) is per-row work fused after the contraction, so W_i never
// reaches HBM.
#include "cg_line.h"

namespace cg {

// ---------------------------------------------------------------------------
// Packed contraction operand: Bp[i][kidx][col], kidx enumerating the modes
// l != i in increasing order with the last of them padded to N4 (zeros), col
// = k_i padded to NC (zeros).  Written from the natural-layout coefficients.
__global__ __launch_bounds__(256) void k_pack_B(const GameConst *__restrict__ gc, const GameStatus *st,
                                                const double *__restrict__ coef, double *__restrict__ Bp)
{
    if (st->converged) return;
    const int d = gc->d, N = gc->N, N4 = gc->N4, NC = gc->NC, K = gc->K;
    const long long per = (long long)K * NC;
    const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= per * d) return;
    const int i = (int)(e / per);
    const int rem = (int)(e % per);
    const int col = rem % NC;
    int kidx = rem / NC;
    const int klast = kidx % N4;
    kidx /= N4;
    double v = 0.0;
    if (klast < N && col < N) {
        // rebuild the multi-index: others in increasing order, last = klast
        const int lastmode = (i == d - 1) ? d - 2 : d - 1;
        int off = 0, mul = 1;
        for (int l = d - 1; l >= 0; --l) {
            int k;
            if (l == i) k = col;
            else if (l == lastmode) k = klast;
            else { k = kidx % N; kidx /= N; }
            off += k * mul;
            mul *= N;
        }
        v = coef[(long long)i * gc->NN + off];
    }
    Bp[e] = v;
}

// ---------------------------------------------------------------------------
// Fused step kernel, FP64.  Block = 4 waves; wave w owns RB row blocks of 16
// nodes of one player.  Lane layout of v_mfma_f64_16x16x4f64: A[r][k] and
// B[k][c] come from lane r + 16 k (resp. c + 16 k); D[g + 4 v][c] sits in
// lane c + 16 g, element v (rows interleaved by 4, unlike the f32 forms).
template <int D, int N4, int NC, int RB>
__global__ __launch_bounds__(256) void k_step_f64(const GameConst *__restrict__ gc, GameStatus *st,
                                                  double *Vbuf, double *Ubuf, const double *__restrict__ Bp,
                                                  int blocks_per_player)
{
    constexpr int NCB = NC / 16;
    constexpr int ROWS_W = RB * 16;
    constexpr int ROWS_B = 4 * ROWS_W;
    constexpr int LDW = NC + 1;
    __shared__ double Wl[ROWS_B * LDW];
    __shared__ double red[4];

    if (st->converged) return;
    const int cur = st->cur;
    const int NN = (int)gc->NN;
    const int N = gc->N;
    const double *Vold = Vbuf + (long long)cur * D * NN;
    const double *Uold = Ubuf + (long long)cur * D * NN;
    double *Vnew = Vbuf + (long long)(1 - cur) * D * NN;
    double *Unew = Ubuf + (long long)(1 - cur) * D * NN;

    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int r16 = lane & 15, kq = lane >> 4;
    const int player = blockIdx.x / blocks_per_player;
    const int tile = blockIdx.x % blocks_per_player;
    const int row0 = tile * ROWS_B + wave * ROWS_W;

    // other modes in increasing order
    int om[D - 1];
#pragma unroll
    for (int t = 0; t < D - 1; ++t) om[t] = t < player ? t : t + 1;

    // ---- prologue: shifted coordinates and basis values of each row ----
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
        double tm1 = 1.0, t0 = xl;  // T_0, T_1
#pragma unroll
        for (int k = 0; k < N4; ++k) {
            double tk;
            if (k == 0) tk = 1.0;
            else if (k == 1) tk = xl;
            else { tk = 2.0 * xl * t0 - tm1; tm1 = t0; t0 = tk; }
            if ((k & 3) == kq) Tl[rb][k >> 2] = tk;
        }
    }

    // ---- contraction on MFMA ----
    f64x4 acc[RB][NCB];
#pragma unroll
    for (int rb = 0; rb < RB; ++rb)
#pragma unroll
        for (int c = 0; c < NCB; ++c) acc[rb][c] = f64x4{0.0, 0.0, 0.0, 0.0};

    const double *B = Bp + (long long)player * gc->K * NC;
    // outer modes: D == 3 -> om[0]; D == 4 -> om[0] (slow), om[1] (fast)
    double Ta_prev[RB], Ta[RB], Tb_prev[RB], Tb[RB];
#pragma unroll
    for (int rb = 0; rb < RB; ++rb) { Ta_prev[rb] = 0.0; Ta[rb] = 1.0; Tb_prev[rb] = 0.0; Tb[rb] = 1.0; }
    const int n_outer = (D == 2) ? 1 : (D == 3 ? N : N * N);
    for (int oc = 0; oc < n_outer; ++oc) {
        double F[RB];
#pragma unroll
        for (int rb = 0; rb < RB; ++rb) F[rb] = (D == 2) ? 1.0 : (D == 3 ? Ta[rb] : Ta[rb] * Tb[rb]);
        const double *Brow = B + (long long)oc * N4 * NC + kq * NC + r16;
#pragma unroll
        for (int t = 0; t < N4 / 4; ++t) {
            double bf[NCB];
#pragma unroll
            for (int c = 0; c < NCB; ++c) bf[c] = Brow[t * 4 * NC + c * 16];
#pragma unroll
            for (int rb = 0; rb < RB; ++rb) {
                const double a = F[rb] * Tl[rb][t];
#pragma unroll
                for (int c = 0; c < NCB; ++c)
                    acc[rb][c] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, bf[c], acc[rb][c], 0, 0, 0);
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

    // ---- accumulators to LDS: row-major [row][col] per block ----
#pragma unroll
    for (int rb = 0; rb < RB; ++rb)
#pragma unroll
        for (int c = 0; c < NCB; ++c)
#pragma unroll
            for (int v = 0; v < 4; ++v)
                Wl[(wave * ROWS_W + rb * 16 + kq + 4 * v) * LDW + c * 16 + r16] = acc[rb][c][v];
    __syncthreads();

    // ---- epilogue: one thread per (player, node) ----
    double resmax = 0.0;
    for (int row = tid; row < ROWS_B; row += 256) {
        const int j = tile * ROWS_B + row;
        if (j >= NN) continue;
        double w[N4];
#pragma unroll
        for (int k = 0; k < N4; ++k) w[k] = Wl[row * LDW + k];
        double p[D], ub[D], b[D];
        node_state<D>(gc, Uold, j, p, ub, b);
        double vn, un;
        line_update<D, N4>(gc, player, p, ub, b, w, vn, un);
        const long long o = (long long)player * NN + j;
        Vnew[o] = vn;
        Unew[o] = un;
        const double e = fabs(vn - Vold[o]);
        resmax = (e > resmax || e != e) ? e : resmax;
    }
    // block max of the residual; NaN propagates as the largest bit pattern
    unsigned long long bits = __double_as_longlong(resmax);
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        const unsigned long long o = __shfl_xor(bits, off);
        bits = o > bits ? o : bits;
    }
    if (lane == 0) red[wave] = __longlong_as_double(bits);
    __syncthreads();
    if (tid == 0) {
        unsigned long long m = 0;
        for (int w = 0; w < 4; ++w) {
            const unsigned long long x = __double_as_longlong(red[w]);
            m = x > m ? x : m;
        }
        atomicMax(&st->res_bits[cur], m);
    }
}

// End of a step: record the residual, test convergence and finiteness, flip
// the state buffers, clear the next residual slot.
__global__ void k_finish(const GameConst *__restrict__ gc, GameStatus *st)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    if (st->converged) return;
    const int cur = st->cur;
    const double r = __longlong_as_double(st->res_bits[cur]);
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
    st->res_bits[1 - cur] = 0ull;
}

// ---------------------------------------------------------------------------
template <int D, int N4>
static hipError_t launch_step_dn(const GameConst &hc, const StepBuffers &b, hipStream_t s)
{
    constexpr int NC = N4 <= 16 ? 16 : 32;
    // 32 rows per wave for large grids (fills the chip evenly), 16 otherwise
    const int NN = (int)hc.NN;
    constexpr int RB = 2;
    const int rows_b = 4 * RB * 16;
    const int bpp = (NN + rows_b - 1) / rows_b;
    hipLaunchKernelGGL((k_step_f64<D, N4, NC, RB>), dim3(bpp * D), dim3(256), 0, s, b.gc, b.status, b.V,
                       b.U, b.Bp, bpp);
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
    // 1. coefficients of every V_i (Algorithm Cnv), natural layout
    hipError_t e = launch_transform_game(hc, b, s);
    if (e != hipSuccess) return e;
    // 2. packed operand
    {
        const long long total = (long long)hc.d * hc.K * hc.NC;
        const int threads = 256;
        hipLaunchKernelGGL(k_pack_B, dim3((unsigned)((total + threads - 1) / threads)), dim3(threads), 0, s,
                           b.gc, b.status, b.coef, b.Bp);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    // 3. fused contraction + line update + residual
    if (b.ev_begin) {
        e = hipEventRecord(b.ev_begin, s);
        if (e != hipSuccess) return e;
    }
    switch (hc.d) {
        case 2: e = launch_step_d<2>(hc, b, s); break;
        case 3: e = launch_step_d<3>(hc, b, s); break;
        case 4: e = launch_step_d<4>(hc, b, s); break;
        default: return hipErrorInvalidValue;
    }
    if (e != hipSuccess) return e;
    if (b.ev_end) {
        e = hipEventRecord(b.ev_end, s);
        if (e != hipSuccess) return e;
    }
    // 4. bookkeeping
    hipLaunchKernelGGL(k_finish, dim3(1), dim3(64), 0, s, b.gc, b.status);
    return hipGetLastError();
}

}  // namespace cg
