// cg_general.hip -- the general form of the value iteration: Section 2.1's
// algorithm for dynamics that are not separable in the controls, with the
// node-wise control polynomials of Section 3.3 (interpolated once, Step 0 of
// Section 3.4) and anisotropic state and control grids.
//
// One iteration, for every player i and state node p_j:
//   transform   coefficients of every V_i^{[r]} (Algorithm Cnv, per mode:
//               the two fastest modes of each slice in one launch, the
//               others in a second that writes the evaluation operand)
//   points      Step 1: the control polynomials of node j are contracted over
//               the modes of the other players at their current controls
//               (the per-node evaluation of Section 3.3), leaving series in
//               u_i that are summed at player i's control nodes; the result
//               gives the update points p_j + h g(p_j, [u_m, u_{-i}]) and the
//               payoff samples.  A 16-lane group per (node, player), one
//               wave per player over four nodes; a block holds whole nodes
//               (the coefficients are stored node-major), so each node's
//               coefficients are read from HBM once and shared through the
//               caches.
//   evaluation  Step 2: V_i^{[r]} at every update point, all players in one
//               launch: the scattered-point evaluation (Khatri-Rao GEMM on
//               FP64 MFMA + Clenshaw).
//   line        Steps 3-4: fit of the samples in u (DCT-I), argmax on
//               [0, u_max], new value and control, per-block residual maxima.
//   finish      residual, TOL test, status.
#include <math.h>
#include <stdarg.h>
#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include <new>
#include <vector>

#include "cg_internal.h"
#include "cg_line.h"

namespace {

using namespace cg;

constexpr int kMaxNu = CG_MAX_NU;

struct GenConst {
    int d;
    int np[kMaxD], nu[kMaxD];
    int ustride[kMaxD];                  // stride of control mode l in a control tensor
    long long NP, UP, NPT;               // state nodes, control nodes, update points
    long long off[kMaxD];                // first update point of player i: NP sum_{l<i} nu[l]
    double h, rho, pmax, umax, delta;
    double uinit[kMaxD];
    double pnode[kMaxD][kMaxN];          // physical state nodes p_max (x_k + 1) / 2
    double tnode[kMaxD][kMaxNu];         // normalised control nodes cos(pi m / (nu - 1))
    double Du[kMaxD][kMaxNu * kMaxNu];   // DCT-I of the fit in u, [l][m], zero-padded
    double Dp[kMaxD][kMaxN * kMaxN];     // DCT-I of state mode l, [l'][k] (np[l] x np[l])
};

struct GenStatus {
    double last_res;
    double tol;
    int converged, steps_done, nonfinite, total_steps;
};

inline size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

struct GenLayout {
    size_t gc, st, V, U, coef, cc, pts, psamp, ev, blk, evws, evws_bytes, total;
};

__global__ void k_gen_init(const GenConst *__restrict__ gc, GenStatus *st, double *V, double *U)
{
    const long long n = (long long)gc->d * gc->NP;
    for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < n;
         e += (long long)gridDim.x * blockDim.x) {
        V[e] = 0.0;
        U[e] = gc->uinit[(int)(e / gc->NP)];
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        st->last_res = 0.0;
        st->tol = 0.0;
        st->converged = 0;
        st->steps_done = 0;
        st->nonfinite = 0;
        st->total_steps = 0;
    }
}

__global__ void k_gen_arm(GenStatus *st, double tol, int clear_done)
{
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        st->tol = tol;
        st->converged = 0;
        st->nonfinite = 0;
        if (clear_done) st->steps_done = 0;
    }
}

// Sum over the 16 lanes of a DPP row (a 16-lane group), returned in every
// lane of the row: pairs and quads by quad permutations, then rotations of
// the row by 4 and 8 lanes (VALU data movement, no LDS traffic).  The last
// two steps add the four quad sums in an order that depends on the quad, so
// lanes may differ in the last bit; each is deterministic.
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v)
{
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffffLL), CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xF, 0xF, false);
    return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}

__device__ __forceinline__ double row16_sum(double v)
{
    v += dpp_f64<0xB1>(v);   // quad_perm [1,0,3,2]
    v += dpp_f64<0x4E>(v);   // quad_perm [2,3,0,1]
    v += dpp_f64<0x124>(v);  // row_ror:4
    v += dpp_f64<0x128>(v);  // row_ror:8
    return v;
}

// Step 1 for the (node, player) pairs of NB = 4 consecutive nodes: wave i of
// the block serves player i and its four 16-lane groups the four nodes, so
// the D players of a node share the node's drift coefficients (one
// contiguous block per node in the node-major layout) through the caches,
// and every branch on the player is uniform over a wave.  NUM >= every
// n_unodes, a multiple of 4 (register arrays stay compile-time sized).
//
// Players i < D - 1: each lane contracts a strided share of the outer control
// indices o (the other modes in C order, the last mode fastest, so that
// neighbouring lanes read neighbouring coefficients) for every coefficient a
// of the series in u_i; the 16 partial sums of each are combined by
// row16_sum; one outer index at a time, with at most 128 VGPRs when the
// (D + 1) NUM accumulators allow it: four waves per SIMD hide more of the
// load latency than a deeper unroll at three (measured 74.6 against 80.1 us
// at d = 3, n_u = 8).  Player D - 1, whose mode has stride 1 in a control tensor:
// lane s n_u + a keeps coefficient a and every S-th index of mode D - 2
// (S = 16 / n_u slices; with n_u even, two neighbouring coefficients per lane
// and one 16-byte load), so that the lanes of a group read one contiguous run
// per load; the S slice sums meet in LDS.
template <int D, int NUM>
__global__ __launch_bounds__(64 * D) __attribute__((amdgpu_waves_per_eu((D + 1) * NUM <= 32 ? 4 : 1)))
void k_gen_points(const GenConst *__restrict__ gc, const GenStatus *__restrict__ st, const double *__restrict__ U,
                  const double *__restrict__ cc, double *__restrict__ pts, double *__restrict__ psamp)
{
    constexpr int L = 16, NB = 4;
    __shared__ double Tb[NB][D][NUM];
    __shared__ double Sb[NB][D + 1][2 * L];
    if (st->converged) return;  // the same for every thread, before any barrier
    const int tid = threadIdx.x, i = tid / 64, g = (tid % 64) / L, lane = tid % L;
    const long long NP = gc->NP, UP = gc->UP;
    const long long j0 = (long long)blockIdx.x * NB;
    // T_a(y_l) at the nodes' current controls, y_l = 2 u_l / u_max - 1
    for (int t = tid; t < NB * D * NUM; t += 64 * D) {
        const int n = t / (D * NUM), l = (t / NUM) % D, a = t % NUM;
        const long long jn = j0 + n < NP ? j0 + n : NP - 1;
        const double y = 2.0 * U[l * NP + jn] / gc->umax - 1.0;
        double tm1 = 1.0, t0 = y, ta = a == 0 ? 1.0 : y;
        for (int k = 2; k <= a; ++k) {
            ta = 2.0 * y * t0 - tm1;
            tm1 = t0;
            t0 = ta;
        }
        Tb[n][l][a] = ta;
    }
    __syncthreads();
    const long long j = j0 + g;
    const bool active = j < NP;
    const int nui = gc->nu[i];
    double acc[D + 1][NUM];
#pragma unroll
    for (int k = 0; k <= D; ++k)
#pragma unroll
        for (int a = 0; a < NUM; ++a) acc[k][a] = 0.0;
    const double *gbase = cc + (active ? j : 0) * (2 * D) * UP;  // drift component k at + k UP
    const double *pbase = gbase + (D + i) * UP;                   // payoff of player i
    if (i < D - 1) {
        if (active) {
            const int si = gc->ustride[i];
            const int nouter = (int)(UP / nui);
            // The loads of one outer index are issued together: no
            // data-dependent branch between them (entries a >= nui read a
            // valid address, entry nui - 1, and are weighted by zero).
#pragma unroll 1
            for (int o = lane; o < nouter; o += L) {
                int rem = o, base = 0;
                double w = 1.0;
#pragma unroll
                for (int l = D - 1; l >= 0; --l) {
                    if (l == i) continue;
                    const int a = rem % gc->nu[l];
                    rem /= gc->nu[l];
                    base += a * gc->ustride[l];
                    w *= Tb[g][l][a];
                }
                double v[D + 1][NUM];
#pragma unroll
                for (int a = 0; a < NUM; ++a) {
                    const int off = base + (a < nui ? a : nui - 1) * si;
#pragma unroll
                    for (int k = 0; k < D; ++k) v[k][a] = gbase[k * UP + off];
                    v[D][a] = pbase[off];
                }
#pragma unroll
                for (int a = 0; a < NUM; ++a) {
                    const double wa = a < nui ? w : 0.0;
#pragma unroll
                    for (int k = 0; k <= D; ++k) acc[k][a] = fma(v[k][a], wa, acc[k][a]);
                }
            }
#pragma unroll
            for (int a = 0; a < NUM; ++a) {
                if (a < nui) {
#pragma unroll
                    for (int k = 0; k <= D; ++k) acc[k][a] = row16_sum(acc[k][a]);
                }
            }
        }
    } else if ((nui & 1) == 0) {
        // even n_u: lane s (n_u / 2) + c keeps coefficients 2c and 2c + 1
        // (one 16-byte load per function; S = 32 / n_u slices)
        const int hw = nui / 2, S = L / hw, a = 2 * (lane % hw), slice = lane / hw;
        double part[D + 1][2];
#pragma unroll
        for (int k = 0; k <= D; ++k) part[k][0] = part[k][1] = 0.0;
        if (active && slice < S) {
            const int nin = gc->nu[D - 2];                        // the mode split over slices
            const int nhi = (int)(UP / ((long long)nin * nui));   // modes 0 .. D-3
            for (int hi = 0; hi < nhi; ++hi) {
                int rem = hi;
                double wh = 1.0;
#pragma unroll
                for (int l = D - 3; l >= 0; --l) {
                    const int al = rem % gc->nu[l];
                    rem /= gc->nu[l];
                    wh *= Tb[g][l][al];
                }
                const int row = hi * nin;
#pragma unroll 2
                for (int b = slice; b < nin; b += S) {
                    const double w = wh * Tb[g][D - 2][b];
                    const int off = (row + b) * nui + a;   // even: 16-byte aligned
                    double2 v[D + 1];
#pragma unroll
                    for (int k = 0; k < D; ++k) v[k] = *(const double2 *)(gbase + k * UP + off);
                    v[D] = *(const double2 *)(pbase + off);
#pragma unroll
                    for (int k = 0; k <= D; ++k) {
                        part[k][0] = fma(v[k].x, w, part[k][0]);
                        part[k][1] = fma(v[k].y, w, part[k][1]);
                    }
                }
            }
        }
#pragma unroll
        for (int k = 0; k <= D; ++k) {
            Sb[g][k][2 * lane] = part[k][0];
            Sb[g][k][2 * lane + 1] = part[k][1];
        }
    } else {
        const int S = L / nui, a = lane % nui, slice = lane / nui;
        double part[D + 1];
#pragma unroll
        for (int k = 0; k <= D; ++k) part[k] = 0.0;
        if (active && slice < S) {
            const int nin = gc->nu[D - 2];                        // the mode split over slices
            const int nhi = (int)(UP / ((long long)nin * nui));   // modes 0 .. D-3
            for (int hi = 0; hi < nhi; ++hi) {
                int rem = hi;
                double wh = 1.0;
#pragma unroll
                for (int l = D - 3; l >= 0; --l) {
                    const int al = rem % gc->nu[l];
                    rem /= gc->nu[l];
                    wh *= Tb[g][l][al];
                }
                const int row = hi * nin;
#pragma unroll 2
                for (int b = slice; b < nin; b += S) {
                    const double w = wh * Tb[g][D - 2][b];
                    const int off = (row + b) * nui + a;
                    double v[D + 1];
#pragma unroll
                    for (int k = 0; k < D; ++k) v[k] = gbase[k * UP + off];
                    v[D] = pbase[off];
#pragma unroll
                    for (int k = 0; k <= D; ++k) part[k] = fma(v[k], w, part[k]);
                }
            }
        }
#pragma unroll
        for (int k = 0; k <= D; ++k) Sb[g][k][lane] = part[k];
    }
    __syncthreads();
    if (i == D - 1 && active) {
        // coefficient a of every series: the slice sums in slice order
        const int S = (nui & 1) ? L / nui : L / (nui / 2);
#pragma unroll
        for (int a = 0; a < NUM; ++a) {
            if (a < nui) {
#pragma unroll
                for (int k = 0; k <= D; ++k) {
                    double s = Sb[g][k][a];
                    for (int q = 1; q < S; ++q) s += Sb[g][k][q * nui + a];
                    acc[k][a] = s;
                }
            }
        }
    }
    if (active && lane < nui) {
        // lane m: control node u_m of player i; series in u_i by Clenshaw
        // (entries a >= nui are zero)
        const double t = gc->tnode[i][lane];
        double p[D];
        long long rem = j;
#pragma unroll
        for (int l = D - 1; l >= 0; --l) {
            const int k = (int)(rem % gc->np[l]);
            rem /= gc->np[l];
            p[l] = gc->pnode[l][k];
        }
        const long long q = gc->off[i] + j * nui + lane;
#pragma unroll
        for (int l = 0; l < D; ++l) {
            const double gl = clenshaw(acc[l], t);
            pts[q * D + l] = 2.0 * fma(gc->h, gl, p[l]) / gc->pmax - 1.0;
        }
        psamp[q] = gc->h * clenshaw(acc[D], t);
    }
}

// Coefficients of every V_i (Algorithm Cnv, Section 3.1: the DCT-I along
// each mode) on the anisotropic grid, written as the evaluation operand
// Bp_i[kidx][col] (kidx = (k_0 .. k_{d-3}) N4 + k_{d-2}, col = k_{d-1}; the
// padding entries stay zero from init), in two launches:
//   k_gen_tf_inner: one block per (player, position over modes 0 .. d-3): the
//     slice over the two fastest modes, both passes in LDS; for d = 2 the
//     slice is the whole tensor and goes straight to the operand, else to
//     the intermediate coefficient tensor;
//   k_gen_tf_outer (d >= 3): one block per (player, run of G positions over
//     the two fastest modes): the plane over modes 0 .. d-3 (one or two
//     modes), its passes in LDS, then the operand.
constexpr int kLd = kMaxN + 1;  // LDS row stride (doubles)

template <int D>
__global__ __launch_bounds__(256) void k_gen_tf_inner(const GenConst *__restrict__ gc,
                                                      const GenStatus *__restrict__ st,
                                                      const double *__restrict__ V, double *__restrict__ coef,
                                                      double *__restrict__ Bp, long long bp_stride, int N4, int NC)
{
    __shared__ double X[kMaxN * kLd], Y[kMaxN * kLd];
    __shared__ double Da[kMaxN * kMaxN], Db[kMaxN * kMaxN];
    if (st->converged) return;
    const int tid = threadIdx.x;
    const int na = gc->np[D - 2], nb = gc->np[D - 1];
    const int S = na * nb;
    const long long NP = gc->NP, nsl = NP / S;
    const int i = (int)(blockIdx.x / nsl);
    const long long o = blockIdx.x % nsl;
    const double *src = V + i * NP + o * S;
    for (int e = tid; e < na * na; e += 256) Da[e] = gc->Dp[D - 2][e];
    for (int e = tid; e < nb * nb; e += 256) Db[e] = gc->Dp[D - 1][e];
    for (int e = tid; e < S; e += 256) X[(e / nb) * kLd + e % nb] = src[e];
    __syncthreads();
    for (int e = tid; e < S; e += 256) {  // mode D-1
        const int a = e / nb, l = e % nb;
        double acc = 0.0;
        for (int k = 0; k < nb; ++k) acc = fma(Db[l * nb + k], X[a * kLd + k], acc);
        Y[a * kLd + l] = acc;
    }
    __syncthreads();
    for (int e = tid; e < S; e += 256) {  // mode D-2
        const int m = e / nb, l = e % nb;
        double acc = 0.0;
        for (int k = 0; k < na; ++k) acc = fma(Da[m * na + k], Y[k * kLd + l], acc);
        if (D == 2)
            Bp[i * bp_stride + (long long)m * NC + l] = acc;
        else
            coef[i * NP + o * S + e] = acc;
    }
}

template <int D>
__global__ __launch_bounds__(256) void k_gen_tf_outer(const GenConst *__restrict__ gc,
                                                      const GenStatus *__restrict__ st,
                                                      const double *__restrict__ coef, double *__restrict__ Bp,
                                                      long long bp_stride, int N4, int NC, int G)
{
    // the plane over modes 0 .. D-3 (n0, or n0 x n1) for G inner positions:
    // T[(p * G + g)], p the flattened outer index
    __shared__ double T0[kMaxN * kMaxN], T1[kMaxN * kMaxN];
    __shared__ double D0[kMaxN * kMaxN], D1[kMaxN * kMaxN];
    if (st->converged) return;
    const int tid = threadIdx.x;
    const int n0 = gc->np[0], n1 = D == 4 ? gc->np[1] : 1;
    const int na = gc->np[D - 2], nb = gc->np[D - 1];
    const int S = na * nb, P = n0 * n1;
    const long long NP = gc->NP;
    const int runs = (S + G - 1) / G;
    const int i = blockIdx.x / runs;
    const int e0 = (blockIdx.x % runs) * G;
    const int GP = G * P;
    for (int e = tid; e < n0 * n0; e += 256) D0[e] = gc->Dp[0][e];
    if (D == 4)
        for (int e = tid; e < n1 * n1; e += 256) D1[e] = gc->Dp[1][e];
    const double *src = coef + i * NP;
    for (int e = tid; e < GP; e += 256) {
        const int p = e / G, g = e % G;
        T0[e] = e0 + g < S ? src[(long long)p * S + e0 + g] : 0.0;
    }
    __syncthreads();
    double *cur = T0;
    if (D == 4) {  // mode 1: p = p0 n1 + p1
        for (int e = tid; e < GP; e += 256) {
            const int p = e / G, g = e % G, p0 = p / n1, l = p % n1;
            double acc = 0.0;
            for (int k = 0; k < n1; ++k) acc = fma(D1[l * n1 + k], T0[(p0 * n1 + k) * G + g], acc);
            T1[e] = acc;
        }
        __syncthreads();
        cur = T1;
    }
    double *nxt = D == 4 ? T0 : T1;
    for (int e = tid; e < GP; e += 256) {  // mode 0
        const int p = e / G, g = e % G, m = p / n1, r = p % n1;
        double acc = 0.0;
        for (int k = 0; k < n0; ++k) acc = fma(D0[m * n0 + k], cur[(k * n1 + r) * G + g], acc);
        nxt[e] = acc;
    }
    __syncthreads();
    for (int e = tid; e < GP; e += 256) {
        const int p = e / G, g = e % G, pos = e0 + g;
        if (pos < S) {
            const int ka = pos / nb, kb = pos % nb;
            Bp[i * bp_stride + ((long long)p * N4 + ka) * NC + kb] = nxt[e];
        }
    }
}

// Steps 3-4, one thread per (player, node).
__global__ __launch_bounds__(256) void k_gen_line(const GenConst *__restrict__ gc, const GenStatus *__restrict__ st,
                                                  double *__restrict__ V, double *__restrict__ U,
                                                  const double *__restrict__ psamp, const double *__restrict__ ev,
                                                  double *__restrict__ blk, int bpp)
{
    __shared__ unsigned long long red[4];
    if (st->converged) return;
    const int i = blockIdx.x / bpp;
    const long long j = (long long)(blockIdx.x % bpp) * 256 + threadIdx.x;
    const long long NP = gc->NP;
    const int nui = gc->nu[i];
    double resmax = 0.0;
    if (j < NP) {
        const long long base = gc->off[i] + j * nui;
        double smp[kMaxNu];
#pragma unroll
        for (int m = 0; m < kMaxNu; ++m) smp[m] = m < nui ? fma(gc->delta, ev[base + m], psamp[base + m]) : 0.0;
        double q[kMaxNu];
        const double *Dm = gc->Du[i];
#pragma unroll
        for (int l = 0; l < kMaxNu; ++l) {
            double a = 0.0;
#pragma unroll
            for (int m = 0; m < kMaxNu; ++m) a = fma(Dm[l * kMaxNu + m], smp[m], a);
            q[l] = a;
        }
        const long long o = (long long)i * NP + j;
        const double s0 = 2.0 * U[o] / gc->umax - 1.0;
        double s;
        const double vn = line_argmax(q, nui, s0, s);
        resmax = fabs(vn - V[o]);  // NaN stays NaN and wins the bitwise maximum
        V[o] = vn;
        U[o] = 0.5 * gc->umax * (s + 1.0);
    }
    unsigned long long bits = __double_as_longlong(resmax);
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        const unsigned long long x = __shfl_xor(bits, off);
        bits = x > bits ? x : bits;
    }
    const int wave = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) red[wave] = bits;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long m = 0;
        for (int w = 0; w < 4; ++w) m = red[w] > m ? red[w] : m;
        blk[blockIdx.x] = __longlong_as_double(m);
    }
}

__global__ __launch_bounds__(256) void k_gen_finish(GenStatus *st, const double *__restrict__ blk, int nblk)
{
    __shared__ unsigned long long red[256];
    if (st->converged) return;
    const int tid = threadIdx.x;
    unsigned long long m = 0;
    for (int k = tid; k < nblk; k += 256) {
        const unsigned long long x = __double_as_longlong(blk[k]);
        m = x > m ? x : m;
    }
    red[tid] = m;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (tid < w) red[tid] = red[tid + w] > red[tid] ? red[tid + w] : red[tid];
        __syncthreads();
    }
    if (tid == 0) {
        const double r = __longlong_as_double(red[0]);
        st->last_res = r;
        st->steps_done += 1;
        st->total_steps += 1;
        if (!(r <= 1.7976931348623157e308)) {
            st->nonfinite = 1;
            st->converged = 1;
        } else if (st->tol > 0.0 && r < st->tol) {
            st->converged = 1;
        }
    }
}

// Step 0 staging: the caller's samples drift[k][j][t] and payoff[i][j][t]
// into the node-major layout cc[j][0..d) (drift), cc[j][d..2d) (payoffs), so
// that everything Step 1 reads for one node is one contiguous block.
__global__ void k_gen_gather(double *cc, const double *drift, const double *payoff, int d, long long NP, long long UP,
                             long long n)
{
    for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < n;
         e += (long long)gridDim.x * blockDim.x) {
        const long long t = e % UP, r = e / UP, j = r % NP, k = r / NP;
        cc[(j * 2 * d + k) * UP + t] = drift[e];
        cc[(j * 2 * d + d + k) * UP + t] = payoff[e];
    }
}

__global__ void k_gen_copy(double *dst, const double *src, long long n)
{
    for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < n;
         e += (long long)gridDim.x * blockDim.x)
        dst[e] = src[e];
}

int gfail(int code, const char *fmt, ...) __attribute__((format(printf, 2, 3)));
int gfail(int code, const char *fmt, ...)
{
    char buf[400];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    return set_error(code, buf);
}

int hfail(hipError_t e, const char *where) { return gfail(CG_EDEVICE, "%s: %s", where, hipGetErrorString(e)); }

#define GEN_TRY(call, where)                      \
    do {                                          \
        hipError_t e_ = (call);                   \
        if (e_ != hipSuccess) return hfail(e_, where); \
    } while (0)

int validate_sizes(const cg_general_desc *g)
{
    if (!g) return gfail(CG_EINVAL, "desc is NULL");
    if (g->d < 2 || g->d > CG_MAX_D) return gfail(CG_EUNSUPPORTED, "d = %d outside [2, %d]", g->d, CG_MAX_D);
    double np = 1.0, up = 1.0;
    for (int l = 0; l < g->d; ++l) {
        if (g->n_nodes[l] < 3 || g->n_nodes[l] > CG_MAX_N)
            return gfail(CG_EUNSUPPORTED, "n_nodes[%d] = %d outside [3, %d]", l, g->n_nodes[l], CG_MAX_N);
        if (g->n_unodes[l] < 3 || g->n_unodes[l] > CG_MAX_NU)
            return gfail(CG_EUNSUPPORTED, "n_unodes[%d] = %d outside [3, %d]", l, g->n_unodes[l], CG_MAX_NU);
        np *= g->n_nodes[l];
        up *= g->n_unodes[l];
    }
    if (np * up > 1e12) return gfail(CG_EUNSUPPORTED, "N_P U_P = %.3g too large", np * up);
    if (!(g->p_max > 0.0) || !isfinite(g->p_max)) return gfail(CG_EINVAL, "p_max must be finite and > 0");
    if (!(g->u_max > 0.0) || !isfinite(g->u_max)) return gfail(CG_EINVAL, "u_max must be finite and > 0");
    return CG_OK;
}

int validate(const cg_general_desc *g)
{
    int rc = validate_sizes(g);
    if (rc != CG_OK) return rc;
    if (!(g->h > 0.0) || !isfinite(g->h)) return gfail(CG_EINVAL, "h must be finite and > 0");
    if (!(g->rho * g->h > 0.0 && g->rho * g->h < 1.0)) return gfail(CG_EINVAL, "need 0 < rho h < 1");
    for (int i = 0; i < g->d; ++i)
        if (!(g->u_init[i] >= 0.0 && g->u_init[i] <= g->u_max))
            return gfail(CG_EINVAL, "u_init[%d] outside [0, u_max]", i);
    if (!g->drift_dev || !g->payoff_dev) return gfail(CG_EINVAL, "drift_dev and payoff_dev are required");
    return CG_OK;
}

double cospi_frac(long long a, long long n)
{
    long long r = a % (2 * n);
    if (r < 0) r += 2 * n;
    return cos(M_PI * (double)r / (double)n);
}

void build_consts(const cg_general_desc *g, GenConst &c)
{
    memset(&c, 0, sizeof c);
    const int d = g->d;
    c.d = d;
    c.NP = 1;
    c.UP = 1;
    for (int l = 0; l < d; ++l) {
        c.np[l] = g->n_nodes[l];
        c.nu[l] = g->n_unodes[l];
        c.NP *= c.np[l];
        c.UP *= c.nu[l];
    }
    int st = 1;
    for (int l = d - 1; l >= 0; --l) {
        c.ustride[l] = st;
        st *= c.nu[l];
    }
    long long acc = 0;
    for (int i = 0; i < d; ++i) {
        c.off[i] = acc;
        acc += c.NP * c.nu[i];
    }
    c.NPT = acc;
    c.h = g->h;
    c.rho = g->rho;
    c.pmax = g->p_max;
    c.umax = g->u_max;
    c.delta = 1.0 - g->rho * g->h;
    for (int l = 0; l < d; ++l) {
        c.uinit[l] = g->u_init[l];
        const int n = c.np[l] - 1;
        for (int k = 0; k <= n; ++k) c.pnode[l][k] = 0.5 * g->p_max * (cospi_frac(k, n) + 1.0);
        const int nu = c.nu[l] - 1;
        for (int m = 0; m <= nu; ++m) c.tnode[l][m] = cospi_frac(m, nu);
        for (int a = 0; a <= nu; ++a)
            for (int m = 0; m <= nu; ++m) {
                double v = cospi_frac((long long)a * m, nu);
                if (m == 0 || m == nu) v *= 0.5;
                c.Du[l][a * kMaxNu + m] = v * ((a == 0 || a == nu) ? 1.0 : 2.0) / (double)nu;
            }
        for (int a = 0; a <= n; ++a)
            for (int k = 0; k <= n; ++k) {
                double v = cospi_frac((long long)a * k, n);
                if (k == 0 || k == n) v *= 0.5;
                c.Dp[l][a * (n + 1) + k] = v * ((a == 0 || a == n) ? 1.0 : 2.0) / (double)n;
            }
    }
}

GenLayout layout(const GenConst &c)
{
    GenLayout L;
    size_t o = 0;
    const size_t d = (size_t)c.d, NP = (size_t)c.NP, UP = (size_t)c.UP, NPT = (size_t)c.NPT;
    L.gc = o; o = align256(o + sizeof(GenConst));
    L.st = o; o = align256(o + sizeof(GenStatus));
    L.V = o; o = align256(o + sizeof(double) * d * NP);
    L.U = o; o = align256(o + sizeof(double) * d * NP);
    L.coef = o; o = align256(o + sizeof(double) * d * NP);
    L.cc = o; o = align256(o + sizeof(double) * 2 * d * NP * UP);
    L.pts = o; o = align256(o + sizeof(double) * NPT * d);
    L.psamp = o; o = align256(o + sizeof(double) * NPT);
    L.ev = o; o = align256(o + sizeof(double) * NPT);
    L.blk = o; o = align256(o + sizeof(double) * d * ((NP + 255) / 256));
    int n[CG_MAX_D];
    for (int l = 0; l < c.d; ++l) n[l] = c.np[l];
    L.evws_bytes = sizeof(double) * d * eval_packed_elems(c.d, n);  // one packed operand per player
    L.evws = o; o = align256(o + L.evws_bytes);
    L.total = o;
    return L;
}

}  // namespace

struct cg_general {
    GenConst hc;
    GenLayout L;
    hipStream_t stream;
    char *ws;
    EvalBatch bt;  // player i: packed operand i, its N_P n_u[i] update points
    bool prof = false;
    std::vector<hipEvent_t> evs;
    size_t ev_used = 0;
    long long timed = 0;

    template <typename T>
    T *at(size_t off) const { return (T *)(ws + off); }
};

namespace {

template <int D, int NUM>
hipError_t launch_points_n(const cg_general *g)
{
    // four nodes per block, one wave per player
    const long long blocks = (g->hc.NP + 3) / 4;
    hipLaunchKernelGGL((k_gen_points<D, NUM>), dim3((unsigned)blocks), dim3(64 * D), 0, g->stream,
                       g->at<GenConst>(g->L.gc), g->at<GenStatus>(g->L.st), g->at<double>(g->L.U),
                       g->at<double>(g->L.cc), g->at<double>(g->L.pts),
                       g->at<double>(g->L.psamp));
    return hipGetLastError();
}

int points_num(const GenConst &c)
{
    int mx = 0;
    for (int l = 0; l < c.d; ++l) mx = c.nu[l] > mx ? c.nu[l] : mx;
    return mx <= 4 ? 4 : mx <= 8 ? 8 : mx <= 12 ? 12 : 16;
}

template <int D>
hipError_t launch_points(const cg_general *g)
{
    switch (points_num(g->hc)) {
    case 4: return launch_points_n<D, 4>(g);
    case 8: return launch_points_n<D, 8>(g);
    case 12: return launch_points_n<D, 12>(g);
    default: return launch_points_n<D, 16>(g);
    }
}

// The transform of every V_i into the evaluation operands (two launches
// for d >= 3, one for d = 2).
template <int D>
hipError_t launch_gen_transform(const cg_general *g)
{
    const GenConst &c = g->hc;
    const int N4 = (c.np[D - 2] + 3) & ~3, NC = c.np[D - 1] <= 16 ? 16 : 32;
    const int S = c.np[D - 2] * c.np[D - 1];
    const long long nsl = c.NP / S;
    double *Bp = g->at<double>(g->L.evws);
    hipLaunchKernelGGL((k_gen_tf_inner<D>), dim3((unsigned)(D * nsl)), dim3(256), 0, g->stream,
                       g->at<GenConst>(g->L.gc), g->at<GenStatus>(g->L.st), g->at<double>(g->L.V),
                       g->at<double>(g->L.coef), Bp, g->bt.bp_stride, N4, NC);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || D == 2) return e;
    const int P = (int)nsl;               // positions over modes 0 .. D-3 (<= 1024)
    const int G = P >= 256 ? 1 : 256 / P;  // inner positions per block
    const int runs = (S + G - 1) / G;
    hipLaunchKernelGGL((k_gen_tf_outer<D>), dim3((unsigned)(D * runs)), dim3(256), 0, g->stream,
                       g->at<GenConst>(g->L.gc), g->at<GenStatus>(g->L.st), g->at<double>(g->L.coef), Bp,
                       g->bt.bp_stride, N4, NC, G);
    return hipGetLastError();
}

int record(cg_general *g, hipEvent_t *slot)
{
    if (!g->prof) return CG_OK;
    if (g->ev_used >= g->evs.size()) {
        for (int k = 0; k < 320; ++k) {
            hipEvent_t e;
            GEN_TRY(hipEventCreate(&e), "hipEventCreate");
            g->evs.push_back(e);
        }
    }
    *slot = g->evs[g->ev_used++];
    GEN_TRY(hipEventRecord(*slot, g->stream), "hipEventRecord");
    return CG_OK;
}

int queue_steps(cg_general *g, int nsteps)
{
    const GenConst &c = g->hc;
    const int d = c.d;
    int n[CG_MAX_D];
    for (int l = 0; l < d; ++l) n[l] = c.np[l];
    const int bpp = (int)((c.NP + 255) / 256);
    for (int s = 0; s < nsteps; ++s) {
        hipEvent_t ev;
        int rc = record(g, &ev);
        if (rc != CG_OK) return rc;
        GEN_TRY(d == 2 ? launch_gen_transform<2>(g) : d == 3 ? launch_gen_transform<3>(g)
                                                             : launch_gen_transform<4>(g),
                "transform");
        if ((rc = record(g, &ev)) != CG_OK) return rc;
        hipError_t e = d == 2 ? launch_points<2>(g) : d == 3 ? launch_points<3>(g) : launch_points<4>(g);
        GEN_TRY(e, "points launch");
        if ((rc = record(g, &ev)) != CG_OK) return rc;
        GEN_TRY(eval_f64_batch(d, n, g->at<double>(g->L.evws), g->at<double>(g->L.pts), g->at<double>(g->L.ev),
                               g->bt, d, g->stream),
                "eval launch");
        if ((rc = record(g, &ev)) != CG_OK) return rc;
        hipLaunchKernelGGL(k_gen_line, dim3((unsigned)(d * bpp)), dim3(256), 0, g->stream, g->at<GenConst>(g->L.gc),
                           g->at<GenStatus>(g->L.st), g->at<double>(g->L.V), g->at<double>(g->L.U),
                           g->at<double>(g->L.psamp), g->at<double>(g->L.ev), g->at<double>(g->L.blk), bpp);
        GEN_TRY(hipGetLastError(), "line launch");
        hipLaunchKernelGGL(k_gen_finish, dim3(1), dim3(256), 0, g->stream, g->at<GenStatus>(g->L.st),
                           g->at<double>(g->L.blk), d * bpp);
        GEN_TRY(hipGetLastError(), "finish launch");
        if ((rc = record(g, &ev)) != CG_OK) return rc;
        if (g->prof) ++g->timed;
    }
    return CG_OK;
}

int read_status(cg_general *g, GenStatus &out)
{
    GEN_TRY(hipMemcpyAsync(&out, g->ws + g->L.st, sizeof(GenStatus), hipMemcpyDeviceToHost, g->stream),
            "hipMemcpyAsync(status)");
    GEN_TRY(hipStreamSynchronize(g->stream), "hipStreamSynchronize");
    return CG_OK;
}

}  // namespace

extern "C" {

int cg_general_nodes(const cg_general_desc *desc, double *pnodes, double *unodes)
{
    int rc = validate_sizes(desc);
    if (rc != CG_OK) return rc;
    GenConst c;
    build_consts(desc, c);
    size_t a = 0, b = 0;
    for (int l = 0; l < c.d; ++l) {
        for (int k = 0; k < c.np[l]; ++k)
            if (pnodes) pnodes[a++] = c.pnode[l][k];
        for (int m = 0; m < c.nu[l]; ++m)
            if (unodes) unodes[b++] = 0.5 * c.umax * (c.tnode[l][m] + 1.0);
    }
    return CG_OK;
}

size_t cg_general_workspace_bytes(const cg_general_desc *desc)
{
    if (validate(desc) != CG_OK) return 0;
    GenConst c;
    build_consts(desc, c);
    return layout(c).total;
}

int cg_general_init(const cg_general_desc *desc, void *ws_dev, size_t ws_bytes, void *stream, cg_general **out)
{
    if (!out) return gfail(CG_EINVAL, "out is NULL");
    *out = nullptr;
    int rc = validate(desc);
    if (rc != CG_OK) return rc;
    cg_general *g = new (std::nothrow) cg_general();
    if (!g) return gfail(CG_ENOMEM, "host allocation failed");
    build_consts(desc, g->hc);
    g->L = layout(g->hc);
    if (!ws_dev || ws_bytes < g->L.total) {
        const size_t need = g->L.total;
        delete g;
        return gfail(CG_ENOMEM, "workspace has %zu bytes, needs %zu", ws_dev ? ws_bytes : 0, need);
    }
    if (((uintptr_t)ws_dev & 255) != 0) {
        delete g;
        return gfail(CG_EINVAL, "workspace must be 256-byte aligned");
    }
    if ((rc = require_gfx950()) != CG_OK) {
        delete g;
        return rc;
    }
    g->ws = (char *)ws_dev;
    g->stream = (hipStream_t)stream;
    const GenConst &c = g->hc;
    {
        int n[CG_MAX_D];
        for (int l = 0; l < c.d; ++l) n[l] = c.np[l];
        g->bt = EvalBatch{};
        g->bt.bp_stride = (long long)eval_packed_elems(c.d, n);
        for (int i = 0; i < c.d; ++i) {
            g->bt.x_off[i] = c.off[i];
            g->bt.npts[i] = c.NP * c.nu[i];
        }
    }
    hipError_t e = hipMemcpyAsync(g->ws + g->L.gc, &g->hc, sizeof(GenConst), hipMemcpyHostToDevice, g->stream);
    // Step 0: control polynomials of every node (node-major: drift components,
    // then payoffs), by the transform in place
    if (e == hipSuccess) {
        const long long n = (long long)c.d * c.NP * c.UP;
        hipLaunchKernelGGL(k_gen_gather, dim3(1024), dim3(256), 0, g->stream, g->at<double>(g->L.cc), desc->drift_dev,
                           desc->payoff_dev, c.d, c.NP, c.UP, n);
        e = hipGetLastError();
    }
    if (e == hipSuccess)
        e = run_transform(c.d, c.nu, g->at<double>(g->L.cc), g->at<double>(g->L.cc), 2LL * c.d * c.NP, g->stream);
    // the padding entries of the evaluation operands stay zero from here on
    if (e == hipSuccess) e = hipMemsetAsync(g->ws + g->L.evws, 0, g->L.evws_bytes, g->stream);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_gen_init, dim3(256), dim3(256), 0, g->stream, g->at<GenConst>(g->L.gc),
                           g->at<GenStatus>(g->L.st), g->at<double>(g->L.V), g->at<double>(g->L.U));
        e = hipGetLastError();
    }
    // the constants are copied from the handle's host memory: wait for it
    if (e == hipSuccess) e = hipStreamSynchronize(g->stream);
    if (e != hipSuccess) {
        delete g;
        return hfail(e, "general init");
    }
    *out = g;
    return CG_OK;
}

int cg_general_step(cg_general *g, int32_t nsteps, double *residual_out)
{
    if (!g) return gfail(CG_EINVAL, "game is NULL");
    if (nsteps < 0) return gfail(CG_EINVAL, "nsteps < 0");
    hipLaunchKernelGGL(k_gen_arm, dim3(1), dim3(64), 0, g->stream, g->at<GenStatus>(g->L.st), 0.0, 0);
    GEN_TRY(hipGetLastError(), "arm launch");
    int rc = queue_steps(g, nsteps);
    if (rc != CG_OK) return rc;
    if (residual_out) {
        GenStatus st;
        if ((rc = read_status(g, st)) != CG_OK) return rc;
        *residual_out = st.last_res;
        if (st.nonfinite) return gfail(CG_ENONFINITE, "non-finite residual after %d steps", st.steps_done);
    }
    return CG_OK;
}

int cg_general_solve(cg_general *g, int32_t max_steps, double tol, int32_t *steps_done, double *residual)
{
    if (!g) return gfail(CG_EINVAL, "game is NULL");
    if (max_steps < 0) return gfail(CG_EINVAL, "max_steps < 0");
    if (!(tol == tol)) return gfail(CG_EINVAL, "tol is NaN");
    hipLaunchKernelGGL(k_gen_arm, dim3(1), dim3(64), 0, g->stream, g->at<GenStatus>(g->L.st), tol > 0.0 ? tol : 0.0,
                       1);
    GEN_TRY(hipGetLastError(), "arm launch");
    GenStatus st;
    int rc;
    if (tol <= 0.0) {
        if ((rc = queue_steps(g, max_steps)) != CG_OK) return rc;
        if ((rc = read_status(g, st)) != CG_OK) return rc;
    } else {
        int queued = 0;
        const int chunk = 8;
        for (;;) {
            const int n = max_steps - queued < chunk ? max_steps - queued : chunk;
            if ((rc = queue_steps(g, n)) != CG_OK) return rc;
            queued += n;
            if ((rc = read_status(g, st)) != CG_OK) return rc;
            if (st.converged || queued >= max_steps) break;
        }
    }
    if (steps_done) *steps_done = st.steps_done;
    if (residual) *residual = st.last_res;
    if (st.nonfinite) return gfail(CG_ENONFINITE, "non-finite residual after %d steps", st.steps_done);
    if (tol > 0.0 && !st.converged) return CG_ENOTCONVERGED;
    return CG_OK;
}

int cg_general_get_state(cg_general *g, double *V_dev, double *U_dev, int32_t *r)
{
    if (!g) return gfail(CG_EINVAL, "game is NULL");
    const long long n = (long long)g->hc.d * g->hc.NP;
    if (V_dev) {
        hipLaunchKernelGGL(k_gen_copy, dim3(256), dim3(256), 0, g->stream, V_dev, g->at<double>(g->L.V), n);
        GEN_TRY(hipGetLastError(), "get_state launch");
    }
    if (U_dev) {
        hipLaunchKernelGGL(k_gen_copy, dim3(256), dim3(256), 0, g->stream, U_dev, g->at<double>(g->L.U), n);
        GEN_TRY(hipGetLastError(), "get_state launch");
    }
    if (r) {
        GenStatus st;
        int rc = read_status(g, st);
        if (rc != CG_OK) return rc;
        *r = st.total_steps;
    }
    return CG_OK;
}

int cg_general_set_state(cg_general *g, const double *V_dev, const double *U_dev)
{
    if (!g) return gfail(CG_EINVAL, "game is NULL");
    if (!V_dev) return gfail(CG_EINVAL, "V is NULL");
    const long long n = (long long)g->hc.d * g->hc.NP;
    hipLaunchKernelGGL(k_gen_copy, dim3(256), dim3(256), 0, g->stream, g->at<double>(g->L.V), V_dev, n);
    GEN_TRY(hipGetLastError(), "set_state launch");
    if (U_dev) {
        hipLaunchKernelGGL(k_gen_copy, dim3(256), dim3(256), 0, g->stream, g->at<double>(g->L.U), U_dev, n);
        GEN_TRY(hipGetLastError(), "set_state launch");
    }
    hipLaunchKernelGGL(k_gen_arm, dim3(1), dim3(64), 0, g->stream, g->at<GenStatus>(g->L.st), 0.0, 0);
    GEN_TRY(hipGetLastError(), "arm launch");
    return CG_OK;
}

int cg_general_profile(cg_general *g, int enable, double *phase_ms, int64_t *steps)
{
    if (!g) return gfail(CG_EINVAL, "game is NULL");
    if (phase_ms || steps) {
        GEN_TRY(hipStreamSynchronize(g->stream), "hipStreamSynchronize");
        double acc[4] = {0, 0, 0, 0};
        for (size_t k = 0; k + 5 <= g->ev_used; k += 5) {
            for (int p = 0; p < 4; ++p) {
                float ms = 0.f;
                GEN_TRY(hipEventElapsedTime(&ms, g->evs[k + p], g->evs[k + p + 1]), "hipEventElapsedTime");
                acc[p] += ms;
            }
        }
        if (phase_ms)
            for (int p = 0; p < 4; ++p) phase_ms[p] = acc[p];
        if (steps) *steps = g->timed;
    }
    g->prof = enable != 0;
    g->ev_used = 0;
    g->timed = 0;
    return CG_OK;
}

int cg_general_destroy(cg_general *g)
{
    if (!g) return CG_OK;
    for (hipEvent_t e : g->evs) (void)hipEventDestroy(e);
    delete g;
    return CG_OK;
}

}  // extern "C"
