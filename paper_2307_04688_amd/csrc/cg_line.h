// cg_line.h -- per-node line work of a value-iteration step (device code):
// the Euler-shifted update point, the Chebyshev series on the control line,
// and the constrained argmax of Step 3.
//
// Series lengths are compile-time (padded to a multiple of 4); the padding
// coefficients are exactly zero, so the recurrences give the same values as
// with the unpadded length, without data-dependent guards in the loops.
#pragma once

#include "cg_internal.h"

namespace cg {

// sum_{k<NW} c_k T_k(x) by Clenshaw's recurrence (coefficients in registers).
template <int NW>
__device__ __forceinline__ double clenshaw(const double (&c)[NW], double x)
{
    double b1 = 0.0, b2 = 0.0;
    const double x2 = 2.0 * x;
#pragma unroll
    for (int k = NW - 1; k >= 1; --k) {
        const double b0 = fma(x2, b1, c[k] - b2);
        b2 = b1;
        b1 = b0;
    }
    return fma(x, b1, c[0] - b2);
}

// Same with the coefficients in LDS (one row of a block tile).
template <int NW>
__device__ __forceinline__ double clenshaw_lds(const double *w, double x)
{
    double b1 = 0.0, b2 = 0.0;
    const double x2 = 2.0 * x;
#pragma unroll
    for (int k = NW - 1; k >= 1; --k) {
        const double b0 = fma(x2, b1, w[k] - b2);
        b2 = b1;
        b1 = b0;
    }
    return fma(x, b1, w[0] - b2);
}

// Value, first and second derivative of sum_{k<NW} c_k T_k at x, from the
// Clenshaw recurrence b_k = c_k + 2x b_{k+1} - b_{k+2} differentiated in x.
template <int NW>
__device__ __forceinline__ void clenshaw3(const double (&c)[NW], double x, double &f, double &f1, double &f2)
{
    double b1 = 0.0, b2 = 0.0, d1 = 0.0, d2 = 0.0, e1 = 0.0, e2 = 0.0;
    const double x2 = 2.0 * x;
#pragma unroll
    for (int k = NW - 1; k >= 1; --k) {
        const double b0 = fma(x2, b1, c[k] - b2);
        const double d0 = fma(x2, d1, 2.0 * b1 - d2);
        const double e0 = fma(x2, e1, 4.0 * d1 - e2);
        b2 = b1; b1 = b0;
        d2 = d1; d1 = d0;
        e2 = e1; e1 = e0;
    }
    f = fma(x, b1, c[0] - b2);
    f1 = fma(x, d1, b1 - d2);
    f2 = fma(x, e1, 2.0 * d1 - e2);
}

// True if the series is certainly strictly concave on [-1,1]: with q'' the
// coefficients of the second derivative (obtained by applying the derivative
// rule c_k q'_k = q'_{k+2} + 2 (k+1) q_{k+1} twice, in one backward sweep),
// q''_0 + sum_{l>=1} |q''_l| < 0 bounds q'' from above since |T_l| <= 1.
template <int NW>
__device__ __forceinline__ bool certainly_concave(const double (&q)[NW])
{
    double dq1 = 0.0, dq2 = 0.0;   // q'_{k+1}, q'_{k+2}
    double ee1 = 0.0, ee2 = 0.0;   // q''_{k+1}, q''_{k+2}
    double sum_abs = 0.0, e0 = 0.0;
#pragma unroll
    for (int k = NW - 2; k >= 0; --k) {
        const double dk = dq2 + 2.0 * (double)(k + 1) * q[k + 1];
        double ek = ee2 + 2.0 * (double)(k + 1) * dq1;
        if (k == 0) ek *= 0.5;
        if (k >= 1) sum_abs += fabs(ek); else e0 = ek;
        dq2 = dq1; dq1 = dk;
        ee2 = ee1; ee1 = ek;
    }
    return e0 + sum_abs < 0.0;
}

// Maximiser over s in [-1,1] of v(s) = sum_l q_l T_l(s) (Step 3; the paper
// recommends Newton's method on v').  Strictly concave lines (the usual case)
// take the endpoint whose one-sided derivative points outward, or a
// bracketed Newton iteration on v' started at s0.  Other lines take the
// global maximum over their local maxima: an endpoint whose one-sided
// derivative points outward and every sign change + to - of v' on a uniform
// grid of 16 n intervals (n = number of control nodes), refined by
// bisection; ties go to the smaller s.  An endpoint where v still rises into
// the interval is no candidate, however close its value.  Returns v(s*) and
// stores s*.
template <int NW>
__device__ double line_argmax(const double (&q)[NW], int n, double s0, double &s_out)
{
    double s;
    if (certainly_concave(q)) {
        // v'(+1) = sum_l l^2 q_l and v'(-1) = sum_l (-1)^(l+1) l^2 q_l; the
        // same sum of magnitudes bounds |T_l'| <= l^2 and so the rounding of v'
        double fr = 0.0, fl = 0.0, mag = 0.0;
#pragma unroll
        for (int l = 1; l < NW; ++l) {
            const double t = (double)(l * l) * q[l];
            fr += t;
            fl += (l & 1) ? t : -t;
            mag += fabs(t);
        }
        const double floor1 = 1e-15 * mag;  // a few eps of the terms of v'
        if (fl <= 0.0) {
            s = -1.0;
        } else if (fr >= 0.0) {
            s = 1.0;
        } else {
            // bracketed Newton on v'.  Stops when v' is within its rounding
            // floor (the root is then resolved as well as v' allows), or
            // after a Newton step <= 1e-12 (quadratic convergence leaves an
            // error of order 1e-24 |v'''/v''|).
            double lo = -1.0, hi = 1.0, f, f1, f2;
            s = fmin(fmax(s0, -1.0), 1.0);
            for (int it = 0; it < 64; ++it) {
                clenshaw3(q, s, f, f1, f2);
                if (f1 > 0.0) lo = s; else hi = s;
                if (fabs(f1) <= floor1) break;
                double sn = s - f1 / f2;
                const bool newton = sn > lo && sn < hi;
                if (!newton) sn = 0.5 * (lo + hi);
                const double step = fabs(sn - s);
                s = sn;
                if ((newton && step <= 1e-12) || hi - lo <= 4.5e-16) break;
            }
        }
    } else {
        const int G = 16 * n;
        double f, f1a, f2;
        clenshaw3(q, -1.0, f, f1a, f2);
        bool have = f1a <= 0.0;  // the left endpoint is a local maximum
        double best_s = -1.0, best_v = have ? clenshaw(q, -1.0) : 0.0;
        double sa = -1.0;
        for (int g = 1; g <= G; ++g) {
            const double sb = -1.0 + 2.0 * (double)g / (double)G;
            double f1b;
            clenshaw3(q, sb, f, f1b, f2);
            if (f1a > 0.0 && f1b <= 0.0) {
                double lo = sa, hi = sb;
                for (int it = 0; it < 200; ++it) {
                    const double mid = 0.5 * (lo + hi);
                    if (mid <= lo || mid >= hi) break;
                    double fm, f1m, f2m;
                    clenshaw3(q, mid, fm, f1m, f2m);
                    if (f1m > 0.0) lo = mid; else hi = mid;
                }
                const double sc = 0.5 * (lo + hi);
                const double v = clenshaw(q, sc);
                if (!have || v > best_v + 1e-15 * fmax(1.0, fabs(best_v))) {
                    best_v = v;
                    best_s = sc;
                    have = true;
                }
            }
            sa = sb;
            f1a = f1b;
        }
        if (f1a >= 0.0) {  // the right endpoint is a local maximum
            const double v1 = clenshaw(q, 1.0);
            if (!have || v1 > best_v + 1e-15 * fmax(1.0, fabs(best_v))) best_s = 1.0;
        }
        s = best_s;  // -1 when v' is not a number (no candidate)
    }
    s_out = s;
    return clenshaw(q, s);
}

// Physical node coordinates p, controls u^{[r]} of all players and the drift
// b = g(p, u^{[r]}(p)) = M p + beta * u at node j (Section 2.1).
template <int D>
__device__ __forceinline__ void node_state(const GameConst *__restrict__ gc, const double *__restrict__ Uold,
                                           int j, double (&p)[D], double (&ub)[D], double (&b)[D])
{
    const int N = gc->N;
    const int NN = (int)gc->NN;
    int rem = j;
#pragma unroll
    for (int l = D - 1; l >= 0; --l) {
        const int k = rem % N;
        rem /= N;
        p[l] = gc->pnode[k];
    }
#pragma unroll
    for (int l = 0; l < D; ++l) ub[l] = Uold[l * NN + j];
#pragma unroll
    for (int l = 0; l < D; ++l) {
        double s = 0.0;
#pragma unroll
        for (int m = 0; m < D; ++m) s = fma(gc->M[l * D + m], p[m], s);
        b[l] = fma(gc->beta[l], ub[l], s);
    }
}

// Step 2 at one (player i, node j), for the control nodes m = part,
// part + parts, ...: sample h G_i + delta V_i on the line whose coefficients
// w (in the normalised i-th coordinate, NW entries zero-padded, in LDS) are
// known, and accumulate their share of the DCT-I fit in u into q (NQ
// entries; the fit matrix is zero beyond the control-node count).
template <int D, int NW, int NQ>
__device__ __forceinline__ void line_fit(const GameConst *__restrict__ gc, int i, const double (&p)[D],
                                         const double (&ub)[D], const double (&b)[D], const double *w, int part,
                                         int parts, double (&q)[NQ])
{
    const double h = gc->h, pmax = gc->pmax;
    const double gamma = 2.0 * h * gc->beta[i] / pmax;
    const double alpha = 2.0 * (p[i] + h * b[i] - h * gc->beta[i] * ub[i]) / pmax - 1.0;
    const double Ai = gc->A[i], dmg = 0.5 * gc->phi[i] * p[i] * p[i];
    const double delta = gc->delta;
    const int Nu = gc->Nu;
#pragma unroll
    for (int l = 0; l < NQ; ++l) q[l] = 0.0;
    for (int m = part; m < Nu; m += parts) {
        const double u = gc->unode[m];
        const double cont = clenshaw_lds<NW>(w, fma(gamma, u, alpha));
        const double val = h * (u * (Ai - 0.5 * u) - dmg) + delta * cont;
        const double *Dcol = gc->Du + m;
#pragma unroll
        for (int l = 0; l < NQ; ++l) q[l] = fma(Dcol[l * kMaxN], val, q[l]);
    }
}

// As line_fit, with the line coefficients in registers, and four control
// nodes evaluated together (four independent Clenshaw chains) so that the
// dependent FP64 operations of one chain overlap those of the others.
// Requires the control-node count to be a multiple of 4 * parts, or the
// fit matrix columns past it to be zero (they are: padding columns of Du).
template <int D, int NW, int NQ>
__device__ __forceinline__ void line_fit_regs(const GameConst *__restrict__ gc, int i, const double (&p)[D],
                                              const double (&ub)[D], const double (&b)[D], const double (&w)[NW],
                                              int part, int parts, double (&q)[NQ])
{
    const double h = gc->h, pmax = gc->pmax;
    const double gamma = 2.0 * h * gc->beta[i] / pmax;
    const double alpha = 2.0 * (p[i] + h * b[i] - h * gc->beta[i] * ub[i]) / pmax - 1.0;
    const double Ai = gc->A[i], dmg = 0.5 * gc->phi[i] * p[i] * p[i];
    const double delta = gc->delta;
    const int Nu = gc->Nu;
#pragma unroll
    for (int l = 0; l < NQ; ++l) q[l] = 0.0;
    for (int m0 = 4 * part; m0 < Nu; m0 += 4 * parts) {
        double x2[4], b1[4], b2[4], val[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            x2[e] = 2.0 * fma(gamma, gc->unode[m0 + e], alpha);
            b1[e] = 0.0;
            b2[e] = 0.0;
        }
#pragma unroll
        for (int k = NW - 1; k >= 1; --k) {
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const double b0 = fma(x2[e], b1[e], w[k] - b2[e]);
                b2[e] = b1[e];
                b1[e] = b0;
            }
        }
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const double u = gc->unode[m0 + e];
            const double cont = fma(0.5 * x2[e], b1[e], w[0] - b2[e]);
            val[e] = (m0 + e < Nu) ? h * (u * (Ai - 0.5 * u) - dmg) + delta * cont : 0.0;
        }
        const double *Dcol = gc->Du + m0;
#pragma unroll
        for (int l = 0; l < NQ; ++l) {
            double t = q[l];
#pragma unroll
            for (int e = 0; e < 4; ++e) t = fma(Dcol[l * kMaxN + e], val[e], t);
            q[l] = t;
        }
    }
}

// Chebyshev coefficients in s of the line function
//     v(s) = h G_i(p_i, u(s)) + delta * sum_{k<NW} w_k T_k(a + c s),
// u(s) = u_max (s + 1) / 2, a = alpha + c, c = gamma u_max / 2, computed
// directly instead of by sampling at the control nodes and fitting.  When
// the number of control nodes is at least N (and at least 3) the fit of
// Step 2 is exact for this polynomial, so both give the same coefficients up
// to rounding.  The continuation term runs Clenshaw's recurrence
// b_k = w_k + 2 (a + c s) b_{k+1} - b_{k+2} on Chebyshev series in s, using
// s T_0 = T_1 and s T_l = (T_{l+1} + T_{l-1}) / 2; b_k has degree NW-1-k.
// The payoff term is the exact quadratic h (A u - u^2/2 - phi p_i^2/2) with
// u = (u_max/2)(T_0 + T_1) and u^2 = (u_max^2/4)(3/2 T_0 + 2 T_1 + 1/2 T_2).
template <int D, int NW>
__device__ __forceinline__ void line_compose(const GameConst *__restrict__ gc, int i, const double (&p)[D],
                                             const double (&ub)[D], const double (&b)[D], const double *w,
                                             double (&q)[NW])
{
    const double h = gc->h, pmax = gc->pmax, um = gc->umax;
    const double gamma = 2.0 * h * gc->beta[i] / pmax;
    const double alpha = 2.0 * (p[i] + h * b[i] - h * gc->beta[i] * ub[i]) / pmax - 1.0;
    const double c = 0.5 * gamma * um;
    const double a = alpha + c;
    const double a2 = 2.0 * a, c2 = 2.0 * c;
    double bb[2][NW];  // bb[k & 1] holds b_k; entries past the degree stay zero
#pragma unroll
    for (int m = 0; m < NW; ++m) { bb[0][m] = 0.0; bb[1][m] = 0.0; }
#pragma unroll
    for (int k = NW - 1; k >= 1; --k) {
        const double *B1 = bb[(k + 1) & 1];  // b_{k+1}
        double *B0 = bb[k & 1];              // b_{k+2}, overwritten by b_k
        const int len = NW - k;              // entries of b_k
#pragma unroll
        for (int m = 0; m < len; ++m) {
            // 2 (a + c s) b_{k+1} - b_{k+2}, coefficient m; the term of c s
            // b_{k+1} is c (b_{m-1} + b_{m+1}) except at m = 0, 1
            const double lin = fma(a2, B1[m], -B0[m]);
            double t;
            if (m == 0) t = fma(c, B1[1], lin);
            else if (m == 1) t = fma(c2, B1[0], fma(c, B1[2], lin));
            else t = fma(c, B1[m - 1] + (m + 1 < NW ? B1[m + 1] : 0.0), lin);
            B0[m] = (m == 0) ? t + w[k] : t;
        }
    }
    // P(s) = w_0 + (a + c s) b_1 - b_2
    const double *B1 = bb[1];
    const double *B2 = bb[0];
    const double Ai = gc->A[i], dmg = 0.5 * gc->phi[i] * p[i] * p[i], delta = gc->delta;
#pragma unroll
    for (int m = 0; m < NW; ++m) {
        double sb;  // coefficient m of c s b_1
        if (m == 0) sb = 0.5 * c * B1[1];
        else if (m == 1) sb = c * (B1[0] + 0.5 * B1[2]);
        else sb = 0.5 * c * (B1[m - 1] + (m + 1 < NW ? B1[m + 1] : 0.0));
        double P = fma(a, B1[m], sb) - B2[m];
        if (m == 0) P += w[0];
        q[m] = delta * P;
    }
    q[0] += h * (Ai * 0.5 * um - 0.1875 * um * um - dmg);
    q[1] += h * (Ai * 0.5 * um - 0.25 * um * um);
    if (NW > 2) q[2] += -0.0625 * h * um * um;
}

// Value and first derivative of sum_{k<NW} c_k T_k at x (the first two
// recurrences of clenshaw3).
template <int NW>
__device__ __forceinline__ void clenshaw2(const double (&c)[NW], double x, double &f, double &f1)
{
    double b1 = 0.0, b2 = 0.0, d1 = 0.0, d2 = 0.0;
    const double x2 = 2.0 * x;
#pragma unroll
    for (int k = NW - 1; k >= 1; --k) {
        const double b0 = fma(x2, b1, c[k] - b2);
        const double d0 = fma(x2, d1, 2.0 * b1 - d2);
        b2 = b1; b1 = b0;
        d2 = d1; d1 = d0;
    }
    f = fma(x, b1, c[0] - b2);
    f1 = fma(x, d1, b1 - d2);
}

// First and second derivative at X >= 1 of sum_k |c_k| T_k: every derivative
// of every T_k is non-negative and non-decreasing on [1, inf), so these bound
// |sum_k c_k T_k'| and |sum_k c_k T_k''| on [-X, X].
template <int NW>
__device__ __forceinline__ void abs_series_bounds(const double (&c)[NW], double X, double &g1, double &g2)
{
    double b1 = 0.0, b2 = 0.0, d1 = 0.0, d2 = 0.0, e1 = 0.0, e2 = 0.0;
    const double x2 = 2.0 * X;
#pragma unroll
    for (int k = NW - 1; k >= 1; --k) {
        const double b0 = fma(x2, b1, fabs(c[k]) - b2);
        const double d0 = fma(x2, d1, 2.0 * b1 - d2);
        const double e0 = fma(x2, e1, 4.0 * d1 - e2);
        b2 = b1; b1 = b0;
        d2 = d1; d1 = d0;
        e2 = e1; e1 = e0;
    }
    g1 = fma(X, d1, b1 - d2);
    g2 = fma(X, e1, 2.0 * d1 - e2);
}

// Step 3 on the line function of line_compose,
//     v(s) = h G_i(p_i, u(s)) + delta W(a + c s),  W = sum_{k<NW} w_k T_k,
// without forming its series in s, for the lines that are certainly strictly
// concave: v''(s) = delta c^2 W''(x) - h u_max^2 / 4 (the payoff is quadratic
// in u), and with X = max(1, |a| + |c|) the bound of abs_series_bounds on
// |W''| over the segment certifies v'' <= -h u_max^2 / 8 when
// delta c^2 sup|W''| <= h u_max^2 / 8.  The maximiser is then found as in the
// concave branch of line_argmax: an endpoint whose one-sided derivative
// points outward, or the bracketed Newton iteration on v' from s0, with
// W, W', W'' at x = a + c s by Clenshaw.  Returns false, touching nothing,
// when the bound does not certify concavity (the caller composes the series
// and takes line_argmax).  Exact arithmetic gives the same maximiser as
// line_argmax on line_compose's coefficients.
template <int D, int NW>
__device__ __forceinline__ bool line_argmax_direct(const GameConst *__restrict__ gc, int i, const double (&p)[D],
                                                   const double (&ub)[D], const double (&b)[D],
                                                   const double (&w)[NW], double s0, double &v_out,
                                                   double &s_out)
{
    const double h = gc->h, pmax = gc->pmax, um = gc->umax;
    const double gamma = 2.0 * h * gc->beta[i] / pmax;
    const double alpha = 2.0 * (p[i] + h * b[i] - h * gc->beta[i] * ub[i]) / pmax - 1.0;
    const double c = 0.5 * gamma * um;
    const double a = alpha + c;
    const double Ai = gc->A[i], dmg = 0.5 * gc->phi[i] * p[i] * p[i], delta = gc->delta;
    const double curv = 0.25 * h * um * um;  // -d^2/ds^2 of the payoff term
    double g1, g2;
    abs_series_bounds(w, fmax(1.0, fabs(a) + fabs(c)), g1, g2);
    if (!(delta * c * c * g2 <= 0.5 * curv)) return false;  // also catches NaN
    const double dc = delta * c, dcc = delta * c * c, hu = 0.5 * h * um;
    // v' at the endpoints: u = 0 at s = -1, u = u_max at s = +1
    double W, W1;
    clenshaw2(w, a - c, W, W1);
    const double fl = fma(dc, W1, hu * Ai);
    clenshaw2(w, a + c, W, W1);
    const double fr = fma(dc, W1, hu * (Ai - um));
    // a few eps of the terms of v' bound its rounding
    const double floor1 = 1e-15 * (fabs(dc) * g1 + hu * (fabs(Ai) + um));
    double s;
    if (fl <= 0.0) {
        s = -1.0;
    } else if (fr >= 0.0) {
        s = 1.0;
    } else {
        // the same stopping rules as line_argmax's Newton iteration
        double lo = -1.0, hi = 1.0;
        s = fmin(fmax(s0, -1.0), 1.0);
        for (int it = 0; it < 64; ++it) {
            double W2;
            clenshaw3(w, fma(c, s, a), W, W1, W2);
            const double u = 0.5 * um * (s + 1.0);
            const double f1 = fma(dc, W1, hu * (Ai - u));
            const double f2 = fma(dcc, W2, -curv);
            if (f1 > 0.0) lo = s; else hi = s;
            if (fabs(f1) <= floor1) break;
            double sn = s - f1 / f2;
            const bool newton = sn > lo && sn < hi;
            if (!newton) sn = 0.5 * (lo + hi);
            const double step = fabs(sn - s);
            s = sn;
            if ((newton && step <= 1e-12) || hi - lo <= 4.5e-16) break;
        }
    }
    const double u = 0.5 * um * (s + 1.0);
    v_out = fma(delta, clenshaw(w, fma(c, s, a)), h * (u * (Ai - 0.5 * u) - dmg));
    s_out = s;
    return true;
}

}  // namespace cg
