// cg_line.h -- per-node line work of a value-iteration step (device code):
// the Euler-shifted update point, the Chebyshev series on the control line,
// and the constrained argmax of Step 3.
#pragma once

#include "cg_internal.h"

namespace cg {

// sum_{k<n} c_k T_k(x) by Clenshaw's recurrence (coefficients in registers).
template <int NMAX>
__device__ __forceinline__ double clenshaw(const double (&c)[NMAX], int n, double x)
{
    double b1 = 0.0, b2 = 0.0;
    const double x2 = 2.0 * x;
#pragma unroll
    for (int k = NMAX - 1; k >= 1; --k) {
        if (k < n) {
            const double b0 = fma(x2, b1, c[k] - b2);
            b2 = b1;
            b1 = b0;
        }
    }
    return fma(x, b1, c[0] - b2);
}

// Value, first and second derivative of sum_{k<n} c_k T_k at x, from the
// Clenshaw recurrence b_k = c_k + 2x b_{k+1} - b_{k+2} differentiated in x.
template <int NMAX>
__device__ __forceinline__ void clenshaw3(const double (&c)[NMAX], int n, double x, double &f, double &f1,
                                          double &f2)
{
    double b1 = 0.0, b2 = 0.0, d1 = 0.0, d2 = 0.0, e1 = 0.0, e2 = 0.0;
    const double x2 = 2.0 * x;
#pragma unroll
    for (int k = NMAX - 1; k >= 1; --k) {
        if (k < n) {
            const double b0 = fma(x2, b1, c[k] - b2);
            const double d0 = fma(x2, d1, 2.0 * b1 - d2);
            const double e0 = fma(x2, e1, 4.0 * d1 - e2);
            b2 = b1; b1 = b0;
            d2 = d1; d1 = d0;
            e2 = e1; e1 = e0;
        }
    }
    f = fma(x, b1, c[0] - b2);
    f1 = fma(x, d1, b1 - d2);
    f2 = fma(x, e1, 2.0 * d1 - e2);
}

// True if the series is certainly strictly concave on [-1,1]: with q'' the
// coefficients of the second derivative (obtained by applying the derivative
// rule c_k q'_k = q'_{k+2} + 2 (k+1) q_{k+1} twice, in one backward sweep),
// q''_0 + sum_{l>=1} |q''_l| < 0 bounds q'' from above since |T_l| <= 1.
template <int NMAX>
__device__ __forceinline__ bool certainly_concave(const double (&q)[NMAX], int n)
{
    double dq1 = 0.0, dq2 = 0.0;   // q'_{k+1}, q'_{k+2}
    double ee1 = 0.0, ee2 = 0.0;   // q''_{k+1}, q''_{k+2}
    double sum_abs = 0.0, e0 = 0.0;
#pragma unroll
    for (int k = NMAX - 2; k >= 0; --k) {
        if (k <= n - 2) {
            const double dk = dq2 + 2.0 * (double)(k + 1) * q[k + 1];
            double ek = ee2 + 2.0 * (double)(k + 1) * dq1;
            if (k == 0) ek *= 0.5;
            if (k >= 1) sum_abs += fabs(ek); else e0 = ek;
            dq2 = dq1; dq1 = dk;
            ee2 = ee1; ee1 = ek;
        }
    }
    return e0 + sum_abs < 0.0;
}

// Maximiser over s in [-1,1] of v(s) = sum_{l<n} q_l T_l(s) (Step 3; the
// paper recommends Newton's method on v').  Strictly concave lines (the
// usual case) take the endpoint whose one-sided derivative points outward,
// or a bracketed Newton iteration on v' started at s0.  Other lines take the
// global maximum over both endpoints and every sign change + to - of v' on a
// uniform grid of 16 n intervals, refined by bisection; ties go to the
// smaller s.  Returns v(s*) and stores s*.
template <int NMAX>
__device__ double line_argmax(const double (&q)[NMAX], int n, double s0, double &s_out)
{
    double s;
    if (certainly_concave(q, n)) {
        double f, fl, fr, f2;
        clenshaw3(q, n, -1.0, f, fl, f2);
        clenshaw3(q, n, 1.0, f, fr, f2);
        if (fl <= 0.0) {
            s = -1.0;
        } else if (fr >= 0.0) {
            s = 1.0;
        } else {
            double lo = -1.0, hi = 1.0;
            s = fmin(fmax(s0, -1.0), 1.0);
            for (int it = 0; it < 100; ++it) {
                double f1;
                clenshaw3(q, n, s, f, f1, f2);
                if (f1 > 0.0) lo = s; else hi = s;
                if (f1 == 0.0) break;
                double sn = s - f1 / f2;
                if (!(sn > lo && sn < hi)) sn = 0.5 * (lo + hi);
                const bool done = fabs(sn - s) <= 4.5e-16 * fmax(1.0, fabs(s));
                s = sn;
                if (done || hi - lo <= 4.5e-16) break;
            }
        }
    } else {
        const int G = 16 * n;
        double best_s = -1.0, best_v = clenshaw(q, n, -1.0);
        double f, f1a, f2;
        clenshaw3(q, n, -1.0, f, f1a, f2);
        double sa = -1.0;
        for (int g = 1; g <= G; ++g) {
            const double sb = -1.0 + 2.0 * (double)g / (double)G;
            double f1b;
            clenshaw3(q, n, sb, f, f1b, f2);
            if (f1a > 0.0 && f1b <= 0.0) {
                double lo = sa, hi = sb;
                for (int it = 0; it < 200; ++it) {
                    const double mid = 0.5 * (lo + hi);
                    if (mid <= lo || mid >= hi) break;
                    double fm, f1m, f2m;
                    clenshaw3(q, n, mid, fm, f1m, f2m);
                    if (f1m > 0.0) lo = mid; else hi = mid;
                }
                const double sc = 0.5 * (lo + hi);
                const double v = clenshaw(q, n, sc);
                if (v > best_v + 1e-15 * fmax(1.0, fabs(best_v))) { best_v = v; best_s = sc; }
            }
            sa = sb;
            f1a = f1b;
        }
        const double v1 = clenshaw(q, n, 1.0);
        if (v1 > best_v + 1e-15 * fmax(1.0, fabs(best_v))) best_s = 1.0;
        s = best_s;
    }
    s_out = s;
    return clenshaw(q, n, s);
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

// Steps 2-4 at one (player i, node j) once w_k, the coefficients of V_i on
// the line {p + h b + t e_i} in the normalised i-th coordinate, are known:
// sample h G_i + delta V_i at the control nodes, fit in u (DCT-I), maximise,
// return the new value and control.
template <int D, int NW>
__device__ __forceinline__ void line_update(const GameConst *__restrict__ gc, int i, const double (&p)[D],
                                            const double (&ub)[D], const double (&b)[D], const double (&w)[NW],
                                            double &v_new, double &u_new)
{
    const double h = gc->h, pmax = gc->pmax;
    const double gamma = 2.0 * h * gc->beta[i] / pmax;
    const double alpha = 2.0 * (p[i] + h * b[i] - h * gc->beta[i] * ub[i]) / pmax - 1.0;
    const double Ai = gc->A[i], dmg = 0.5 * gc->phi[i] * p[i] * p[i];
    const int Nu = gc->Nu, N = gc->N;
    double q[kMaxN];
#pragma unroll
    for (int l = 0; l < kMaxN; ++l) q[l] = 0.0;
    for (int m = 0; m < Nu; ++m) {
        const double u = gc->unode[m];
        const double cont = clenshaw(w, N, fma(gamma, u, alpha));
        const double val = h * (u * (Ai - 0.5 * u) - dmg) + gc->delta * cont;
#pragma unroll
        for (int l = 0; l < kMaxN; ++l)
            if (l < Nu) q[l] = fma(gc->Du[l * kMaxN + m], val, q[l]);
    }
    const double s0 = 2.0 * ub[i] / gc->umax - 1.0;
    double s;
    v_new = line_argmax(q, Nu, s0, s);
    u_new = 0.5 * gc->umax * (s + 1.0);
}

}  // namespace cg
