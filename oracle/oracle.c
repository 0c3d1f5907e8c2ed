/*
 * oracle.c -- plain, slow, FP64 CPU reference of the tensorial Chebyshev
 * value iteration for the J-player transboundary-pollution game
 * (de Castro, Gaton & Gomez, "A tensorial-parallel Chebyshev method for a
 * differential game theory problem", arXiv 2307.04688).
 *
 * TEST INFRASTRUCTURE ONLY.  The test suite, the smoke check and the CPU
 * baseline leg of the benchmark load this file; the GPU library shares no
 * code, header, table or helper with it.
 *
 * Every function computes its result from the plain definition in the
 * paper, in IEEE binary64 (see OR_REAL below), built with -O2
 * -ffp-contract=off (no fused multiply-add, no fast-math).  Readings of
 * places where the paper is silent or garbled are marked "Reading:".
 *
 * Array conventions: an n-dimensional array of shape N[0] x ... x N[d-1] is
 * stored in C order (last mode fastest).  Index k of a mode is the Lobatto
 * node x_k = cos(pi k / (N-1)), so index 0 is x = +1.
 */
#include <tgmath.h>
#include <omp.h>
#include <stdlib.h>
#include <string.h>

/* Arithmetic type.  The oracle is binary64 (OR_REAL undefined: double).
 * The same source built with -DOR_REAL="long double" (x87 extended format,
 * 64-bit significand, unit roundoff 2^-64 against 2^-53) is a second
 * reference whose rounding error is 2^-11 of the binary64 one: it measures
 * the binary64 oracle's own rounding error, nothing else changes.  Every
 * array and scalar below is of this type; <tgmath.h> picks cos/fabs/fmax of
 * the same precision. */
#ifndef OR_REAL
#define OR_REAL double
#endif
typedef OR_REAL real;
#define OR_PI ((real)3.14159265358979323846264338327950288L)

#define OR_MAXD 4
#define OR_MAXN 64

/* Number of OpenMP threads the parallel loops below use. */
int or_num_threads(void) { return omp_get_max_threads(); }

/* cos(pi a / n) with a reduced modulo 2n first, so the argument stays in
 * [0, 2 pi).  Chebyshev nodes and T_l(alpha^k) = cos(pi l k / n) (Section
 * 3.1) both use it. */
static real cos_pi_frac(long a, long n)
{
    long r = a % (2 * n);
    if (r < 0) r += 2 * n;
    return cos(OR_PI * (real)r / (real)n);
}

/* Chebyshev-Lobatto nodes alpha^k = cos(pi k / n), k = 0..n, n = N-1 (Section
 * 3.1, the extrema of T_n). */
void or_nodes(int N, real *x)
{
    int n = N - 1;
    for (int k = 0; k < N; ++k) x[k] = (n == 0) ? 1.0 : cos_pi_frac(k, n);
}

/* T_0..T_{cnt-1} at x by the three-term recurrence T_{k+1} = 2 x T_k - T_{k-1}.
 * Equals cos(k arccos x) on [-1,1] (Section 3.1) and continues the same
 * polynomials outside it.  Reading: update points that leave the box by
 * O(h) are evaluated by polynomial extrapolation, not clamped. */
void or_cheb_T(int cnt, real x, real *T)
{
    if (cnt > 0) T[0] = 1.0;
    if (cnt > 1) T[1] = x;
    for (int k = 2; k < cnt; ++k) T[k] = 2.0 * x * T[k - 1] - T[k - 2];
}

/* One-dimensional interpolation coefficients, eq. (forcoef) of Definition
 * "interpolant in one variable" (Section 3.1):
 *   p_l = (w_l / n) sum''_{k=0..n} F_k T_l(alpha^k),  w_l = 1 for l in {0,n},
 *   else 2; the double prime halves the k = 0 and k = n terms.
 * Input F and output p are strided views of length N = n+1. */
void or_coef_1d(int N, const real *F, long fstride, real *p, long pstride)
{
    int n = N - 1;
    if (n == 0) { p[0] = F[0]; return; }
    for (int l = 0; l <= n; ++l) {
        real s = 0.0;
        for (int k = 0; k <= n; ++k) {
            real term = F[k * fstride] * cos_pi_frac((long)l * k, n);
            if (k == 0 || k == n) term *= 0.5;
            s += term;
        }
        real w = (l == 0 || l == n) ? 1.0 : 2.0;
        p[l * pstride] = (w / (real)n) * s;
    }
}

/* n-dimensional coefficients, Algorithm Cnv (Section 3.1): the 1-D rule of
 * eq. (forcoef) along every mode in turn.  'order' lists the modes in the
 * order they are processed (NULL = 0..d-1); the result does not depend on it
 * because the n-dimensional transform is a tensor product of 1-D ones. */
void or_transform(int d, const int *N, const int *order, const real *vals, real *coef)
{
    long total = 1;
    for (int l = 0; l < d; ++l) total *= N[l];
    real *buf = (real *)malloc(sizeof(real) * (size_t)total);
    real *tmp = (real *)malloc(sizeof(real) * OR_MAXN);
    memcpy(coef, vals, sizeof(real) * (size_t)total);
    for (int t = 0; t < d; ++t) {
        int m = order ? order[t] : t;
        long stride = 1;
        for (int l = m + 1; l < d; ++l) stride *= N[l];
        long outer = total / (stride * N[m]);
        memcpy(buf, coef, sizeof(real) * (size_t)total);
        for (long o = 0; o < outer; ++o)
            for (long in = 0; in < stride; ++in) {
                const real *F = buf + o * N[m] * stride + in;
                or_coef_1d(N[m], F, stride, tmp, 1);
                for (int l = 0; l < N[m]; ++l) coef[o * N[m] * stride + in + l * stride] = tmp[l];
            }
    }
    free(tmp);
    free(buf);
}

/* Value of the n-dimensional series sum_k c_k T_{k_1}(x_1)...T_{k_d}(x_d)
 * (Definition "interpolant in n variables") at one point, by successive
 * mode-n products with the vectors (T_l(x_m))_l, last mode first (the
 * evaluation of Section 3.2 with one point per mode).  'work' must hold
 * prod(N)/N[d-1] doubles. */
real or_eval_point(int d, const int *N, const real *coef, const real *x, real *work)
{
    real T[OR_MAXN];
    long outer = 1;
    for (int l = 0; l < d - 1; ++l) outer *= N[l];
    const real *src = coef;
    for (int m = d - 1; m >= 0; --m) {
        or_cheb_T(N[m], x[m], T);
        for (long o = 0; o < outer; ++o) {
            real s = 0.0;
            for (int k = 0; k < N[m]; ++k) s += src[o * N[m] + k] * T[k];
            work[o] = s;
        }
        src = work;
        if (m > 0) outer /= N[m - 1];
    }
    return src[0];
}

/* Series values at npts points x (npts x d, row-major). */
void or_eval(int d, const int *N, const real *coef, const real *x, long npts, real *out)
{
    long wsz = 1;
    for (int l = 0; l < d - 1; ++l) wsz *= N[l];
    #pragma omp parallel
    {
        real *work = (real *)malloc(sizeof(real) * (size_t)(wsz > 0 ? wsz : 1));
        #pragma omp for schedule(static)
        for (long q = 0; q < npts; ++q) out[q] = or_eval_point(d, N, coef, x + q * d, work);
        free(work);
    }
}

/* Derivative coefficients (Proposition in Section 3.1): for a series
 * sum_{j=0..n} p_j T_j, the derivative on [-1,1] is sum_{l=0..n-1} q_l T_l with
 *   q_l = (2 / c_l) sum_{j=l+1..n, j+l odd} j p_j,  c_0 = 2, c_l = 1 (l >= 1).
 * Reading: the printed "2/c_l + sum" is a product "2/c_l * sum"; the interval
 * factor 2/(b-a) is applied by the caller. */
void or_chebder(int cnt, const real *p, real *q)
{
    int n = cnt - 1;
    for (int l = 0; l < n; ++l) {
        real s = 0.0;
        for (int j = l + 1; j <= n; ++j)
            if ((j + l) % 2 == 1) s += (real)j * p[j];
        q[l] = (l == 0 ? 1.0 : 2.0) * s;
    }
    if (n >= 0) q[n] = 0.0;
}

/* sum_{l<cnt} q_l T_l(s), with T_l generated by the recurrence. */
real or_series(int cnt, const real *q, real s)
{
    real T[OR_MAXN];
    or_cheb_T(cnt, s, T);
    real v = 0.0;
    for (int l = 0; l < cnt; ++l) v += q[l] * T[l];
    return v;
}

/* Global maximiser on [-1,1] of v(s) = sum_{l<cnt} q_l T_l(s).
 * Reading: the paper asks for the argmax over the admissible controls and
 * recommends Newton's method without a start, a stopping rule or a rule for
 * the constraint.  The oracle takes the plain definition instead: the
 * candidates are the local maxima of v on [-1,1], that is an endpoint where
 * v' points out of the interval (v'(-1) <= 0, v'(+1) >= 0) and every interior
 * point where v' changes sign from + to -, found on a uniform grid of 16*cnt
 * intervals and refined by bisection of v' down to adjacent doubles; the
 * largest v wins and a tie (within 1e-15 max(1,|v|)) goes to the smaller s.
 * An endpoint where v still increases into the interval is no maximiser, so
 * it is no candidate however close its value comes to the interior maximum.
 * Returns v at the maximiser; *s_star receives the maximiser and *n_crit the
 * number of sign changes of v' seen on the grid (>= 2 flags a non-concave
 * line function). */
real or_argmax_line(int cnt, const real *q, real *s_star, int *n_crit)
{
    real dq[OR_MAXN];
    or_chebder(cnt, q, dq);
    const int G = 16 * cnt;
    int ncr = 0;
    real sa = -1.0, da = or_series(cnt, dq, -1.0);
    int last_sign = (da > 0.0) - (da < 0.0);
    int have = da <= 0.0; /* the left endpoint is a local maximum */
    real best_s = -1.0, best_v = have ? or_series(cnt, q, -1.0) : 0.0;
    for (int g = 1; g <= G; ++g) {
        real sb = -1.0 + 2.0 * (real)g / (real)G;
        real db = or_series(cnt, dq, sb);
        int sgn = (db > 0.0) - (db < 0.0);
        if (sgn != 0) {
            if (last_sign != 0 && sgn != last_sign) ++ncr;
            last_sign = sgn;
        }
        if (da > 0.0 && db <= 0.0) {
            real lo = sa, hi = sb;
            for (int it = 0; it < 200; ++it) {
                real mid = 0.5 * (lo + hi);
                if (mid <= lo || mid >= hi) break;
                if (or_series(cnt, dq, mid) > 0.0) lo = mid; else hi = mid;
            }
            real s = 0.5 * (lo + hi);
            real v = or_series(cnt, q, s);
            if (!have || v > best_v + 1e-15 * fmax(1.0, fabs(best_v))) { best_v = v; best_s = s; have = 1; }
        }
        sa = sb;
        da = db;
    }
    if (da >= 0.0) { /* the right endpoint is a local maximum */
        real v1 = or_series(cnt, q, 1.0);
        if (!have || v1 > best_v + 1e-15 * fmax(1.0, fabs(best_v))) { best_v = v1; best_s = 1.0; have = 1; }
    }
    if (!have) { /* only when v' is not a number: let it reach the value */
        best_s = -1.0;
        best_v = or_series(cnt, q, -1.0) + da;
    }
    *s_star = best_s;
    if (n_crit) *n_crit = ncr;
    return best_v;
}

/* ---------------------------------------------------------------------- */
/* The game (Section 2 and Section 2.1).                                    */

typedef struct {
    int d, N, Nu;                /* players = state dims; nodes per dim; control nodes */
    real h, rho, pmax, umax;
    real K[OR_MAXD * OR_MAXD]; /* exchange matrix, row-major */
    real m[OR_MAXD], c[OR_MAXD], beta[OR_MAXD], A[OR_MAXD], phi[OR_MAXD];
} or_game;

/* Drift g(p,u) of Section 2.1.  Reading: the examples' K has a negative
 * diagonal and positive off-diagonal entries; the drift is taken in the
 * matrix form g_i = (K p)_i / m_i - c_i p_i + beta_i u_i, which is the
 * diffusive exchange sum_{j != i} k_ij (p_j - p_i) / m_i for zero row sums
 * (a more negative diagonal is leakage to the outside). */
static void drift(const or_game *g, const real *p, const real *u, real *out)
{
    for (int i = 0; i < g->d; ++i) {
        real s = 0.0;
        for (int j = 0; j < g->d; ++j) s += g->K[i * g->d + j] * p[j];
        out[i] = s / g->m[i] - g->c[i] * p[i] + g->beta[i] * u[i];
    }
}

/* Instant payoff G_i(p_i, u_i) = u_i (A_i - u_i/2) - phi_i p_i^2 / 2 (LQ
 * specification of Section 2). */
static real payoff(const or_game *g, int i, real p_i, real u_i)
{
    return u_i * (g->A[i] - 0.5 * u_i) - 0.5 * g->phi[i] * p_i * p_i;
}

static long ipow(int b, int e) { long r = 1; while (e-- > 0) r *= b; return r; }

/* Update of one (player i, node j) from the coefficient tensor coef_i of
 * V_i^{[r]} and the controls U^{[r]} (Steps 1-4 of Section 2.1 with the
 * implementation of Section 3.4):
 *   - b = g(p, u^{[r]}(p)) at the node p (physical units);
 *   - for each control node u_m of [0, U_M] the update point is
 *     y = p + h g(p, [u_m, u^{[r]}_{-i}]) = p + h b + h beta_i (u_m - u_i) e_i,
 *     and the sample is h G_i(p_i, u_m) + delta_h V_i^{[r]}(y)
 *     (Reading: the Bellman form of Section 2.1; Steps 2-4 print only the
 *     continuation value, which from V^{[0]} = 0 would keep V = 0);
 *   - the samples are fitted in u by eq. (forcoef) (Algorithm C1v);
 *   - the new control is the global argmax of the fit over [0, U_M] and the
 *     new value is the fit at that control (Step 3, Step 4).
 * 'work' holds N^(d-1) doubles. */
static void update_node(const or_game *g, int i, long j, const real *coef_i,
                        const real *U, const real *xnodes, const real *unodes,
                        real *V_out, real *U_out, int *ncrit, real *work)
{
    int d = g->d, N = g->N, Nu = g->Nu;
    long NN = ipow(N, d);
    int Nd[OR_MAXD];
    real p[OR_MAXD], ubar[OR_MAXD], b[OR_MAXD], y[OR_MAXD], x[OR_MAXD];
    real vals[OR_MAXN], q[OR_MAXN];
    long rem = j;
    for (int l = d - 1; l >= 0; --l) {
        int k = (int)(rem % N);
        rem /= N;
        p[l] = 0.5 * g->pmax * (xnodes[k] + 1.0); /* node mapped to [0, P_M] (Section 3.4) */
        Nd[l] = N;
    }
    for (int l = 0; l < d; ++l) ubar[l] = U[l * NN + j];
    drift(g, p, ubar, b);
    real delta = 1.0 - g->rho * g->h; /* delta_h = 1 - rho h (Section 2.1) */
    for (int m = 0; m < Nu; ++m) {
        for (int l = 0; l < d; ++l) y[l] = p[l] + g->h * b[l];
        y[i] += g->h * g->beta[i] * (unodes[m] - ubar[i]);
        for (int l = 0; l < d; ++l) x[l] = 2.0 * y[l] / g->pmax - 1.0;
        real cont = or_eval_point(d, Nd, coef_i, x, work);
        vals[m] = g->h * payoff(g, i, p[i], unodes[m]) + delta * cont;
    }
    or_coef_1d(Nu, vals, 1, q, 1);
    real s;
    real v = or_argmax_line(Nu, q, &s, ncrit);
    *V_out = v;
    *U_out = 0.5 * g->umax * (s + 1.0); /* s in [-1,1] back to u in [0, U_M] */
}

static void grids(const or_game *g, real *xnodes, real *unodes)
{
    or_nodes(g->N, xnodes);
    real su[OR_MAXN];
    or_nodes(g->Nu, su);
    for (int m = 0; m < g->Nu; ++m) unodes[m] = 0.5 * g->umax * (su[m] + 1.0);
}

/* Coefficients of every player's value tensor (Algorithm Cnv per player). */
static void all_coefs(const or_game *g, const real *V, real *coef)
{
    int Nd[OR_MAXD];
    for (int l = 0; l < g->d; ++l) Nd[l] = g->N;
    long NN = ipow(g->N, g->d);
    for (int i = 0; i < g->d; ++i) or_transform(g->d, Nd, NULL, V + i * NN, coef + i * NN);
}

/* One iteration r -> r+1 for every player and node.  V, U, Vn, Un have shape
 * (d, N^d).  Returns max_{i,j} |Vn - V| (the TOL test of Step 4, on the
 * nodes) and the number of (i,j) whose line function is not concave. */
real or_step(const or_game *g, const real *V, const real *U, real *Vn, real *Un,
               long *n_nonconcave)
{
    int d = g->d;
    long NN = ipow(g->N, d);
    real xnodes[OR_MAXN], unodes[OR_MAXN];
    grids(g, xnodes, unodes);
    real *coef = (real *)malloc(sizeof(real) * (size_t)(d * NN));
    all_coefs(g, V, coef);
    real res = 0.0;
    long nnc = 0;
    long wsz = NN / g->N;
    #pragma omp parallel reduction(max:res) reduction(+:nnc)
    {
        real *work = (real *)malloc(sizeof(real) * (size_t)(wsz > 0 ? wsz : 1));
        #pragma omp for schedule(dynamic, 16)
        for (long t = 0; t < d * NN; ++t) {
            int i = (int)(t / NN);
            long j = t % NN;
            int ncr = 0;
            update_node(g, i, j, coef + i * NN, U, xnodes, unodes, Vn + t, Un + t, &ncr, work);
            if (ncr >= 2) ++nnc;
            real e = fabs(Vn[t] - V[t]);
            if (e > res) res = e;
        }
        free(work);
    }
    free(coef);
    if (n_nonconcave) *n_nonconcave = nnc;
    return res;
}

/* The same update for a list of (player, node) pairs only: used to check
 * large grids on sampled outputs. */
void or_step_sample(const or_game *g, const real *V, const real *U, long count,
                    const int *players, const long *nodes, real *Vn, real *Un)
{
    int d = g->d;
    long NN = ipow(g->N, d);
    real xnodes[OR_MAXN], unodes[OR_MAXN];
    grids(g, xnodes, unodes);
    real *coef = (real *)malloc(sizeof(real) * (size_t)(d * NN));
    all_coefs(g, V, coef);
    long wsz = NN / g->N;
    #pragma omp parallel
    {
        real *work = (real *)malloc(sizeof(real) * (size_t)(wsz > 0 ? wsz : 1));
        #pragma omp for schedule(dynamic, 1)
        for (long t = 0; t < count; ++t) {
            int ncr;
            update_node(g, players[t], nodes[t], coef + players[t] * NN, U, xnodes, unodes,
                        Vn + t, Un + t, &ncr, work);
        }
        free(work);
    }
    free(coef);
}

/* Value iteration from (V, U) for 'steps' iterations, or until the residual
 * drops below tol (strict, Step 4) when tol > 0.  V and U are updated in
 * place; residuals[r] receives the residual of iteration r.  Returns the
 * number of iterations done. */
int or_solve(const or_game *g, real *V, real *U, int steps, real tol, real *residuals)
{
    long n = (long)g->d * ipow(g->N, g->d);
    real *Vn = (real *)malloc(sizeof(real) * (size_t)n);
    real *Un = (real *)malloc(sizeof(real) * (size_t)n);
    int r;
    for (r = 0; r < steps; ++r) {
        long nnc;
        real res = or_step(g, V, U, Vn, Un, &nnc);
        memcpy(V, Vn, sizeof(real) * (size_t)n);
        memcpy(U, Un, sizeof(real) * (size_t)n);
        if (residuals) residuals[r] = res;
        if (tol > 0.0 && res < tol) { ++r; break; }
    }
    free(Vn);
    free(Un);
    return r;
}

/* Equilibrium time paths (the emission and pollution paths of Section 4):
 * from p_0, p_{n+1} = p_n + h g(p_n, u*(p_n)), where u*_i(p) is the
 * Chebyshev interpolant of the nodal controls U_i (Section 3.1) at p, and
 * the payoff-relevant control is kept in [0, U_M].  Reading: the paper plots
 * these paths without stating how they are produced; the explicit Euler
 * step with the scheme's own h and drift is the discrete dynamics the
 * iteration assumes (Section 2.1), and the interpolant of controls that sit
 * on the bounds can leave [0, U_M] between nodes, hence the clip.
 * U has shape (d, N^d); paths (n_steps+1) x d; controls n_steps x d. */
void or_simulate(const or_game *g, const real *U, const real *p0, int n_steps, real *paths,
                 real *controls)
{
    int d = g->d, Nd[OR_MAXD];
    for (int l = 0; l < d; ++l) Nd[l] = g->N;
    long NN = ipow(g->N, d);
    real *coef = (real *)malloc(sizeof(real) * (size_t)(d * NN));
    real *work = (real *)malloc(sizeof(real) * (size_t)(NN / g->N > 0 ? NN / g->N : 1));
    for (int i = 0; i < d; ++i) or_transform(d, Nd, NULL, U + i * NN, coef + i * NN);
    real p[OR_MAXD], u[OR_MAXD], x[OR_MAXD], b[OR_MAXD];
    for (int l = 0; l < d; ++l) p[l] = paths[l] = p0[l];
    for (int n = 0; n < n_steps; ++n) {
        for (int l = 0; l < d; ++l) x[l] = 2.0 * p[l] / g->pmax - 1.0;
        for (int i = 0; i < d; ++i) {
            real v = or_eval_point(d, Nd, coef + i * NN, x, work);
            u[i] = v < 0.0 ? 0.0 : (v > g->umax ? g->umax : v);
            if (controls) controls[n * d + i] = u[i];
        }
        drift(g, p, u, b);
        for (int l = 0; l < d; ++l) {
            p[l] = p[l] + g->h * b[l];
            paths[(n + 1) * d + l] = p[l];
        }
    }
    free(work);
    free(coef);
}

/* ---------------------------------------------------------------------- */
/* The generalised algorithm of Section 2.1 (the form the paper gives for  */
/* dynamics that are not separable in the controls), with anisotropic     */
/* grids N_p, N_u (Step 0) and node-wise control polynomials g^i_p(u)     */
/* (Section 3.3; Step 0 of Section 3.4).                                   */

typedef struct {
    int d;
    int Np[OR_MAXD];   /* Lobatto nodes of each state dimension */
    int Nu[OR_MAXD];   /* control nodes of each player on [0, U_M] */
    real h, rho, pmax, umax;
} or_gen;

/* Update of every player at state node j (Steps 1-4 of the generalised
 * algorithm).  gvals[k][j][.] and pvals[i][j][.] hold, on the tensor grid of
 * control nodes (shape Nu, C order), the drift component k and the payoff
 * of player i at node j.  For each player i:
 *   - Step 0, done here per node: the control polynomials interpolate those
 *     values (Algorithm Cnv over the control modes);
 *   - Step 1: along the line u -> [u, u^{[r]}_{-i}(p_j)] they give the drift
 *     vector and the payoff, evaluated at the control nodes u_m of player i
 *     (the n-d series at the full control vector);
 *   - Step 2: the samples are h G_i + delta_h V_i^{[r]}(p_j + h g(u_m))
 *     (Reading: the Bellman form of Section 2.1 with the payoff, as in the
 *     separable case);
 *   - Steps 3-4: the samples are fitted in u by eq. (forcoef), the new
 *     control is the global argmax of the fit on [0, U_M] and the new value
 *     the fit there.
 * coefV holds the coefficient tensors of V^{[r]} ([d][N_P]), U the controls
 * u^{[r]} ([d][N_P]); vn, un receive the d new values and controls of node
 * j.  'ctl' holds 2 d prod(Nu) doubles, 'work' max(prod(Np), prod(Nu)). */
static void gen_node(const or_gen *g, long j, const real *gvals, const real *pvals,
                     const real *coefV, const real *U, real xn[][OR_MAXN],
                     real un[][OR_MAXN], real *vn, real *un_out, real *ctl, real *work)
{
    int d = g->d;
    long NP = 1, UP = 1;
    for (int l = 0; l < d; ++l) { NP *= g->Np[l]; UP *= g->Nu[l]; }
    real p[OR_MAXD], ubar[OR_MAXD], u[OR_MAXD], yv[OR_MAXD], x[OR_MAXD], gd[OR_MAXD];
    real vals[OR_MAXN], q[OR_MAXN];
    long rem = j;
    for (int l = d - 1; l >= 0; --l) {
        int k = (int)(rem % g->Np[l]);
        rem /= g->Np[l];
        p[l] = 0.5 * g->pmax * (xn[l][k] + 1.0); /* node mapped to [0, P_M] (Section 3.4) */
    }
    for (int l = 0; l < d; ++l) ubar[l] = U[l * NP + j];
    /* Step 0 for this node: drift components 0..d-1, then the payoffs */
    for (int k = 0; k < d; ++k) {
        or_transform(d, g->Nu, NULL, gvals + ((long)k * NP + j) * UP, ctl + (long)k * UP);
        or_transform(d, g->Nu, NULL, pvals + ((long)k * NP + j) * UP, ctl + (long)(d + k) * UP);
    }
    real delta = 1.0 - g->rho * g->h;
    for (int i = 0; i < d; ++i) {
        int nu = g->Nu[i];
        for (int m = 0; m < nu; ++m) {
            for (int l = 0; l < d; ++l) u[l] = ubar[l];
            u[i] = un[i][m];
            for (int l = 0; l < d; ++l) yv[l] = 2.0 * u[l] / g->umax - 1.0;
            for (int k = 0; k < d; ++k) gd[k] = or_eval_point(d, g->Nu, ctl + (long)k * UP, yv, work);
            real G = or_eval_point(d, g->Nu, ctl + (long)(d + i) * UP, yv, work);
            for (int l = 0; l < d; ++l) x[l] = 2.0 * (p[l] + g->h * gd[l]) / g->pmax - 1.0;
            real cont = or_eval_point(d, g->Np, coefV + (long)i * NP, x, work);
            vals[m] = g->h * G + delta * cont;
        }
        or_coef_1d(nu, vals, 1, q, 1);
        real s;
        vn[i] = or_argmax_line(nu, q, &s, NULL);
        un_out[i] = 0.5 * g->umax * (s + 1.0);
    }
}

/* Update of the listed nodes (every node when nodes == NULL, count = N_P).
 * V, U are [d][N_P]; Vn, Un receive [d][count].  Returns the largest
 * |Vn - V| over the listed nodes (the TOL test of Step 4 when all are). */
static real gen_update(const or_gen *g, const real *gvals, const real *pvals, const real *V,
                         const real *U, long count, const long *nodes, real *Vn, real *Un)
{
    int d = g->d;
    long NP = 1, UP = 1;
    for (int l = 0; l < d; ++l) { NP *= g->Np[l]; UP *= g->Nu[l]; }
    real xn[OR_MAXD][OR_MAXN], un[OR_MAXD][OR_MAXN];
    for (int l = 0; l < d; ++l) {
        or_nodes(g->Np[l], xn[l]);
        real su[OR_MAXN];
        or_nodes(g->Nu[l], su);
        for (int m = 0; m < g->Nu[l]; ++m) un[l][m] = 0.5 * g->umax * (su[m] + 1.0);
    }
    real *coefV = (real *)malloc(sizeof(real) * (size_t)(d * NP));
    for (int i = 0; i < d; ++i) or_transform(d, g->Np, NULL, V + i * NP, coefV + i * NP);
    long wsz = NP > UP ? NP : UP;
    real res = 0.0;
    #pragma omp parallel reduction(max:res)
    {
        real *ctl = (real *)malloc(sizeof(real) * (size_t)(2 * d * UP));
        real *work = (real *)malloc(sizeof(real) * (size_t)wsz);
        real vn[OR_MAXD], unn[OR_MAXD];
        #pragma omp for schedule(dynamic, 4)
        for (long t = 0; t < count; ++t) {
            long j = nodes ? nodes[t] : t;
            gen_node(g, j, gvals, pvals, coefV, U, xn, un, vn, unn, ctl, work);
            for (int i = 0; i < d; ++i) {
                Vn[(long)i * count + t] = vn[i];
                Un[(long)i * count + t] = unn[i];
                real e = fabs(vn[i] - V[(long)i * NP + j]);
                if (!(e <= res)) res = e; /* a NaN wins */
            }
        }
        free(work);
        free(ctl);
    }
    free(coefV);
    return res;
}

/* One iteration of the generalised algorithm on every node: V, U, Vn, Un
 * are [d][N_P]; gvals, pvals [d][N_P][prod(Nu)].  Returns max |Vn - V|. */
real or_gen_step(const or_gen *g, const real *gvals, const real *pvals, const real *V,
                   const real *U, real *Vn, real *Un)
{
    long NP = 1;
    for (int l = 0; l < g->d; ++l) NP *= g->Np[l];
    return gen_update(g, gvals, pvals, V, U, NP, NULL, Vn, Un);
}

/* The same update at the listed nodes only (every player of each); Vn, Un
 * receive [d][count].  Used to check large grids on sampled outputs. */
void or_gen_step_sample(const or_gen *g, const real *gvals, const real *pvals, const real *V,
                        const real *U, long count, const long *nodes, real *Vn, real *Un)
{
    gen_update(g, gvals, pvals, V, U, count, nodes, Vn, Un);
}
