/*
 * sanitize_main.c -- driver that runs every entry point of the oracle on
 * small inputs, for a build under AddressSanitizer and
 * UndefinedBehaviorSanitizer (tests/test_oracle_sanitize.py compiles it with
 * gcc -fsanitize=address,undefined and runs it).  The oracle's source is
 * included, so the driver sees its structs and static helpers.
 *
 * TEST INFRASTRUCTURE ONLY: it checks memory and undefined-behaviour errors,
 * not values (the value pins are the Python tests).
 */
#include "oracle.c"

#include <stdio.h>

static real *alloc(long n)
{
    real *p = (real *)malloc(sizeof(real) * (size_t)(n > 0 ? n : 1));
    for (long i = 0; i < n; ++i) p[i] = (real)0.25 * (real)((i * 7919) % 13) / (real)13 - (real)0.1;
    return p;
}

static void game(or_game *g, int d, int N, int Nu)
{
    memset(g, 0, sizeof *g);
    g->d = d;
    g->N = N;
    g->Nu = Nu;
    g->h = 0.01;
    g->rho = 0.1;
    g->pmax = 1.0;
    g->umax = 1.0;
    for (int i = 0; i < d; ++i) {
        for (int j = 0; j < d; ++j) g->K[i * d + j] = (i == j) ? -(real)(d - 1) : (real)1;
        g->m[i] = 1.0;
        g->c[i] = 0.5;
        g->beta[i] = 1.0;
        g->A[i] = 0.5;
        g->phi[i] = 1.0;
    }
}

int main(void)
{
    /* one-dimensional pieces up to the largest node count */
    for (int N = 1; N <= 32; N += 31) {
        real *x = alloc(N), *F = alloc(N), *p = alloc(N), *q = alloc(N), *T = alloc(N);
        or_nodes(N, x);
        or_cheb_T(N, (real)0.3, T);
        or_coef_1d(N, F, 1, p, 1);
        or_chebder(N, p, q);
        (void)or_series(N, p, (real)-1.0);
        real s;
        int nc;
        (void)or_argmax_line(N, p, &s, &nc);
        free(x); free(F); free(p); free(q); free(T);
    }
    /* n-dimensional transform and evaluation, anisotropic, d = 1..4 */
    const int shapes[4][4] = {{9, 1, 1, 1}, {5, 4, 1, 1}, {4, 6, 3, 1}, {3, 4, 3, 5}};
    for (int d = 1; d <= 4; ++d) {
        long total = 1;
        for (int l = 0; l < d; ++l) total *= shapes[d - 1][l];
        real *v = alloc(total), *c = alloc(total), *pts = alloc(7 * d), *out = alloc(7);
        const int order[4] = {3 % d, 1 % d, 2 % d, 0};
        or_transform(d, shapes[d - 1], NULL, v, c);
        if (d == 4) or_transform(d, shapes[d - 1], order, v, c);
        or_eval(d, shapes[d - 1], c, pts, 7, out);
        free(v); free(c); free(pts); free(out);
    }
    /* the game: steps, sampled step, solve, equilibrium paths, d = 2..4 */
    const int gs[3][3] = {{2, 5, 5}, {3, 4, 3}, {4, 3, 3}};
    for (int k = 0; k < 3; ++k) {
        or_game g;
        game(&g, gs[k][0], gs[k][1], gs[k][2]);
        long NN = ipow(g.N, g.d), n = (long)g.d * NN;
        real *V = alloc(n), *U = alloc(n), *Vn = alloc(n), *Un = alloc(n), *res = alloc(3);
        for (long i = 0; i < n; ++i) U[i] = (real)0.5;
        long nnc;
        (void)or_step(&g, V, U, Vn, Un, &nnc);
        int players[4] = {0, g.d - 1, 1, 0};
        long nodes[4] = {0, NN - 1, NN / 2, 1};
        real vs[4], us[4];
        or_step_sample(&g, V, U, 4, players, nodes, vs, us);
        (void)or_solve(&g, V, U, 3, 0.0, res);
        real p0[4] = {0.2, 0.4, 0.6, 0.8}, *paths = alloc(6 * g.d), *ctrl = alloc(5 * g.d);
        or_simulate(&g, U, p0, 5, paths, ctrl);
        free(V); free(U); free(Vn); free(Un); free(res); free(paths); free(ctrl);
    }
    /* the general form, anisotropic state and control grids */
    {
        or_gen g;
        memset(&g, 0, sizeof g);
        g.d = 3;
        const int Np[3] = {4, 3, 5}, Nu[3] = {3, 4, 3};
        for (int l = 0; l < 3; ++l) { g.Np[l] = Np[l]; g.Nu[l] = Nu[l]; }
        g.h = 0.01; g.rho = 0.1; g.pmax = 1.0; g.umax = 1.0;
        long NP = 4 * 3 * 5, UP = 3 * 4 * 3;
        real *gv = alloc(3 * NP * UP), *pv = alloc(3 * NP * UP), *V = alloc(3 * NP), *U = alloc(3 * NP);
        real *Vn = alloc(3 * NP), *Un = alloc(3 * NP), *Vs = alloc(3 * 2), *Us = alloc(3 * 2);
        for (long i = 0; i < 3 * NP; ++i) U[i] = (real)0.5;
        (void)or_gen_step(&g, gv, pv, V, U, Vn, Un);
        long nodes[2] = {0, NP - 1};
        or_gen_step_sample(&g, gv, pv, V, U, 2, nodes, Vs, Us);
        free(gv); free(pv); free(V); free(U); free(Vn); free(Un); free(Vs); free(Us);
    }
    printf("sanitize: ok (%d threads)\n", or_num_threads());
    return 0;
}
