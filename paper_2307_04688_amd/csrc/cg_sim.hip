// cg_sim.hip -- equilibrium time paths (the emission and pollution paths the
// paper plots in Section 4): from p_0, p_{n+1} = p_n + h g(p_n, u*(p_n)), with
// u*_i the Chebyshev interpolant of the game's nodal controls U_i evaluated
// at p (Section 3.1) and kept in [0, U_M].
#include <stdio.h>

#include "cg_internal.h"

using namespace cg;

namespace {

// One block per path.  Per step: thread l < d builds T_0..T_{N-1} of mode l at
// the current point in LDS; every thread sums coefficient terms e = tid +
// 256 k of every player (coalesced); a fixed-order tree reduction gives the
// interpolated controls; thread 0 clips them and takes the Euler step.
template <int D>
__global__ __launch_bounds__(256) void k_simulate(const GameConst *__restrict__ gc, const double *__restrict__ coefU,
                                                  const double *__restrict__ p0, int n_steps,
                                                  double *__restrict__ paths, double *__restrict__ controls)
{
    __shared__ double T[D][kMaxN];
    __shared__ double red[D][256];
    __shared__ double p[D];
    const int path = blockIdx.x, tid = threadIdx.x;
    const int N = gc->N;
    const long long NN = gc->NN;
    double *out = paths + (long long)path * (n_steps + 1) * D;
    if (tid < D) {
        p[tid] = p0[(long long)path * D + tid];
        out[tid] = p[tid];
    }
    __syncthreads();
    for (int n = 0; n < n_steps; ++n) {
        if (tid < D) {
            const double x = 2.0 * p[tid] / gc->pmax - 1.0;
            double tm = 1.0, tc = x;
            T[tid][0] = 1.0;
            for (int k = 1; k < N; ++k) {
                T[tid][k] = tc;
                const double tn = 2.0 * x * tc - tm;
                tm = tc;
                tc = tn;
            }
        }
        __syncthreads();
        double acc[D];
#pragma unroll
        for (int i = 0; i < D; ++i) acc[i] = 0.0;
        for (long long e = tid; e < NN; e += 256) {
            long long rem = e;
            double prod = 1.0;
#pragma unroll
            for (int l = D - 1; l >= 0; --l) {
                prod *= T[l][(int)(rem % N)];
                rem /= N;
            }
#pragma unroll
            for (int i = 0; i < D; ++i) acc[i] = fma(coefU[i * NN + e], prod, acc[i]);
        }
#pragma unroll
        for (int i = 0; i < D; ++i) red[i][tid] = acc[i];
        __syncthreads();
        for (int w = 128; w > 0; w >>= 1) {
            if (tid < w) {
#pragma unroll
                for (int i = 0; i < D; ++i) red[i][tid] += red[i][tid + w];
            }
            __syncthreads();
        }
        if (tid == 0) {
            double u[D], pn[D];
#pragma unroll
            for (int i = 0; i < D; ++i) {
                const double v = red[i][0];
                u[i] = v < 0.0 ? 0.0 : (v > gc->umax ? gc->umax : v);
                if (controls) controls[((long long)path * n_steps + n) * D + i] = u[i];
            }
#pragma unroll
            for (int i = 0; i < D; ++i) {
                double s = 0.0;
#pragma unroll
                for (int j = 0; j < D; ++j) s = fma(gc->M[i * D + j], p[j], s);
                pn[i] = p[i] + gc->h * fma(gc->beta[i], u[i], s);
            }
#pragma unroll
            for (int i = 0; i < D; ++i) {
                p[i] = pn[i];
                out[(long long)(n + 1) * D + i] = pn[i];
            }
        }
        __syncthreads();
    }
}

}  // namespace

extern "C" int cg_simulate(cg_game *game, const double *p0_dev, int32_t n_paths, int32_t n_steps, double *paths_dev,
                           double *controls_dev)
{
    if (!game) return set_error(CG_EINVAL, "game is NULL");
    if (n_paths < 0 || n_steps < 0) return set_error(CG_EINVAL, "n_paths < 0 or n_steps < 0");
    if (n_paths == 0) return CG_OK;
    if (!p0_dev || !paths_dev) return set_error(CG_EINVAL, "p0 or paths is NULL");
    const GameConst &hc = game_consts(game);
    const InstPtrs &I = game_inst(game);
    hipStream_t s = game_stream(game);
    // controls of the current iterate -> coefficient tensors (in the game's transform buffer)
    int rc = cg_get_state(game, nullptr, I.coef, nullptr);
    if (rc != CG_OK) return rc;
    int n[CG_MAX_D];
    for (int l = 0; l < hc.d; ++l) n[l] = hc.N;
    hipError_t e = run_transform(hc.d, n, I.coef, I.coef, hc.d, s);
    if (e == hipSuccess) {
        switch (hc.d) {
            case 2:
                hipLaunchKernelGGL(k_simulate<2>, dim3(n_paths), dim3(256), 0, s, I.gc, I.coef, p0_dev, n_steps,
                                   paths_dev, controls_dev);
                break;
            case 3:
                hipLaunchKernelGGL(k_simulate<3>, dim3(n_paths), dim3(256), 0, s, I.gc, I.coef, p0_dev, n_steps,
                                   paths_dev, controls_dev);
                break;
            default:
                hipLaunchKernelGGL(k_simulate<4>, dim3(n_paths), dim3(256), 0, s, I.gc, I.coef, p0_dev, n_steps,
                                   paths_dev, controls_dev);
                break;
        }
        e = hipGetLastError();
    }
    if (e != hipSuccess) {
        char buf[200];
        snprintf(buf, sizeof buf, "simulate: %s", hipGetErrorString(e));
        return set_error(CG_EDEVICE, buf);
    }
    return CG_OK;
}
