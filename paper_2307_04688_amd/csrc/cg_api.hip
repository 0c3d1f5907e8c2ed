// cg_api.hip -- host side of the C ABI declared in include/chebgame.h.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "cg_internal.h"

using namespace cg;

namespace {

thread_local std::string g_last_error;

int fail(int code, const char *fmt, ...) __attribute__((format(printf, 2, 3)));
int fail(int code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return code;
}

int hip_fail(hipError_t e, const char *where)
{
    return fail(CG_EDEVICE, "%s: %s", where, hipGetErrorString(e));
}

#define HIP_TRY(call, where)                         \
    do {                                             \
        hipError_t e_ = (call);                      \
        if (e_ != hipSuccess) return hip_fail(e_, where); \
    } while (0)

inline size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

int check_device()
{
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev), "hipGetDevice");
    hipDeviceProp_t prop;
    HIP_TRY(hipGetDeviceProperties(&prop, dev), "hipGetDeviceProperties");
    if (strncmp(prop.gcnArchName, "gfx950", 6) != 0)
        return fail(CG_EDEVICE, "device %d is %s; libchebgame is built for gfx950 only", dev, prop.gcnArchName);
    return CG_OK;
}

struct Layout {
    size_t gc, st, tab, V, U, coef, tmp, Bp, W, Bp32, Bs16, E, blk, total;
};

int validate(const cg_game_desc *g, int precision)
{
    if (!g) return fail(CG_EINVAL, "desc is NULL");
    if (g->d < 2 || g->d > CG_MAX_D) return fail(CG_EUNSUPPORTED, "d = %d outside [2, %d]", g->d, CG_MAX_D);
    if (g->n_nodes < 3 || g->n_nodes > CG_MAX_N)
        return fail(CG_EUNSUPPORTED, "n_nodes = %d outside [3, %d]", g->n_nodes, CG_MAX_N);
    const int nu = g->n_unodes ? g->n_unodes : g->n_nodes;
    if (nu < 3 || nu > CG_MAX_N) return fail(CG_EUNSUPPORTED, "n_unodes = %d outside [3, %d]", nu, CG_MAX_N);
    if (nu > ((g->n_nodes + 3) & ~3))
        return fail(CG_EUNSUPPORTED, "n_unodes = %d above n_nodes rounded up to a multiple of 4", nu);
    if (g->reserved != 0) return fail(CG_EINVAL, "reserved must be 0");
    long long NN = 1;
    for (int l = 0; l < g->d; ++l) NN *= g->n_nodes;
    if (NN > (1LL << 30)) return fail(CG_EUNSUPPORTED, "N^d too large");
    if (!(g->h > 0.0) || !isfinite(g->h)) return fail(CG_EINVAL, "h must be finite and > 0");
    if (!(g->rho * g->h > 0.0 && g->rho * g->h < 1.0)) return fail(CG_EINVAL, "need 0 < rho h < 1");
    if (!(g->p_max > 0.0) || !isfinite(g->p_max)) return fail(CG_EINVAL, "p_max must be finite and > 0");
    if (!(g->u_max > 0.0) || !isfinite(g->u_max)) return fail(CG_EINVAL, "u_max must be finite and > 0");
    if (!g->K || !g->c || !g->beta || !g->A || !g->phi) return fail(CG_EINVAL, "K, c, beta, A, phi are required");
    for (int i = 0; i < g->d * g->d; ++i)
        if (!isfinite(g->K[i])) return fail(CG_EINVAL, "K[%d] is not finite", i);
    for (int i = 0; i < g->d; ++i) {
        if (!isfinite(g->c[i]) || !isfinite(g->beta[i]) || !isfinite(g->A[i]) || !isfinite(g->phi[i]))
            return fail(CG_EINVAL, "parameter of player %d is not finite", i);
        if (g->m && !(g->m[i] > 0.0 && isfinite(g->m[i]))) return fail(CG_EINVAL, "m[%d] must be > 0", i);
    }
    if (precision != CG_FP64 && precision != CG_FP32_CORR)
        return fail(CG_EUNSUPPORTED, "game precision %d not supported (CG_FP64 or CG_FP32_CORR)", precision);
    return CG_OK;
}

void dims(const cg_game_desc *g, int &N4, int &NC, int &K, long long &NN)
{
    const int N = g->n_nodes;
    N4 = (N + 3) & ~3;
    NC = N <= 16 ? 16 : 32;
    K = N4;
    for (int l = 0; l < g->d - 2; ++l) K *= N;
    NN = 1;
    for (int l = 0; l < g->d; ++l) NN *= N;
}

Layout layout(const cg_game_desc *g, int precision)
{
    int N4, NC, K;
    long long NN;
    dims(g, N4, NC, K, NN);
    Layout L;
    size_t o = 0;
    L.gc = o; o = align256(o + sizeof(GameConst));
    L.st = o; o = align256(o + sizeof(GameStatus));
    L.tab = o; o = align256(o + sizeof(Inst));
    L.V = o; o = align256(o + sizeof(double) * 2 * g->d * NN);
    L.U = o; o = align256(o + sizeof(double) * 2 * g->d * NN);
    L.coef = o; o = align256(o + sizeof(double) * g->d * NN);
    L.tmp = o; o = align256(o + sizeof(double) * g->d * NN);
    L.Bp = o; o = align256(o + sizeof(double) * (size_t)g->d * K * NC);
    L.W = o; o = align256(o + sizeof(double) * (size_t)g->d * NN * NC);
    L.blk = o; o = align256(o + sizeof(double) * (size_t)g->d * ((NN + 63) / 64));
    L.Bp32 = L.Bs16 = L.E = 0;
    if (precision == CG_FP32_CORR) {
        L.Bp32 = o; o = align256(o + sizeof(float) * (size_t)g->d * K * NC);
        if (corr3_split16(g->d, N4)) {
            L.Bs16 = o;
            o = align256(o + sizeof(unsigned short) * (size_t)g->d * split16_player(g->n_nodes, NC));
        }
        // Taylor tensors [d][d][N^(d-1)][NC] (FP64), then the d = 3 nodal tensors
        // [d][d-1][N^(d-2)][64 lanes][corr3_chunk] (binary32, fragment order)
        L.E = o; o = align256(o + sizeof(double) * (size_t)g->d * g->d * (NN / g->n_nodes) * NC +
                              sizeof(float) * (size_t)g->d * (g->d - 1) * (NN / g->n_nodes / g->n_nodes) * 64 *
                                  corr3_chunk(N4, NC));
    }
    L.total = o;
    return L;
}

double cos_pi_frac(long long a, long long n)
{
    long long r = a % (2 * n);
    if (r < 0) r += 2 * n;
    return cos(M_PI * (double)r / (double)n);
}

// DCT-I matrix of size N (eq. (forcoef)) into a kMaxN-strided table.
void dct1_matrix(int N, double *D)
{
    const int n = N - 1;
    for (int l = 0; l < N; ++l)
        for (int k = 0; k < N; ++k) {
            double v = cos_pi_frac((long long)l * k, n);
            if (k == 0 || k == n) v *= 0.5;
            D[l * kMaxN + k] = v * ((l == 0 || l == n) ? 1.0 : 2.0) / (double)n;
        }
}

// Nodal differentiation matrix: Dd[j][k] = sum_m T_m'(x_j) Dx[m][k], the
// derivative at node j of the interpolant of values at the nodes.  T_m' by
// the recurrence T'_{m+1} = 2 T_m + 2 x T'_m - T'_{m-1}.
void diff_matrix(int N, const double *Dx, const double *x, double *Dd)
{
    for (int j = 0; j < N; ++j) {
        double T[kMaxN], Tp[kMaxN];
        T[0] = 1.0; Tp[0] = 0.0;
        if (N > 1) { T[1] = x[j]; Tp[1] = 1.0; }
        for (int m = 1; m + 1 < N; ++m) {
            T[m + 1] = 2.0 * x[j] * T[m] - T[m - 1];
            Tp[m + 1] = 2.0 * T[m] + 2.0 * x[j] * Tp[m] - Tp[m - 1];
        }
        for (int k = 0; k < N; ++k) {
            double s = 0.0;
            for (int m = 0; m < N; ++m) s += Tp[m] * Dx[m * kMaxN + k];
            Dd[j * kMaxN + k] = s;
        }
    }
}

// Basis at the nodes: TnP[j][k] = (T_k(x_j), T_k'(x_j)) for k < N, by the
// three-term recurrences in long double from the (double) node x_j, then
// rounded; zero for k >= N and j >= N.
void node_basis(int N, const double *x, double *TnP)
{
    for (int e = 0; e < kMaxN * kMaxN * 2; ++e) TnP[e] = 0.0;
    for (int j = 0; j < N; ++j) {
        const long double xj = x[j];
        long double t0 = 1.0L, t1 = xj, p0 = 0.0L, p1 = 1.0L;
        for (int k = 0; k < N; ++k) {
            double *e = TnP + 2 * (j * kMaxN + k);
            if (k == 0) { e[0] = 1.0; e[1] = 0.0; continue; }
            e[0] = (double)t1;
            e[1] = (double)p1;
            const long double t2 = 2.0L * xj * t1 - t0, p2 = 2.0L * t1 + 2.0L * xj * p1 - p0;
            t0 = t1; t1 = t2; p0 = p1; p1 = p2;
        }
    }
}

}  // namespace

struct cg_game {
    GameConst hc;       // host copy of the constants
    Layout L;
    char *ws;
    hipStream_t stream;
    int precision;
    StepBuffers b;
    InstPtrs inst;      // device pointers of the game
    Inst entry;         // host copy of the one-entry device table
    long long launched; // iterations queued (including no-ops after convergence)
    bool prof;                     // record events around the contraction kernel
    int prof_period;               // ... of every prof_period-th iteration
    long long prof_seen;           // iterations queued since profiling was enabled
    std::vector<hipEvent_t> evs;   // pairs (begin, end), one pair per profiled launch
    size_t ev_used;
    ~cg_game()
    {
        for (hipEvent_t e : evs) (void)hipEventDestroy(e);
    }
};

namespace cg {
void default_tiles(int d, int N4, long long NN, int precision, int &rb, int &ocb)
{
    // measured (contraction per launch): d = 3, N = 32: FP64 fastest at
    // (2, 2), FP32_CORR in the split bfloat16 form at (2, 2) (44.5 against
    // 45.6 us at (1, 2)); d = 3, N = 24: both at (1, 2) (FP64 39.6 against
    // 51.9 us, split 25.1 against 31.0: two row blocks per wave leave 1.3
    // waves per SIMD there); binary32 form at (1, 2); d = 4, N = 24: FP64 at
    // (1, 1), FP32_CORR at (1, 2).  Two row blocks per wave once the game has
    // rows for three such waves per SIMD.
    const long long row_blocks = (long long)d * NN / 16;
    const bool wide = row_blocks >= 2LL * 3 * 1024;
    const bool split = precision == CG_FP32_CORR && corr3_split16(d, N4);
    if (d == 4 || (precision == CG_FP32_CORR && !split))
        rb = 1;
    else
        rb = wide ? 2 : 1;
    ocb = d >= 3 && !(d == 4 && precision != CG_FP32_CORR) ? 2 : 1;
}
const GameConst &game_consts(const cg_game *g) { return g->hc; }
const InstPtrs &game_inst(const cg_game *g) { return g->inst; }
Inst inst_offsets(const InstPtrs &p, const void *table_dev)
{
    const char *b = (const char *)table_dev;
    auto off = [b](const void *q) -> long long { return q ? (long long)((const char *)q - b) : 0; };
    Inst e;
    e.gc = off(p.gc);
    e.st = off(p.st);
    e.V = off(p.V);
    e.U = off(p.U);
    e.coef = off(p.coef);
    e.tmp = off(p.tmp);
    e.Bp = off(p.Bp);
    e.W = off(p.W);
    e.Bp32 = off(p.Bp32);
    e.Bs16 = off(p.Bs16);
    e.E = off(p.E);
    e.blk = off(p.blk);
    return e;
}
int game_precision(const cg_game *g) { return g->precision; }
hipStream_t game_stream(const cg_game *g) { return g->stream; }
int set_error(int code, const char *msg)
{
    g_last_error = msg;
    return code;
}
int require_gfx950() { return check_device(); }
}  // namespace cg

namespace {

__global__ void k_zero(double *p, long long n)
{
    for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (long long)gridDim.x * blockDim.x)
        p[e] = 0.0;
}

__global__ void k_fill_state(double *V, double *U, const GameConst *__restrict__ gc, GameStatus *st)
{
    const long long n = (long long)gc->d * gc->NN;
    for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < 2 * n;
         e += (long long)gridDim.x * blockDim.x) {
        const int i = (int)((e % n) / gc->NN);
        V[e] = 0.0;
        U[e] = gc->A[i];
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        st->last_res = 0.0;
        st->converged = 0;
        st->steps_done = 0;
        st->total_steps = 0;
        st->cur = 0;
        st->nonfinite = 0;
    }
}

__global__ void k_set_state(double *V, double *U, const double *Vin, const double *Uin,
                            const GameConst *__restrict__ gc, GameStatus *st)
{
    const long long n = (long long)gc->d * gc->NN;
    const int cur = st->cur;
    for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < n;
         e += (long long)gridDim.x * blockDim.x) {
        V[cur * n + e] = Vin[e];
        U[cur * n + e] = Uin ? Uin[e] : gc->A[(int)(e / gc->NN)];
    }
}

__global__ void k_get_state(const double *V, const double *U, double *Vout, double *Uout,
                            const GameConst *__restrict__ gc, const GameStatus *st)
{
    const long long n = (long long)gc->d * gc->NN;
    const int cur = st->cur;
    for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < n;
         e += (long long)gridDim.x * blockDim.x) {
        if (Vout) Vout[e] = V[cur * n + e];
        if (Uout) Uout[e] = U[cur * n + e];
    }
}

// Reset the convergence test (and set its threshold) before a solve.
__global__ void k_arm(GameConst *gc, GameStatus *st, double tol, int clear_done)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        gc->tol = tol;
        st->converged = 0;
        st->nonfinite = 0;
        if (clear_done) st->steps_done = 0;
    }
}

int read_status(cg_game *g, GameStatus &out)
{
    HIP_TRY(hipMemcpyAsync(&out, g->ws + g->L.st, sizeof(GameStatus), hipMemcpyDeviceToHost, g->stream),
            "hipMemcpyAsync(status)");
    HIP_TRY(hipStreamSynchronize(g->stream), "hipStreamSynchronize");
    return CG_OK;
}

int queue_steps(cg_game *g, int n)
{
    for (int s = 0; s < n; ++s) {
        StepBuffers b = g->b;
        if (g->prof && (g->prof_seen++ % g->prof_period) == 0) {
            if (g->ev_used + 2 > g->evs.size()) {
                for (int k = 0; k < 256; ++k) {
                    hipEvent_t e;
                    HIP_TRY(hipEventCreate(&e), "hipEventCreate");
                    g->evs.push_back(e);
                }
            }
            b.ev_begin = g->evs[g->ev_used];
            b.ev_end = g->evs[g->ev_used + 1];
            g->ev_used += 2;
        }
        hipError_t e = launch_step(g->hc, b, g->stream);
        if (e != hipSuccess) return hip_fail(e, "step launch");
    }
    g->launched += n;
    return CG_OK;
}

// Constants of a game description (Step 0: grids, matrices, parameters).
void build_consts(const cg_game_desc *g, GameConst &hc)
{
    memset(&hc, 0, sizeof hc);
    const int d = g->d, N = g->n_nodes, Nu = g->n_unodes ? g->n_unodes : g->n_nodes;
    hc.d = d;
    hc.N = N;
    hc.Nu = Nu;
    dims(g, hc.N4, hc.NC, hc.K, hc.NN);
    hc.h = g->h;
    hc.rho = g->rho;
    hc.pmax = g->p_max;
    hc.umax = g->u_max;
    hc.delta = 1.0 - g->rho * g->h;
    for (int i = 0; i < d; ++i) {
        const double mi = g->m ? g->m[i] : 1.0;
        for (int j = 0; j < d; ++j) hc.M[i * d + j] = g->K[i * d + j] / mi - (i == j ? g->c[i] : 0.0);
        hc.beta[i] = g->beta[i];
        hc.A[i] = g->A[i];
        hc.phi[i] = g->phi[i];
    }
    hc.tol = 0.0;
    for (int k = 0; k < N; ++k) {
        hc.xnode[k] = cos_pi_frac(k, N - 1);
        hc.pnode[k] = 0.5 * g->p_max * (hc.xnode[k] + 1.0);
    }
    for (int m = 0; m < Nu; ++m) hc.unode[m] = 0.5 * g->u_max * (cos_pi_frac(m, Nu - 1) + 1.0);
    dct1_matrix(Nu, hc.Du);
    dct1_matrix(N, hc.Dx);
    diff_matrix(N, hc.Dx, hc.xnode, hc.Dd);
    node_basis(N, hc.xnode, hc.TnP);
}

}  // namespace

extern "C" {

const char *cg_last_error(void) { return g_last_error.c_str(); }

const char *cg_strerror(int status)
{
    switch (status) {
        case CG_OK: return "ok";
        case CG_ENOTCONVERGED: return "tolerance not reached within max_steps";
        case CG_EINVAL: return "invalid argument";
        case CG_EUNSUPPORTED: return "size or precision not supported";
        case CG_EDEVICE: return "HIP device error";
        case CG_ENOMEM: return "workspace too small";
        case CG_ENONFINITE: return "non-finite value in the iterate";
    }
    return "unknown status";
}

size_t cg_workspace_bytes(const cg_game_desc *desc, int precision)
{
    if (validate(desc, precision) != CG_OK) return 0;
    return layout(desc, precision).total;
}

int cg_init_game(const cg_game_desc *g, int precision, void *ws_dev, size_t ws_bytes, void *stream,
                 cg_game **out)
{
    if (!out) return fail(CG_EINVAL, "out is NULL");
    *out = nullptr;
    int rc = validate(g, precision);
    if (rc != CG_OK) return rc;
    rc = check_device();
    if (rc != CG_OK) return rc;
    Layout L = layout(g, precision);
    if (!ws_dev) return fail(CG_EINVAL, "workspace is NULL");
    if (((uintptr_t)ws_dev & 255) != 0) return fail(CG_EINVAL, "workspace must be 256-byte aligned");
    if (ws_bytes < L.total) return fail(CG_ENOMEM, "workspace has %zu bytes, needs %zu", ws_bytes, L.total);

    cg_game *G = new (std::nothrow) cg_game();
    if (!G) return fail(CG_ENOMEM, "host allocation failed");
    GameConst &hc = G->hc;
    build_consts(g, hc);

    G->L = L;
    G->ws = (char *)ws_dev;
    G->stream = (hipStream_t)stream;
    G->precision = precision;
    G->launched = 0;
    StepBuffers &b = G->b;
    b.gc = (const GameConst *)(G->ws + L.gc);
    b.status = (GameStatus *)(G->ws + L.st);
    b.V = (double *)(G->ws + L.V);
    b.U = (double *)(G->ws + L.U);
    b.coef = (double *)(G->ws + L.coef);
    b.tmp = (double *)(G->ws + L.tmp);
    b.Bp = (double *)(G->ws + L.Bp);
    b.W = (double *)(G->ws + L.W);
    b.Bp32 = precision == CG_FP32_CORR ? (float *)(G->ws + L.Bp32) : nullptr;
    b.Bs16 = L.Bs16 ? (unsigned short *)(G->ws + L.Bs16) : nullptr;
    b.E = precision == CG_FP32_CORR ? (double *)(G->ws + L.E) : nullptr;
    b.blk = (double *)(G->ws + L.blk);
    b.precision = precision;
    b.ev_begin = b.ev_end = nullptr;
    b.tab = (const Inst *)(G->ws + L.tab);
    b.count = 1;
    default_tiles(hc.d, hc.N4, hc.NN, precision, b.rb, b.ocb);
    InstPtrs &hi = G->inst;
    hi.gc = b.gc;
    hi.st = b.status;
    hi.V = b.V;
    hi.U = b.U;
    hi.coef = b.coef;
    hi.tmp = b.tmp;
    hi.Bp = b.Bp;
    hi.W = b.W;
    hi.Bp32 = b.Bp32;
    hi.Bs16 = b.Bs16;
    hi.E = b.E;
    hi.blk = b.blk;
    G->prof = false;
    G->prof_period = 1;
    G->prof_seen = 0;
    G->ev_used = 0;

    hipError_t e = hipMemcpyAsync(G->ws + L.gc, &hc, sizeof hc, hipMemcpyHostToDevice, G->stream);
    G->entry = inst_offsets(G->inst, G->ws + L.tab);
    if (e == hipSuccess) e = hipMemcpyAsync(G->ws + L.tab, &G->entry, sizeof(Inst), hipMemcpyHostToDevice, G->stream);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_fill_state, dim3(256), dim3(256), 0, G->stream, b.V, b.U, b.gc, b.status);
        e = hipGetLastError();
    }
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_zero, dim3(256), dim3(256), 0, G->stream, b.Bp, (long long)hc.d * hc.K * hc.NC);
        e = hipGetLastError();
    }
    if (e == hipSuccess && b.Bp32) {
        // binary32 operand: zero it through a double view (its size is a multiple of 2 floats)
        hipLaunchKernelGGL(k_zero, dim3(256), dim3(256), 0, G->stream, (double *)b.Bp32,
                           (long long)hc.d * hc.K * hc.NC / 2);
        e = hipGetLastError();
    }
    if (e == hipSuccess && b.Bs16) {  // padding pieces stay zero (4 bf16 per double)
        hipLaunchKernelGGL(k_zero, dim3(256), dim3(256), 0, G->stream, (double *)b.Bs16,
                           (long long)hc.d * split16_player(hc.N, hc.NC) / 4);
        e = hipGetLastError();
    }
    if (e == hipSuccess && b.E) {
        hipLaunchKernelGGL(k_zero, dim3(256), dim3(256), 0, G->stream, b.E,
                           (long long)hc.d * hc.d * (hc.NN / hc.N) * hc.NC);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipStreamSynchronize(G->stream);  // hc and inst must outlive the copies
    if (e != hipSuccess) {
        delete G;
        return hip_fail(e, "cg_init_game");
    }
    *out = G;
    return CG_OK;
}

int cg_destroy(cg_game *game)
{
    delete game;
    return CG_OK;
}

int cg_reset_game(cg_game *G, const cg_game_desc *g)
{
    if (!G) return fail(CG_EINVAL, "game is NULL");
    int rc = validate(g, G->precision);
    if (rc != CG_OK) return rc;
    const int Nu = g->n_unodes ? g->n_unodes : g->n_nodes;
    if (g->d != G->hc.d || g->n_nodes != G->hc.N || Nu != G->hc.Nu)
        return fail(CG_EINVAL, "reset needs the same d, n_nodes and control nodes (%d, %d, %d)", G->hc.d, G->hc.N,
                    G->hc.Nu);
    GameConst hc;
    build_consts(g, hc);
    hc.tol = 0.0;
    HIP_TRY(hipMemcpyAsync(G->ws + G->L.gc, &hc, sizeof hc, hipMemcpyHostToDevice, G->stream),
            "hipMemcpyAsync(constants)");
    hipLaunchKernelGGL(k_fill_state, dim3(256), dim3(256), 0, G->stream, G->b.V, G->b.U, G->b.gc, G->b.status);
    HIP_TRY(hipGetLastError(), "reset launch");
    HIP_TRY(hipStreamSynchronize(G->stream), "hipStreamSynchronize");  // hc must outlive the copy
    G->hc = hc;
    return CG_OK;
}

int cg_chebyshev_transform(int d, const int32_t *n, const double *vals_dev, double *coef_dev, int64_t batch,
                           void *stream)
{
    if (d < 1 || d > CG_MAX_D) return fail(CG_EUNSUPPORTED, "d = %d outside [1, %d]", d, CG_MAX_D);
    if (batch < 0) return fail(CG_EINVAL, "batch < 0");
    if (!n || (batch > 0 && (!vals_dev || !coef_dev))) return fail(CG_EINVAL, "NULL argument");
    int nn[kMaxD];
    for (int l = 0; l < d; ++l) {
        if (n[l] < 2 || n[l] > CG_MAX_N) return fail(CG_EUNSUPPORTED, "n[%d] = %d outside [2, %d]", l, n[l], CG_MAX_N);
        nn[l] = n[l];
    }
    if (batch > 0 && vals_dev == coef_dev) return fail(CG_EINVAL, "vals and coef must not overlap");
    int rc = check_device();
    if (rc != CG_OK) return rc;
    if (batch == 0) return CG_OK;
    HIP_TRY(run_transform(d, nn, vals_dev, coef_dev, batch, (hipStream_t)stream), "transform launch");
    return CG_OK;
}

size_t cg_eval_workspace_bytes(int d, const int32_t *n, int precision)
{
    if (d < 1 || d > CG_MAX_D || !n) return 0;
    int nn[kMaxD];
    for (int l = 0; l < d; ++l) nn[l] = n[l];
    return eval_ws_bytes(d, nn, precision);
}

// Scratch of cg_chebyshev_eval_noalloc: the packed coefficient operand of the
// evaluation.  Sized for the largest operand of the compiled set (d = 4,
// N = 32, FP64: 32^3 rows of 32 doubles, plus the 256 bytes of slack every
// evaluation workspace carries), 8 MiB + 256 B per GPU, held until the
// process ends.  The packing kernel writes every element the evaluation
// reads, so nothing has to be cleared between calls.  Host code never uses
// the array's name as an address: each device's address comes from
// hipGetSymbolAddress (eval_scratch_ptr).
constexpr size_t kEvalScratchBytes = (size_t)32 * 32 * 32 * 32 * 8 + 256;
static __device__ __align__(256) unsigned char scratch[kEvalScratchBytes];

namespace {

// Arguments shared by cg_chebyshev_eval and cg_chebyshev_eval_noalloc; copies
// the sizes into nn.
int check_eval_args(int d, const int32_t *n, const double *coef_dev, const double *x_dev, int64_t npts,
                    const void *out_dev, int precision, int *nn)
{
    if (d < 1 || d > CG_MAX_D) return fail(CG_EUNSUPPORTED, "d = %d outside [1, %d]", d, CG_MAX_D);
    if (npts < 0) return fail(CG_EINVAL, "npts < 0");
    if (!n || !coef_dev || (npts > 0 && (!x_dev || !out_dev))) return fail(CG_EINVAL, "NULL argument");
    if (precision != CG_FP64 && precision != CG_FP32 && precision != CG_BF16 && precision != CG_FP32_SPLIT)
        return fail(CG_EUNSUPPORTED, "eval precision %d not supported", precision);
    for (int l = 0; l < d; ++l) {
        if (n[l] < 2 || n[l] > CG_MAX_N) return fail(CG_EUNSUPPORTED, "n[%d] = %d outside [2, %d]", l, n[l], CG_MAX_N);
        nn[l] = n[l];
    }
    return CG_OK;
}

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

// Device address of 'scratch' on the current device, looked up once per
// device (with that device current) and kept.
int eval_scratch_ptr(void **out)
{
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev), "hipGetDevice");
    if (dev < 0 || dev >= kMaxDevices) return fail(CG_EDEVICE, "device %d beyond %d devices", dev, kMaxDevices);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)), "hipGetSymbolAddress(scratch)");
        if (!p) return fail(CG_EDEVICE, "hipGetSymbolAddress(scratch) returned NULL");
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return CG_OK;
}

}  // namespace

int cg_chebyshev_eval(int d, const int32_t *n, const double *coef_dev, const double *x_dev, int64_t npts,
                      void *out_dev, int precision, void *ws_dev, size_t ws_bytes, void *stream)
{
    int nn[kMaxD];
    int rc = check_eval_args(d, n, coef_dev, x_dev, npts, out_dev, precision, nn);
    if (rc != CG_OK) return rc;
    const size_t need = eval_ws_bytes(d, nn, precision);
    if (need > 0 && (!ws_dev || ws_bytes < need))
        return fail(CG_ENOMEM, "eval workspace has %zu bytes, needs %zu", ws_dev ? ws_bytes : 0, need);
    if (need > 0 && ((uintptr_t)ws_dev & 255) != 0) return fail(CG_EINVAL, "workspace must be 256-byte aligned");
    rc = check_device();
    if (rc != CG_OK) return rc;
    HIP_TRY(launch_eval(d, nn, coef_dev, x_dev, npts, out_dev, precision, ws_dev, ws_bytes, (hipStream_t)stream),
            "eval launch");
    return CG_OK;
}

int cg_chebyshev_eval_noalloc(int d, const int32_t *n, const double *coef_dev, const double *x_dev, int64_t npts,
                              void *out_dev, int precision, void *stream)
{
    int nn[kMaxD];
    int rc = check_eval_args(d, n, coef_dev, x_dev, npts, out_dev, precision, nn);
    if (rc != CG_OK) return rc;
    const size_t need = eval_ws_bytes(d, nn, precision);
    if (need > kEvalScratchBytes)
        return fail(CG_EUNSUPPORTED, "eval needs %zu bytes of scratch, the static scratch holds %zu", need,
                    kEvalScratchBytes);
    rc = check_device();
    if (rc != CG_OK) return rc;
    void *ws = nullptr;
    rc = eval_scratch_ptr(&ws);
    if (rc != CG_OK) return rc;
    HIP_TRY(launch_eval(d, nn, coef_dev, x_dev, npts, out_dev, precision, ws, kEvalScratchBytes,
                        (hipStream_t)stream),
            "eval launch");
    return CG_OK;
}

int cg_step(cg_game *g, int32_t nsteps, double *residual_out)
{
    if (!g) return fail(CG_EINVAL, "game is NULL");
    if (nsteps < 0) return fail(CG_EINVAL, "nsteps < 0");
    hipLaunchKernelGGL(k_arm, dim3(1), dim3(64), 0, g->stream, (GameConst *)g->b.gc, g->b.status, 0.0, 0);
    HIP_TRY(hipGetLastError(), "arm launch");
    int rc = queue_steps(g, nsteps);
    if (rc != CG_OK) return rc;
    if (residual_out) {
        GameStatus st;
        rc = read_status(g, st);
        if (rc != CG_OK) return rc;
        *residual_out = st.last_res;
        if (st.nonfinite) return fail(CG_ENONFINITE, "non-finite residual after %d steps", st.steps_done);
    }
    return CG_OK;
}

int cg_solve(cg_game *g, int32_t max_steps, double tol, int32_t *steps_done, double *residual)
{
    if (!g) return fail(CG_EINVAL, "game is NULL");
    if (max_steps < 0) return fail(CG_EINVAL, "max_steps < 0");
    if (!(tol == tol)) return fail(CG_EINVAL, "tol is NaN");
    hipLaunchKernelGGL(k_arm, dim3(1), dim3(64), 0, g->stream, (GameConst *)g->b.gc, g->b.status,
                       tol > 0.0 ? tol : 0.0, 1);
    HIP_TRY(hipGetLastError(), "arm launch");
    GameStatus st;
    int rc;
    if (tol <= 0.0) {
        rc = queue_steps(g, max_steps);
        if (rc != CG_OK) return rc;
        rc = read_status(g, st);
        if (rc != CG_OK) return rc;
    } else {
        // queue in chunks; the device-side test turns the tail of a chunk into no-ops
        int queued = 0;
        const int chunk = 32;
        for (;;) {
            const int n = max_steps - queued < chunk ? max_steps - queued : chunk;
            rc = queue_steps(g, n);
            if (rc != CG_OK) return rc;
            queued += n;
            rc = read_status(g, st);
            if (rc != CG_OK) return rc;
            if (st.converged || queued >= max_steps) break;
        }
    }
    if (steps_done) *steps_done = st.steps_done;
    if (residual) *residual = st.last_res;
    if (st.nonfinite) return fail(CG_ENONFINITE, "non-finite residual after %d steps", st.steps_done);
    if (tol > 0.0 && !st.converged) return CG_ENOTCONVERGED;
    return CG_OK;
}

int cg_get_state(cg_game *g, double *V_dev, double *U_dev, int32_t *r)
{
    if (!g) return fail(CG_EINVAL, "game is NULL");
    if (V_dev || U_dev) {
        hipLaunchKernelGGL(k_get_state, dim3(256), dim3(256), 0, g->stream, g->b.V, g->b.U, V_dev, U_dev, g->b.gc,
                           g->b.status);
        HIP_TRY(hipGetLastError(), "get_state launch");
    }
    if (r) {
        GameStatus st;
        int rc = read_status(g, st);
        if (rc != CG_OK) return rc;
        *r = st.total_steps;
    }
    return CG_OK;
}

int cg_set_tiles(cg_game *g, int32_t rb, int32_t ocb)
{
    if (!g) return fail(CG_EINVAL, "game is NULL");
    if (!(rb == 1 || rb == 2 || rb == 4)) return fail(CG_EINVAL, "rb must be 1, 2 or 4");
    if (!(ocb == 1 || (ocb == 2 && g->hc.d >= 3))) return fail(CG_EINVAL, "ocb must be 1 (or 2 when d >= 3)");
    g->b.rb = rb;
    g->b.ocb = ocb;
    return CG_OK;
}

int cg_profile(cg_game *g, int enable, double *kernel_ms, int64_t *launches)
{
    if (!g) return fail(CG_EINVAL, "game is NULL");
    if (kernel_ms || launches) {
        HIP_TRY(hipStreamSynchronize(g->stream), "hipStreamSynchronize");
        double tot = 0.0;
        for (size_t k = 0; k + 1 < g->ev_used; k += 2) {
            float ms = 0.f;
            HIP_TRY(hipEventElapsedTime(&ms, g->evs[k], g->evs[k + 1]), "hipEventElapsedTime");
            tot += ms;
        }
        if (kernel_ms) *kernel_ms = tot;
        if (launches) *launches = (int64_t)(g->ev_used / 2);
    }
    if (enable < 0) return fail(CG_EINVAL, "enable < 0");
    g->prof = enable != 0;
    g->prof_period = enable > 0 ? enable : 1;
    g->prof_seen = 0;
    g->ev_used = 0;
    return CG_OK;
}

int cg_set_state(cg_game *g, const double *V_dev, const double *U_dev)
{
    if (!g) return fail(CG_EINVAL, "game is NULL");
    if (!V_dev) return fail(CG_EINVAL, "V is NULL");
    hipLaunchKernelGGL(k_set_state, dim3(256), dim3(256), 0, g->stream, g->b.V, g->b.U, V_dev, U_dev, g->b.gc,
                       g->b.status);
    HIP_TRY(hipGetLastError(), "set_state launch");
    hipLaunchKernelGGL(k_arm, dim3(1), dim3(64), 0, g->stream, (GameConst *)g->b.gc, g->b.status, 0.0, 0);
    HIP_TRY(hipGetLastError(), "arm launch");
    return CG_OK;
}

}  // extern "C"
