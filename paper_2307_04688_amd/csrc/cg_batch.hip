// cg_batch.hip -- batched value iteration over many games (C ABI part of
// include/chebgame.h): grouping, device tables, one captured iteration
// (groups spread over parallel graph branches) replayed as a hipGraph, and
// the tile autotuner.
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <new>
#include <vector>

#include "cg_internal.h"

using namespace cg;

namespace {

// Parallel branches of the captured iteration: groups are spread over up to
// this many capture streams that fork from and join into one stream, so the
// replayed graph runs independent groups concurrently (the runtime maps graph
// branches to its hardware queues).
constexpr int kBranches = 4;

struct Group {
    GameConst hc;              // constants of the first game (d, N, sizes)
    int precision;
    std::vector<int> members;  // indices into the batch's game list
    size_t tab_off;            // byte offset of the group's table in the workspace
    int rb;                    // row blocks of 16 per wave in the contraction
    int ocb;                   // outer-mode values per LDS slab in the contraction
};

inline size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

int hip_err(hipError_t e, const char *where)
{
    char buf[256];
    snprintf(buf, sizeof buf, "%s: %s", where, hipGetErrorString(e));
    return set_error(CG_EDEVICE, buf);
}

// Per-game state words gathered for one host copy.
struct StatusCopy {
    double last_res;
    int converged, steps_done, nonfinite, pad;
};

__global__ void k_batch_arm(const Inst *__restrict__ tab, int count, double tol, int clear_done)
{
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= count) return;
    const InstView I = inst_view(tab, g);
    GameConst *gc = const_cast<GameConst *>(I.gc);
    GameStatus *st = I.st;
    gc->tol = tol;
    st->converged = 0;
    st->nonfinite = 0;
    if (clear_done) st->steps_done = 0;
}

__global__ void k_batch_gather(const Inst *__restrict__ tab, int count, StatusCopy *out)
{
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= count) return;
    const GameStatus *st = inst_view(tab, g).st;
    out[g].last_res = st->last_res;
    out[g].converged = st->converged;
    out[g].steps_done = st->steps_done;
    out[g].nonfinite = st->nonfinite;
    out[g].pad = 0;
}

// Zero terminal value V = 0, u = A, status cleared, for every game.
__global__ void k_batch_reset(const Inst *__restrict__ tab, int count)
{
    const int g = blockIdx.y;
    if (g >= count) return;
    const InstView I = inst_view(tab, g);
    const GameConst *gc = I.gc;
    const long long n = (long long)gc->d * gc->NN;
    for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < 2 * n;
         e += (long long)gridDim.x * blockDim.x) {
        I.V[e] = 0.0;
        I.U[e] = gc->A[(int)((e % n) / gc->NN)];
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        GameStatus *st = I.st;
        st->last_res = 0.0;
        st->converged = 0;
        st->steps_done = 0;
        st->cur = 0;
        st->nonfinite = 0;
    }
}

}  // namespace

struct cg_batch {
    std::vector<cg_game *> games;
    std::vector<Group> groups;
    char *ws;
    size_t all_tab_off;        // table of every game (for arm / gather / reset)
    size_t status_off;         // StatusCopy[count]
    hipStream_t stream;        // caller's stream
    hipStream_t cap;           // private stream used for capture only (branch 0)
    hipStream_t side[kBranches - 1];   // capture streams of the other branches
    hipEvent_t fork, join[kBranches - 1];
    hipGraph_t graph;
    hipGraphExec_t exec;
    bool have_graph;
    int branches;              // parallel branches of the captured iteration
    int max_branches;          // at most this many (the autotuner's choice; kBranches before)
    std::vector<int> branch_of;  // per group
    std::vector<StatusCopy> host_status;
    ~cg_batch()
    {
        if (have_graph) {
            (void)hipGraphExecDestroy(exec);
            (void)hipGraphDestroy(graph);
        }
        if (cap) (void)hipStreamDestroy(cap);
        for (int b = 0; b < kBranches - 1; ++b) {
            if (side[b]) (void)hipStreamDestroy(side[b]);
            if (join[b]) (void)hipEventDestroy(join[b]);
        }
        if (fork) (void)hipEventDestroy(fork);
    }
};

namespace {

StepBuffers group_buffers(cg_batch *B, const Group &G)
{
    StepBuffers b;
    memset(&b, 0, sizeof b);
    b.precision = G.precision;
    b.tab = (const Inst *)(B->ws + G.tab_off);
    b.count = (int)G.members.size();
    b.rb = G.rb;
    b.ocb = G.ocb;
    return b;
}

// Queue one iteration of every group on stream s (autotuning, one branch).
hipError_t queue_iteration(cg_batch *B, hipStream_t s)
{
    for (const Group &G : B->groups) {
        hipError_t e = launch_step(G.hc, group_buffers(B, G), s);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

// Relative cost of one iteration of a group: its contraction flops, with a
// floor for the latency of its launches.
double group_cost(const Group &G)
{
    const double flops = (double)G.members.size() * G.hc.d * 2.0 * (double)G.hc.NN * (double)G.hc.NN / G.hc.N;
    return flops + 2e8;
}

// Groups to branches: largest first, each to the currently cheapest branch.
void assign_branches(cg_batch *B)
{
    const int ng = (int)B->groups.size();
    B->branches = std::min(B->max_branches, ng);
    B->branch_of.assign(ng, 0);
    std::vector<double> load(B->branches, 0.0);
    for (int g = 0; g < ng; ++g) {  // groups are sorted largest first
        int best = 0;
        for (int b = 1; b < B->branches; ++b)
            if (load[b] < load[best]) best = b;
        B->branch_of[g] = best;
        load[best] += group_cost(B->groups[g]);
    }
}

// One iteration captured with branch b's groups on its own stream, forked
// from and joined into the capture stream.
hipError_t capture_iteration(cg_batch *B)
{
    hipError_t e = hipSuccess;
    if (B->branches > 1) {
        e = hipEventRecord(B->fork, B->cap);
        for (int b = 1; b < B->branches && e == hipSuccess; ++b) e = hipStreamWaitEvent(B->side[b - 1], B->fork, 0);
    }
    for (size_t g = 0; g < B->groups.size() && e == hipSuccess; ++g) {
        const int b = B->branch_of[g];
        e = launch_step(B->groups[g].hc, group_buffers(B, B->groups[g]), b == 0 ? B->cap : B->side[b - 1]);
    }
    for (int b = 1; b < B->branches && e == hipSuccess; ++b) {
        e = hipEventRecord(B->join[b - 1], B->side[b - 1]);
        if (e == hipSuccess) e = hipStreamWaitEvent(B->cap, B->join[b - 1], 0);
    }
    return e;
}

int build_graph(cg_batch *B)
{
    if (B->have_graph) {
        (void)hipGraphExecDestroy(B->exec);
        (void)hipGraphDestroy(B->graph);
        B->have_graph = false;
    }
    assign_branches(B);
    hipError_t e = hipStreamBeginCapture(B->cap, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return hip_err(e, "hipStreamBeginCapture");
    hipError_t eq = capture_iteration(B);
    e = hipStreamEndCapture(B->cap, &B->graph);
    if (eq != hipSuccess) return hip_err(eq, "capture of one iteration");
    if (e != hipSuccess) return hip_err(e, "hipStreamEndCapture");
    e = hipGraphInstantiate(&B->exec, B->graph, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        (void)hipGraphDestroy(B->graph);
        return hip_err(e, "hipGraphInstantiate");
    }
    B->have_graph = true;
    return CG_OK;
}

int read_statuses(cg_batch *B)
{
    const int n = (int)B->games.size();
    hipLaunchKernelGGL(k_batch_gather, dim3((n + 127) / 128), dim3(128), 0, B->stream,
                       (const Inst *)(B->ws + B->all_tab_off), n, (StatusCopy *)(B->ws + B->status_off));
    hipError_t e = hipGetLastError();
    if (e == hipSuccess)
        e = hipMemcpyAsync(B->host_status.data(), B->ws + B->status_off, sizeof(StatusCopy) * n,
                           hipMemcpyDeviceToHost, B->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(B->stream);
    return e == hipSuccess ? CG_OK : hip_err(e, "batch status");
}

}  // namespace

extern "C" {

size_t cg_batch_workspace_bytes(int32_t count)
{
    if (count < 1) return 0;
    // one table entry per game twice (group tables + the full table) + status copies
    return align256(sizeof(Inst) * (size_t)count) * 2 + CG_MAX_GROUPS * 256 +
           align256(sizeof(StatusCopy) * (size_t)count) + 256;
}

int cg_batch_create(cg_game *const *games, int32_t count, void *ws_dev, size_t ws_bytes, void *stream,
                    cg_batch **out)
{
    if (!out) return set_error(CG_EINVAL, "out is NULL");
    *out = nullptr;
    if (!games || count < 1) return set_error(CG_EINVAL, "need at least one game");
    if (!ws_dev || ((uintptr_t)ws_dev & 255)) return set_error(CG_EINVAL, "workspace NULL or not 256-byte aligned");
    if (ws_bytes < cg_batch_workspace_bytes(count)) return set_error(CG_ENOMEM, "batch workspace too small");
    for (int i = 0; i < count; ++i) {
        if (!games[i]) return set_error(CG_EINVAL, "NULL game in the batch");
        for (int j = 0; j < i; ++j)
            if (games[j] == games[i]) return set_error(CG_EINVAL, "a game appears twice in the batch");
    }
    cg_batch *B = new (std::nothrow) cg_batch();
    if (!B) return set_error(CG_ENOMEM, "host allocation failed");
    B->games.assign(games, games + count);
    B->ws = (char *)ws_dev;
    B->stream = (hipStream_t)stream;
    B->cap = nullptr;
    B->fork = nullptr;
    for (int b = 0; b < kBranches - 1; ++b) {
        B->side[b] = nullptr;
        B->join[b] = nullptr;
    }
    B->have_graph = false;
    B->branches = 1;
    B->max_branches = kBranches;
    B->host_status.resize(count);
    // group by (d, N, control-fit path, precision)
    for (int i = 0; i < count; ++i) {
        const GameConst &hc = game_consts(games[i]);
        const int prec = game_precision(games[i]);
        Group *found = nullptr;
        for (Group &G : B->groups)
            if (G.hc.d == hc.d && G.hc.N == hc.N && (G.hc.Nu >= G.hc.N) == (hc.Nu >= hc.N) && G.precision == prec)
                found = &G;
        if (!found) {
            if ((int)B->groups.size() >= CG_MAX_GROUPS) {
                delete B;
                return set_error(CG_EUNSUPPORTED, "too many (d, N, precision) groups in one batch");
            }
            Group G;
            G.hc = hc;
            G.precision = prec;
            default_tiles(hc.d, hc.N4, hc.NN, prec, G.rb, G.ocb);
            G.tab_off = 0;
            B->groups.push_back(G);
            found = &B->groups.back();
        }
        found->members.push_back(i);
    }
    // largest groups first in the launch order
    std::stable_sort(B->groups.begin(), B->groups.end(), [](const Group &a, const Group &b) {
        return a.hc.NN * a.hc.d * (long long)a.members.size() > b.hc.NN * b.hc.d * (long long)b.members.size();
    });
    // device tables: one per group, then the full one, then the status copies
    std::vector<Inst> host_tab;
    size_t off = 0;
    std::vector<std::pair<size_t, std::vector<Inst>>> uploads;
    for (Group &G : B->groups) {
        G.tab_off = off;
        std::vector<Inst> t;
        for (int m : G.members) t.push_back(inst_offsets(game_inst(games[m]), B->ws + G.tab_off));
        off = align256(off + sizeof(Inst) * t.size());
        uploads.push_back({G.tab_off, t});
    }
    B->all_tab_off = off;
    {
        std::vector<Inst> t;
        for (int i = 0; i < count; ++i) t.push_back(inst_offsets(game_inst(games[i]), B->ws + off));
        uploads.push_back({off, t});
        off = align256(off + sizeof(Inst) * t.size());
    }
    B->status_off = off;
    hipError_t e = hipSuccess;
    for (auto &u : uploads) {
        e = hipMemcpyAsync(B->ws + u.first, u.second.data(), sizeof(Inst) * u.second.size(), hipMemcpyHostToDevice,
                           B->stream);
        if (e != hipSuccess) break;
    }
    if (e == hipSuccess) e = hipStreamSynchronize(B->stream);  // host tables go out of scope
    // capture streams (default priority) and the fork / join events
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&B->cap, hipStreamNonBlocking);
    for (int b = 0; b < kBranches - 1 && e == hipSuccess; ++b) {
        e = hipStreamCreateWithFlags(&B->side[b], hipStreamNonBlocking);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&B->join[b], hipEventDisableTiming);
    }
    if (e == hipSuccess) e = hipEventCreateWithFlags(&B->fork, hipEventDisableTiming);
    if (e != hipSuccess) {
        delete B;
        return hip_err(e, "cg_batch_create");
    }
    *out = B;
    return CG_OK;
}

int cg_batch_autotune(cg_batch *B, int32_t trial_steps)
{
    if (!B) return set_error(CG_EINVAL, "batch is NULL");
    if (trial_steps < 1) return set_error(CG_EINVAL, "trial_steps < 1");
    const int n = (int)B->games.size();
    const Inst *all = (const Inst *)(B->ws + B->all_tab_off);
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess) return set_error(CG_EDEVICE, "hipEventCreate");
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return set_error(CG_EDEVICE, "hipEventCreate");
    }
    int rc = CG_OK;
    hipLaunchKernelGGL(k_batch_arm, dim3((n + 127) / 128), dim3(128), 0, B->stream, all, n, 0.0, 1);
    for (Group &G : B->groups) {
        const int cands[6][2] = {{1, 1}, {2, 1}, {4, 1}, {1, 2}, {2, 2}, {4, 2}};
        float best = 1e30f;
        int best_rb = G.rb, best_ocb = G.ocb;
        for (const auto &cnd : cands) {
            if (cnd[1] == 2 && G.hc.d < 3) continue;  // one outer value when d = 2
            G.rb = cnd[0];
            G.ocb = cnd[1];
            StepBuffers b = group_buffers(B, G);
            hipError_t e = launch_step(G.hc, b, B->stream);  // warm-up
            if (e == hipSuccess) e = hipEventRecord(e0, B->stream);
            for (int s = 0; s < trial_steps && e == hipSuccess; ++s) e = launch_step(G.hc, b, B->stream);
            if (e == hipSuccess) e = hipEventRecord(e1, B->stream);
            if (e == hipSuccess) e = hipEventSynchronize(e1);
            float ms = 0.f;
            if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
            if (e != hipSuccess) {
                rc = hip_err(e, "autotune");
                break;
            }
            if (ms < best) {
                best = ms;
                best_rb = G.rb;
                best_ocb = G.ocb;
            }
        }
        G.rb = best_rb;
        G.ocb = best_ocb;
        if (rc != CG_OK) break;
    }
    // then the parallel branches of the captured iteration: trial_steps
    // replays of the graph with 1 .. kBranches branches; more branches are
    // kept only when at least 2 % faster
    const int nb_max = std::min(kBranches, (int)B->groups.size());
    float best_t = 1e30f;
    int best_nb = nb_max;
    for (int nb = 1; nb <= nb_max && rc == CG_OK; ++nb) {
        B->max_branches = nb;
        rc = build_graph(B);
        if (rc != CG_OK) break;
        hipError_t e = hipGraphLaunch(B->exec, B->stream);  // warm-up
        if (e == hipSuccess) e = hipEventRecord(e0, B->stream);
        for (int s = 0; s < trial_steps && e == hipSuccess; ++s) e = hipGraphLaunch(B->exec, B->stream);
        if (e == hipSuccess) e = hipEventRecord(e1, B->stream);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        float ms = 0.f;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
        if (e != hipSuccess) {
            rc = hip_err(e, "autotune branches");
            break;
        }
        if (ms < 0.98f * best_t) {
            best_t = ms;
            best_nb = nb;
        }
    }
    B->max_branches = best_nb;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc != CG_OK) return rc;
    // back to the zero terminal value
    long long maxn = 0;
    for (const Group &G : B->groups) maxn = std::max(maxn, (long long)G.hc.d * G.hc.NN);
    dim3 grid((unsigned)std::min<long long>((2 * maxn + 255) / 256, 1024), (unsigned)n);
    hipLaunchKernelGGL(k_batch_reset, grid, dim3(256), 0, B->stream, all, n);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = hipStreamSynchronize(B->stream);
    if (e != hipSuccess) return hip_err(e, "autotune reset");
    return build_graph(B);
}

int cg_batch_solve(cg_batch *B, int32_t max_steps, double tol, int32_t *steps_done, double *residuals)
{
    if (!B) return set_error(CG_EINVAL, "batch is NULL");
    if (max_steps < 0) return set_error(CG_EINVAL, "max_steps < 0");
    if (!(tol == tol)) return set_error(CG_EINVAL, "tol is NaN");
    if (!B->have_graph) {
        int rc = build_graph(B);
        if (rc != CG_OK) return rc;
    }
    const int n = (int)B->games.size();
    hipLaunchKernelGGL(k_batch_arm, dim3((n + 127) / 128), dim3(128), 0, B->stream,
                       (const Inst *)(B->ws + B->all_tab_off), n, tol > 0.0 ? tol : 0.0, 1);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_err(e, "batch arm");
    int queued = 0;
    const int chunk = tol > 0.0 ? 32 : max_steps;
    int rc = CG_OK;
    for (;;) {
        const int m = std::min(chunk, max_steps - queued);
        for (int s = 0; s < m; ++s) {
            e = hipGraphLaunch(B->exec, B->stream);
            if (e != hipSuccess) return hip_err(e, "hipGraphLaunch");
        }
        queued += m;
        rc = read_statuses(B);
        if (rc != CG_OK) return rc;
        bool all_done = true;
        for (int g = 0; g < n; ++g) all_done &= B->host_status[g].converged != 0;
        if (queued >= max_steps || (tol > 0.0 && all_done) || m == 0) break;
    }
    bool nonfinite = false, notconv = false;
    for (int g = 0; g < n; ++g) {
        const StatusCopy &s = B->host_status[g];
        if (steps_done) steps_done[g] = s.steps_done;
        if (residuals) residuals[g] = s.last_res;
        nonfinite |= s.nonfinite != 0;
        notconv |= !s.converged;
    }
    if (nonfinite) return set_error(CG_ENONFINITE, "a game of the batch produced a non-finite value");
    if (tol > 0.0 && notconv) return CG_ENOTCONVERGED;
    return CG_OK;
}

int cg_batch_groups(cg_batch *B, int32_t *rb, int32_t *ocb)
{
    if (!B) return set_error(CG_EINVAL, "batch is NULL");
    for (size_t i = 0; i < B->groups.size(); ++i) {
        if (rb) rb[i] = B->groups[i].rb;
        if (ocb) ocb[i] = B->groups[i].ocb;
    }
    return (int)B->groups.size();
}

int cg_batch_branches(cg_batch *B)
{
    if (!B) return set_error(CG_EINVAL, "batch is NULL");
    if (!B->have_graph) {
        int rc = build_graph(B);
        if (rc != CG_OK) return rc;
    }
    return B->branches;
}

int cg_batch_destroy(cg_batch *B)
{
    delete B;
    return CG_OK;
}

}  // extern "C"
