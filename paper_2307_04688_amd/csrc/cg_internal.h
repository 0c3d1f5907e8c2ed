// cg_internal.h -- shared declarations of libchebgame's gfx950 kernels and
// the host API that launches them.  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/chebgame.h"

namespace cg {

constexpr int kMaxD = CG_MAX_D;
constexpr int kMaxN = CG_MAX_N;
constexpr int kWave = 64;

typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// Device-resident constants of one game (read through a pointer in the
// workspace; every field is FP64 or int).
struct GameConst {
    int d, N, Nu, N4;          // N4 = N rounded up to a multiple of 4
    int NC;                    // free-mode columns padded to 16 or 32
    int K;                     // contraction length per player (padded)
    long long NN;              // N^d nodes
    double h, rho, pmax, umax, delta;
    double M[kMaxD * kMaxD];   // K / m - diag(c), row-major
    double beta[kMaxD], A[kMaxD], phi[kMaxD];
    double tol;                // convergence threshold of the device test (<= 0: off)
    double xnode[kMaxN];       // Lobatto nodes cos(pi k / (N-1))
    double pnode[kMaxN];       // physical nodes p_max (x + 1) / 2
    double unode[kMaxN];       // control nodes u_max (cos(pi m / (Nu-1)) + 1) / 2
    double Du[kMaxN * kMaxN];  // DCT-I matrix of the control fit, [l][m]
    double Dx[kMaxN * kMaxN];  // DCT-I matrix of the state transform, [l][k]
    double Dd[kMaxN * kMaxN];  // nodal differentiation: derivative at node j of the
                               // interpolant of nodal values, [j][k] (normalised x)
    double TnP[kMaxN * kMaxN * 2];  // basis at the nodes, [j][k][2]: T_k(x_j), T_k'(x_j)
                                    // (k < N; zero past N)
};

// d = 3 mixed contraction: floats per lane of one nodal tensor slab stored
// in MFMA fragment order (lane-contiguous, padded to whole float4 loads).
__host__ __device__ constexpr int corr3_chunk(int N4, int NC) { return ((N4 / 4) * (NC / 16) + 3) & ~3; }

// d = 3 mixed contraction in split bfloat16 form: every binary32 coefficient
// of the packed operand is stored as three bfloat16 pieces (exact sum), and
// the main product runs on bf16 MFMA with K = 32 per step.  Used from N4 = 20
// on; below, the padding of K to 32 costs more than the bf16 rate gains.
__host__ __device__ constexpr bool corr3_split16(int d, int N4) { return d == 3 && N4 >= 20; }
// bf16 elements of the split operand of one player: N outer values x 3
// pieces x (NC / 16) column blocks x 64 lanes x 8
__host__ __device__ constexpr long long split16_player(int N, int NC) { return (long long)N * 3 * (NC / 16) * 512; }

// Per-game device status words.
struct GameStatus {
    double last_res;                 // residual of the last finished step
    int converged;                   // set once a residual < tol (or non-finite): later steps are no-ops
    int steps_done;                  // iterations performed since the last solve started
    int cur;                         // which of the two state buffers holds V^{[r]}, u^{[r]}
    int nonfinite;                   // a non-finite residual was produced
    int total_steps;                 // iterations performed since init
};

// ---- launchers (defined in the .hip files) ----

// Mode-m pass of the DCT-I transform over 'batch' tensors of shape n[0..d-1].
// in and out may alias (the pass loads a whole fiber before writing it).
hipError_t launch_transform_mode(const double *in, double *out, int d, const int *n, int mode,
                                 long long batch, const double *D_dev, hipStream_t s);

// Full transform (d passes) using the DCT matrices for each distinct n.
hipError_t run_transform(int d, const int *n, const double *vals, double *coef, long long batch,
                         hipStream_t s);

// Device pointers of one game instance (host side).
struct InstPtrs {
    const GameConst *gc;
    GameStatus *st;
    double *V, *U;           // [2][d][NN] each
    double *coef, *tmp;      // transform intermediates
    double *Bp;              // packed operand (FP64)
    double *W;               // line coefficients
    float *Bp32;             // packed operand (binary32, FP32_CORR)
    unsigned short *Bs16;    // packed operand split in bfloat16 pieces (FP32_CORR, corr3_split16)
    double *E;               // FP32_CORR Taylor tensors
    double *blk;             // per-block residual maxima of the line kernel
};

// Entry of a device table of instances: the same pointers as byte offsets
// from the table's own address.  Step kernels take a table and serve entry
// blockIdx.x / blocks_per_instance, so that one launch covers every instance
// of a group with the same d and N.  Pointers rebuilt from the table (a
// kernel argument) plus an offset are known to the compiler to be global
// memory, so loads and stores through them are global (not flat) accesses.
struct Inst {
    long long gc, st, V, U, coef, tmp, Bp, W, Bp32, Bs16, E, blk;
};
Inst inst_offsets(const InstPtrs &p, const void *table_dev);

struct InstView {
    const GameConst *gc;
    GameStatus *st;
    double *V, *U, *coef, *tmp, *Bp, *W;
    float *Bp32;
    unsigned short *Bs16;
    double *E, *blk;
};
__device__ __forceinline__ InstView inst_view(const Inst *tab, int k)
{
    const Inst &e = tab[k];
    const char *b = (const char *)tab;
    InstView v;
    v.gc = (const GameConst *)(b + e.gc);
    v.st = (GameStatus *)(b + e.st);
    v.V = (double *)(b + e.V);
    v.U = (double *)(b + e.U);
    v.coef = (double *)(b + e.coef);
    v.tmp = (double *)(b + e.tmp);
    v.Bp = (double *)(b + e.Bp);
    v.W = (double *)(b + e.W);
    v.Bp32 = (float *)(b + e.Bp32);
    v.Bs16 = (unsigned short *)(b + e.Bs16);
    v.E = (double *)(b + e.E);
    v.blk = (double *)(b + e.blk);
    return v;
}

// One value-iteration step of a game (all kernels of Steps 1-4).
struct StepBuffers {
    const GameConst *gc;     // device
    GameStatus *status;      // device
    double *V, *U;           // two state buffers each, [2][d][NN]; status->cur selects
    double *coef;            // d * NN, natural layout (transform intermediate)
    double *tmp;             // d * NN, transform intermediate
    double *Bp;              // d * K * NC packed operand (FP64)
    double *W;               // d * NN * NC line coefficients (contraction output)
    float *Bp32;             // d * K * NC packed operand in binary32 (FP32_CORR)
    unsigned short *Bs16;    // d * split16_player bf16 pieces of it (FP32_CORR, corr3_split16)
    double *E;               // FP32_CORR: [d][d][N^(d-1)][NC] value / first-order tensors
    double *blk;             // per-block residual maxima of the line kernel (d ceil(N^d / 64))
    int precision;
    hipEvent_t ev_begin, ev_end;  // recorded around the contraction kernel when non-null
    const Inst *tab;              // device table of the instances of this launch
    int count;                    // instances in the table (same d, N, precision)
    int rb;                       // rows blocks of 16 per wave in the contraction (1, 2 or 4)
    int ocb;                      // outer-mode values per LDS slab in the contraction (1 or 2)
};
hipError_t launch_transform_game(const GameConst &hc, const StepBuffers &b, hipStream_t s);
// The passes after the first (modes 0..d-3 and the packed operand; none for d = 2).
hipError_t launch_transform_rest(const GameConst &hc, const StepBuffers &b, hipStream_t s);
// First transform pass and Taylor tensors in one launch (mixed path).
hipError_t launch_tf_taylor(const GameConst &hc, const StepBuffers &b, hipStream_t s);
hipError_t launch_step(const GameConst &hc, const StepBuffers &b, hipStream_t s);
hipError_t launch_contract_corr(const GameConst &hc, const StepBuffers &b, hipStream_t s);

hipError_t launch_eval(int d, const int *n, const double *coef, const double *x, long long npts,
                       void *out, int precision, void *ws, size_t ws_bytes, hipStream_t s);
size_t eval_ws_bytes(int d, const int *n, int precision);

// Batched FP64 evaluation of up to kMaxD series of one shape n: member b
// uses packed operand Bp + b bp_stride and the npts[b] points starting at
// row x_off[b] of x (outputs at the same offsets).
struct EvalBatch {
    long long bp_stride;
    long long x_off[kMaxD];
    long long npts[kMaxD];
};
// Elements of one packed FP64 operand of shape n.
size_t eval_packed_elems(int d, const int *n);
// Packs 'count' coefficient tensors (coef + b coef_stride) into Bp + b eval_packed_elems.
hipError_t pack_eval_f64(int d, const int *n, const double *coef, long long count, long long coef_stride,
                         double *Bp, hipStream_t s);
hipError_t eval_f64_batch(int d, const int *n, const double *Bp, const double *x, double *out, const EvalBatch &bt,
                          int count, hipStream_t s);

// One 16 x 16 tile of C = op(A) op(B) (NP x NP, NP = 16 or 32) with both
// operands in LDS (row stride LD doubles, zero beyond the data), on
// v_mfma_f64_16x16x4f64.  Wave w < (NP/16)^2 computes tile (ti, tj) = (w / T,
// w % T); element v of lane r16 + 16 kq holds C[16 ti + kq + 4 v][16 tj + r16].
// TA: A[r][k] is stored at a[k LD + r]; TB: B[k][c] at b[c LD + k].
template <int NP, int LD, bool TA, bool TB>
__device__ __forceinline__ bool plane_mfma(const double *a, const double *b, int wave, int lane, f64x4 &acc, int &ti,
                                           int &tj)
{
    constexpr int T = NP / 16;
    if (wave >= T * T) return false;
    ti = wave / T;
    tj = wave % T;
    const int r16 = lane & 15, kq = lane >> 4;
    const int ra = ti * 16 + r16, cb = tj * 16 + r16;
    acc = f64x4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int ks = 0; ks < NP / 4; ++ks) {
        const int k = ks * 4 + kq;
        const double av = TA ? a[k * LD + ra] : a[ra * LD + k];
        const double bv = TB ? b[cb * LD + k] : b[k * LD + cb];
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc, 0, 0, 0);
    }
    return true;
}

// Accessors of a game handle for the batch code (defined with the handle).
const GameConst &game_consts(const cg_game *g);
const InstPtrs &game_inst(const cg_game *g);
int game_precision(const cg_game *g);
hipStream_t game_stream(const cg_game *g);
// Default contraction tile shapes (row blocks per wave, outer values per slab).
void default_tiles(int d, int N4, long long NN, int precision, int &rb, int &ocb);
// Records an error message for cg_last_error(); returns code.
int set_error(int code, const char *msg);
// CG_OK if the current device is a gfx950, else CG_EDEVICE with a message.
int require_gfx950();

}  // namespace cg
