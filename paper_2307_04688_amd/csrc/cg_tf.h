// cg_tf.h -- device code of the coefficient transform: the DCT-I matrix
// entries, the first pass of the game transform (the two fastest modes of
// every N x N slice) and the packed-operand index, shared by the transform
// launches and the fused transform + Taylor kernel of the mixed path.
#pragma once

#include "cg_internal.h"

namespace cg {

// Entry (l, k) of the DCT-I matrix of one mode of size N (n = N - 1):
// (w_l / n) e_k cos(pi l k / n), w_0 = w_n = 1 else 2, e_0 = e_n = 1/2 else 1.
__device__ inline double dct1_entry(int l, int k, int N)
{
    const int n = N - 1;
    const int r = (l * k) % (2 * n);
    double v = cospi((double)r / (double)n);
    if (k == 0 || k == n) v *= 0.5;
    return v * ((l == 0 || l == n) ? 1.0 : 2.0) / (double)n;
}

__device__ __forceinline__ long long packed_index(const GameConst *__restrict__ gc, int i, const int *dig)
{
    const int d = gc->d, N = gc->N;
    const int lastother = (i == d - 1) ? d - 2 : d - 1;
    int col = 0, kl = 0, kout = 0;
    for (int l = 0; l < d; ++l) {
        if (l == i) col = dig[l];
        else if (l == lastother) kl = dig[l];
        else kout = kout * N + dig[l];
    }
    return ((long long)i * gc->K + (long long)kout * gc->N4 + kl) * gc->NC + col;
}

// Split form of the d = 3 packed operand (corr3_split16): element
// (k_o, k_n, k_i) of player i, rounded to binary32, as three bfloat16 pieces
// whose sum is that binary32 value exactly (each piece takes the leading bits
// of what the previous ones left; 3 x 8 significand bits cover 24).  Order:
// MFMA fragments of v_mfma_f32_16x16x32_bf16 with k_n as the K index, per
// (player, k_o, piece, column block k_i / 16) 64 lanes x 8 elements, element
// (k_n, k_i) in lane (k_n mod 4) 16 + k_i mod 16 at position k_n / 4.
__device__ __forceinline__ void store_split16(unsigned short *__restrict__ Bs, const GameConst *__restrict__ gc, int i,
                                              const int *dig, double v)
{
    const int ko = dig[i == 0 ? 1 : 0], kn = dig[i == 2 ? 1 : 2], ki = dig[i];
    const int NCB = gc->NC / 16;
    const long long frag0 = ((long long)i * gc->N + ko) * 3 * NCB + (ki >> 4);
    const int slot = ((kn & 3) * 16 + (ki & 15)) * 8 + (kn >> 2);
    float r = (float)v;
#pragma unroll
    for (int p = 0; p < 3; ++p) {
        const __bf16 h = (__bf16)r;
        Bs[(frag0 + (long long)p * NCB) * 512 + slot] = __builtin_bit_cast(unsigned short, h);
        r -= (float)h;
    }
}

// Body of the first transform pass for block 'bid' (sm: 3 kMaxN (kMaxN + 1)
// doubles of LDS), shared by k_tf_fast and the fused pass + Taylor kernel.
template <int NP>
__device__ __forceinline__ void tf_fast_block(const Inst *__restrict__ tab, int bpi, int mixed, int bid, double *sm)
{
    const InstView I = inst_view(tab, bid / bpi);
    const int blk = bid % bpi;
    const GameConst *__restrict__ gc = I.gc;
    const GameStatus *st = I.st;
    const double *Vbuf = I.V;
    double *out = I.tmp, *Bp = I.Bp;
    float *Bp32 = mixed ? I.Bp32 : nullptr;
    constexpr int LD = kMaxN + 1;  // odd stride: column reads hit distinct banks
    double *Dm = sm, *X = sm + kMaxN * LD, *Y = sm + 2 * kMaxN * LD;
    if (st->converged) return;
    const int N = gc->N, d = gc->d, NN2 = N * N;
    const long long NN = gc->NN;
    const int nslice = (int)(NN / NN2);
    const int i = blk / nslice, sl = blk % nslice;
    const double *src = Vbuf + (long long)st->cur * d * NN + (long long)i * NN + (long long)sl * NN2;
    for (int e = threadIdx.x; e < NP * NP; e += blockDim.x) {  // zero beyond N
        const int r = e / NP, c = e % NP;
        const bool in = r < N && c < N;
        Dm[r * LD + c] = in ? gc->Dx[r * kMaxN + c] : 0.0;
        X[r * LD + c] = in ? src[r * N + c] : 0.0;
    }
    __syncthreads();
    // Y = D X (mode d-2), then Z = Y D^T (mode d-1), on FP64 MFMA
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int r16 = lane & 15, kq = lane >> 4;
    f64x4 acc;
    int ti, tj;
    if (plane_mfma<NP, LD, false, false>(Dm, X, wave, lane, acc, ti, tj)) {
#pragma unroll
        for (int v = 0; v < 4; ++v) Y[(ti * 16 + kq + 4 * v) * LD + tj * 16 + r16] = acc[v];
    }
    __syncthreads();
    if (plane_mfma<NP, LD, false, true>(Y, Dm, wave, lane, acc, ti, tj)) {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int r = ti * 16 + kq + 4 * v, c = tj * 16 + r16;
            if (r >= N || c >= N) continue;
            if (d > 2) {
                out[(long long)i * NN + (long long)sl * NN2 + r * N + c] = acc[v];
            } else {
                int dig[kMaxD] = {r, c, 0, 0};
                const long long o = packed_index(gc, i, dig);
                if (Bp32) Bp32[o] = (float)acc[v]; else Bp[o] = acc[v];
            }
        }
    }
}


}  // namespace cg
