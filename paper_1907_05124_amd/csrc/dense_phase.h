// Field product of one dense update phase on the fp32 matrix cores, with the
// annealing update fused into the epilogue (device code; included by the
// library's dense translation unit).
//
// Phi[P, runs] = J[P, :] * M[:, runs] for the spins P = [p0, p1) of the phase
// (Algorithm 1's Phi_i = sum_j J_ij s_j), then m = tanh(Phi / T) per run.
//
// Workgroup tile: 128 spins x 128 runs; K (all N spins) streamed in slabs of
// 32 through double-buffered LDS.  The WM x WN waves each own a
// (128/WM) x (128/WN) sub-tile made of 32 x 32 blocks of the 32x32x2 fp32
// MFMA.  J is symmetric, so the slab J[k0:k0+32, i0:i0+128] read row-wise is
// the transposed A tile: both operands arrive as [k][128] rows with
// coalesced 16-byte loads and sit in LDS k-major, where every MFMA operand
// read is 32 consecutive floats per half-wave.  The fragments of half a slab
// are read from LDS into registers before its MFMAs are issued, so LDS
// latency overlaps the matrix pipeline instead of preceding every MFMA.
//
// Accumulation: the matrix cores add each slab's 32 products per element in
// fp32; the slab's sum is then added to an fp64 total and the fp32
// accumulator restarts at zero.  The rounding of the field thus grows with
// the 16 additions of one slab instead of the N/2 additions of the whole row
// (for N = 2000, about 4 units in the last place of the field instead of
// ~30), which keeps the fp32 form's trajectories close to an fp64 evaluation
// of Algorithm 1 through the low temperatures of the last levels, where 1/T
// amplifies every change of the field.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace mars {

typedef float floatx16 __attribute__((ext_vector_type(16)));

constexpr int DBM = 128, DBN = 128, DBK = 32;


// RAW: instead of the update, write the field Phi = J M + h/2 of the
// phase's rows to phi (same layout as M) for a sequential pass over them.
// invT64 (or null): the runs' 1/T in fp64 (same layout as invT); with it the
// update's argument (Phi + h/2) / T is formed in fp64 from the fp64 field and
// rounded once before the fp32 tanh.
// One workgroup tile (tile index `tile` of the phase's nrt x nct grid).
// skip (or null): per 128-run column block, nonzero = leave the tile out (its
// runs are all frozen and both state buffers already hold their values).
template <int WM, int WN, int PF, bool RAW>
__device__ __forceinline__ void dense_phase_f32_tile(
    const float *__restrict__ J, int ldj, const float *__restrict__ Mold, float *__restrict__ Mnew, int ldm, int R,
    int p0, int p1, int a0, int nrt, int nct, int kpad, const float *__restrict__ invT,
    const double *__restrict__ invT64, const float *__restrict__ hhalf, float gamma, uint32_t *__restrict__ dmax,
    float *__restrict__ phi, int tile, const int32_t *__restrict__ skip)
{
    constexpr int NT = 64 * WM * WN;
    constexpr int TM = DBM / WM, TN = DBN / WN;  // wave sub-tile
    constexpr int MB = TM / 32, NB = TN / 32;    // 32x32 blocks per wave
    constexpr int LPT = (DBK * DBM / 4) / NT;    // float4 loads per thread per operand
    constexpr int ROWS_PER_PASS = NT / 32;       // slab rows covered by one pass of the threads
    static_assert(MB >= 1 && NB >= 1 && LPT >= 1, "tile shape");
    static_assert(PF == 1 || PF == 2, "prefetch distance");

    __shared__ float As[2][DBK][DBM];
    __shared__ float Bs[2][DBK][DBN];

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int wm = wave / WN, wn = wave % WN;

    // Tiles are ordered so that the workgroups resident on one XCD (the
    // hardware deals workgroups round-robin over the 8 XCDs) share a band of
    // run columns: each XCD's L2 then holds its own slice of M plus the
    // phase's J rows, instead of every XCD streaming all of M.
    const int total = nrt * nct;
    int t = tile;
    if ((total & 7) == 0)
        t = (t & 7) * (total >> 3) + (t >> 3);
    const int rt = t % nrt, ct = t / nrt;
    if (skip && skip[ct])
        return;
    const int i0 = a0 + rt * DBM;
    const int c0 = ct * DBN;

    floatx16 acc[MB][NB];
    double tot[MB][NB][16];
#pragma unroll
    for (int a = 0; a < MB; ++a)
#pragma unroll
        for (int b = 0; b < NB; ++b)
#pragma unroll
            for (int v = 0; v < 16; ++v) {
                acc[a][b][v] = 0.0f;
                tot[a][b][v] = 0.0;
            }

    const int lrow = tid >> 5;        // slab row of this thread's first load
    const int lcol = (tid & 31) * 4;  // column (float4 granularity)
    const int nk = kpad / DBK;
    const int ka = lane >> 5;  // which k of the MFMA's pair this lane supplies
    const int li = lane & 31;

    // Global slab loads go through registers: set X holds slab t when t is
    // even, set Y when t is odd.  With PF = 2 the loads of slab t+2 are issued
    // while slab t is multiplied, so each load has two slabs of matrix work
    // to arrive; with PF = 1 they are issued one slab ahead.
    float4 xa[LPT], xb[LPT], ya[LPT], yb[LPT];
#define DP_LOAD(RA, RB, k0)                                                                                   \
    _Pragma("unroll") for (int q = 0; q < LPT; ++q)                                                           \
    {                                                                                                         \
        const int row_ = (k0) + lrow + ROWS_PER_PASS * q;                                                     \
        RA[q] = *reinterpret_cast<const float4 *>(J + (size_t)row_ * ldj + i0 + lcol);                        \
        RB[q] = *reinterpret_cast<const float4 *>(((row_ < p0) ? Mnew : Mold) + (size_t)row_ * ldm + c0 + lcol); \
    }
#define DP_STORE(RA, RB, buf)                                                                                 \
    _Pragma("unroll") for (int q = 0; q < LPT; ++q)                                                           \
    {                                                                                                         \
        *reinterpret_cast<float4 *>(&As[(buf)][lrow + ROWS_PER_PASS * q][lcol]) = RA[q];                      \
        *reinterpret_cast<float4 *>(&Bs[(buf)][lrow + ROWS_PER_PASS * q][lcol]) = RB[q];                      \
    }
#define DP_MMA(buf)                                                                                           \
    {                                                                                                         \
        _Pragma("unroll") for (int hk = 0; hk < 2; ++hk)                                                      \
        {                                                                                                     \
            float fa_[DBK / 4][MB], fb_[DBK / 4][NB];                                                         \
            _Pragma("unroll") for (int kk = 0; kk < DBK / 4; ++kk)                                            \
            {                                                                                                 \
                const int kr_ = 2 * (hk * (DBK / 4) + kk) + ka;                                               \
                _Pragma("unroll") for (int a = 0; a < MB; ++a) fa_[kk][a] = As[(buf)][kr_][wm * TM + a * 32 + li]; \
                _Pragma("unroll") for (int b = 0; b < NB; ++b) fb_[kk][b] = Bs[(buf)][kr_][wn * TN + b * 32 + li]; \
            }                                                                                                 \
            _Pragma("unroll") for (int kk = 0; kk < DBK / 4; ++kk)                                            \
                _Pragma("unroll") for (int a = 0; a < MB; ++a)                                                \
                    _Pragma("unroll") for (int b = 0; b < NB; ++b)                                            \
                        acc[a][b] = __builtin_amdgcn_mfma_f32_32x32x2f32(fa_[kk][a], fb_[kk][b], acc[a][b], 0, 0, 0); \
        }                                                                                                     \
        _Pragma("unroll") for (int a = 0; a < MB; ++a)                                                        \
            _Pragma("unroll") for (int b = 0; b < NB; ++b)                                                    \
                _Pragma("unroll") for (int v = 0; v < 16; ++v)                                                \
                {                                                                                             \
                    tot[a][b][v] += (double)acc[a][b][v];                                                     \
                    acc[a][b][v] = 0.0f;                                                                      \
                }                                                                                             \
    }

    DP_LOAD(xa, xb, 0);
    if (PF == 2 && nk > 1)
        DP_LOAD(ya, yb, DBK);
    DP_STORE(xa, xb, 0);
    __syncthreads();
    if (PF == 1) {
        for (int kt = 0; kt < nk; ++kt) {
            const int cur = kt & 1;
            if (kt + 1 < nk)
                DP_LOAD(xa, xb, (kt + 1) * DBK);
            DP_MMA(cur);
            if (kt + 1 < nk)
                DP_STORE(xa, xb, cur ^ 1);
            __syncthreads();
        }
    } else {
        // two slabs per trip so that the register sets are named statically
        for (int kt = 0; kt < nk; kt += 2) {
            // slab kt (in LDS buffer 0) while slab kt+1 sits in Y
            if (kt + 2 < nk)
                DP_LOAD(xa, xb, (kt + 2) * DBK);
            DP_MMA(0);
            if (kt + 1 < nk)
                DP_STORE(ya, yb, 1);
            __syncthreads();
            if (kt + 1 >= nk)
                break;
            // slab kt+1 (in LDS buffer 1) while slab kt+2 sits in X
            if (kt + 3 < nk)
                DP_LOAD(ya, yb, (kt + 3) * DBK);
            DP_MMA(1);
            if (kt + 2 < nk)
                DP_STORE(xa, xb, 0);
            __syncthreads();
        }
    }
#undef DP_LOAD
#undef DP_STORE
#undef DP_MMA

    if constexpr (RAW) {
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            const int col = c0 + wn * TN + b * 32 + li;
#pragma unroll
            for (int a = 0; a < MB; ++a)
#pragma unroll
                for (int v = 0; v < 16; ++v) {
                    const int row = i0 + wm * TM + a * 32 + 8 * (v >> 2) + 4 * ka + (v & 3);
                    if (col < R && row >= p0 && row < p1)
                        phi[(size_t)row * ldm + col] = (float)(tot[a][b][v] + (hhalf ? (double)hhalf[row] : 0.0));
                }
        }
        return;
    }

    // Epilogue (Algorithm 1 with the interface's sign: m = tanh(Phi / T)).
    // 32x32 MFMA result layout: lane l holds column l%32; register v holds row
    // 8*(v/4) + 4*(l/32) + v%4 of the 32 x 32 block.  The operands (1/T per
    // run, old state, h/2) are loaded first and unconditionally (the tile's
    // rows and columns lie inside the padded buffers), so that the loads
    // overlap instead of one round trip per element.
    const bool damp = gamma != 1.0f;
    float itv[NB], ov[NB][MB][16], hv[MB][16];
    double itd[NB];
#pragma unroll
    for (int b = 0; b < NB; ++b) {
        const int col = c0 + wn * TN + b * 32 + li;
        itv[b] = invT[col];
        itd[b] = invT64 ? invT64[col] : (double)itv[b];
#pragma unroll
        for (int a = 0; a < MB; ++a)
#pragma unroll
            for (int v = 0; v < 16; ++v)
                ov[b][a][v] = Mold[(size_t)(i0 + wm * TM + a * 32 + 8 * (v >> 2) + 4 * ka + (v & 3)) * ldm + col];
    }
#pragma unroll
    for (int a = 0; a < MB; ++a)
#pragma unroll
        for (int v = 0; v < 16; ++v) {
            hv[a][v] = hhalf ? hhalf[i0 + wm * TM + a * 32 + 8 * (v >> 2) + 4 * ka + (v & 3)] : 0.0f;
#pragma unroll
            for (int b = 0; b < NB; ++b)
                tot[a][b][v] += (double)hv[a][v];
        }
#pragma unroll
    for (int b = 0; b < NB; ++b) {
        const int col = c0 + wn * TN + b * 32 + li;
        float dl = 0.0f;
        if (col < R) {
            const float it = itv[b];
#pragma unroll
            for (int a = 0; a < MB; ++a) {
#pragma unroll
                for (int v = 0; v < 16; ++v) {
                    const int row = i0 + wm * TM + a * 32 + 8 * (v >> 2) + 4 * ka + (v & 3);
                    if (row >= p0 && row < p1) {
                        const float old = ov[b][a][v];
                        float nw = old;
                        if (it >= 0.0f) {
                            // the argument in fp64 (from the fp64 field and 1/T),
                            // rounded once; tanh in fp32
                            const float th = invT64 ? tanhf((float)(tot[a][b][v] * itd[b]))
                                                    : tanhf((float)tot[a][b][v] * it);
                            nw = damp ? (1.0f - gamma) * old + gamma * th : th;
                        }
                        Mnew[(size_t)row * ldm + col] = nw;
                        dl = fmaxf(dl, fabsf(nw - old));
                    }
                }
            }
        }
        if (dmax) {
            dl = fmaxf(dl, __shfl_xor(dl, 32));
            if (ka == 0 && col < R)
                atomicMax(&dmax[col], __float_as_uint(dl));
        }
    }
}

// Level state of one run after a sweep (Algorithm 1's repeat ... until, read
// as d < d_min, with the max_sweeps cap): state[2r] = level index,
// state[2r+1] = sweeps done at this level, -1 once the run has finished its
// levels; invT_cur[r] (and invT64_cur[r]) = 1/T of its current level, -1
// when finished; dmax[r] = bit pattern of the sweep's largest change, read
// and cleared; runstat[r] = (sweeps, levels, cap hits, -); spl (or null):
// [R x cap] sweeps run at each visited level.  Returns whether the run still
// anneals.
__device__ inline bool dense_advance_one(int r, const float *table, const double *table64, int ldt,
                                         const int32_t *nlev, int max_sweeps, double d_min, float *invT_cur,
                                         double *invT64_cur, int32_t *state, int64_t *runstat, uint32_t *dmax,
                                         int32_t *spl, int cap)
{
    int sw = state[2 * r + 1];
    if (sw < 0)
        return false;
    const float d = __uint_as_float(dmax[r]);
    dmax[r] = 0u;
    ++sw;
    runstat[(size_t)r * 4 + 0] += 1;
    const bool conv = (double)d < d_min;
    if (conv || sw >= max_sweeps) {
        if (!conv && max_sweeps > 1)
            runstat[(size_t)r * 4 + 2] += 1;
        runstat[(size_t)r * 4 + 1] += 1;
        if (spl && state[2 * r] < cap)
            spl[(size_t)r * cap + state[2 * r]] = sw;
        const int lv = state[2 * r] + 1;
        state[2 * r] = lv;
        sw = 0;
        if (lv >= nlev[r]) {
            sw = -1;
            invT_cur[r] = -1.0f;
            if (table64)
                invT64_cur[r] = -1.0;
        } else {
            invT_cur[r] = table[(size_t)lv * ldt + r];
            if (table64)
                invT64_cur[r] = table64[(size_t)lv * ldt + r];
        }
    }
    state[2 * r + 1] = sw;
    return sw >= 0;
}

template <int WM, int WN, int PF, bool RAW>
__global__ __launch_bounds__(64 * WM * WN) void k_dense_phase_f32(
    const float *__restrict__ J, int ldj, const float *__restrict__ Mold, float *__restrict__ Mnew, int ldm, int R,
    int p0, int p1, int a0, int nrt, int nct, int kpad, const float *__restrict__ invT,
    const double *__restrict__ invT64, const float *__restrict__ hhalf, float gamma, uint32_t *__restrict__ dmax,
    float *__restrict__ phi)
{
    dense_phase_f32_tile<WM, WN, PF, RAW>(J, ldj, Mold, Mnew, ldm, R, p0, p1, a0, nrt, nct, kpad, invT, invT64, hhalf,
                                          gamma, dmax, phi, blockIdx.x, nullptr);
}

}  // namespace mars
