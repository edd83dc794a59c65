// BF16 form of the dense update phase: couplings and magnetisations stored in
// bfloat16, products on the bf16 matrix cores with fp32 accumulation, the
// update (tanh, damping, per-run max change) in fp32, the new magnetisation
// rounded to bf16 (device code; included by the library's dense unit).
//
// State layout: M^T [ldr x ldk] bf16, row = run, spins contiguous.  One phase
// computes Phi^T[runs, P] = M^T[runs, :] * J[:, P] = M^T * (J[P, :])^T (J is
// symmetric), so both operands are K-contiguous rows: run rows of M^T and
// spin rows of J.  Ping-pong exactly as the fp32 form: spins k < p0 come from
// the buffer being written this sweep, the rest from the previous one.
//
// Workgroup tile BM runs x BN spins, K in 64-element slabs through
// double-buffered LDS (rows padded to 72 elements) fed from a register ring
// of PF slabs, WM x WN waves, each wave (BM/WM) x (BN/WN) made of 32 x 32
// blocks of the 32x32x16 bf16 MFMA.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace mars {

typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef unsigned short ushortx8 __attribute__((ext_vector_type(8)));

constexpr int HBK = 64;        // default slab depth (elements)

__device__ inline float bf16_to_float(unsigned short h) { return __uint_as_float((uint32_t)h << 16); }

// round to nearest even (finite inputs; magnetisations are in [-1, 1])
__device__ inline unsigned short float_to_bf16(float f)
{
    const uint32_t u = __float_as_uint(f);
    return (unsigned short)((u + 0x7fffu + ((u >> 16) & 1u)) >> 16);
}

// tanh(a) = 1 - 2 / (exp(2a) + 1) on |a| with the hardware exp2 and
// reciprocal, sign restored afterwards; absolute error ~1e-7, far below the
// bf16 rounding of the result (2^-9)
__device__ inline float bf16_form_tanh(float x)
{
    const float a = fabsf(x);
    const float e = __builtin_amdgcn_exp2f(a * 2.8853900817779268f);
    const float t = 1.0f - 2.0f * __builtin_amdgcn_rcpf(e + 1.0f);
    return copysignf(t, x);
}

// LDS of one workgroup: double-buffered A and B slabs, rows padded by 8
template <int BM, int BN, int BK>
constexpr size_t bf16_phase_lds_bytes()
{
    return (size_t)2 * (BM + BN) * (BK + 8) * sizeof(unsigned short);
}

// One workgroup tile of a phase: tile t (0 <= t < nrt * nct) of the phase's
// grid; lds: bf16_phase_lds_bytes<BM, BN, BK>() bytes, 16-byte aligned.
// skip (or null): per BM-run row block, nonzero = leave the tile out (its
// runs are all frozen and both state buffers already hold their values).
template <int BM, int BN, int WM, int WN, int PF, int BK, bool BLEND>
__device__ __forceinline__ void bf16_phase_tile(
    const unsigned short *__restrict__ J, int ldj, const unsigned short *__restrict__ Mold,
    unsigned short *__restrict__ Mnew, int ldk, int R, int p0, int p1, int nrt, int nct, int kpad,
    const float *__restrict__ invT, const float *__restrict__ hhalf, float gamma, uint32_t *__restrict__ dmax,
    unsigned char *lds, int tile, const int32_t *__restrict__ skip = nullptr)
{
    constexpr int NT = 64 * WM * WN;
    constexpr int TM = BM / WM, TN = BN / WN;
    constexpr int MB = TM / 32, NB = TN / 32;
    constexpr int CA = BM * BK / 8, CB = BN * BK / 8;  // 16-byte chunks per slab
    constexpr int CR = BK / 8;                         // chunks per slab row
    constexpr int LDR = BK + 8;                        // padded LDS row (elements)
    constexpr int LA = (CA + NT - 1) / NT, LB = (CB + NT - 1) / NT;
    static_assert(MB >= 1 && NB >= 1, "tile shape");
    static_assert(PF >= 1 && PF <= 4, "prefetch ring");

    typedef unsigned short ATile[BM][LDR];
    typedef unsigned short BTile[BN][LDR];
    ATile *As = reinterpret_cast<ATile *>(lds);
    BTile *Bs = reinterpret_cast<BTile *>(lds + (size_t)2 * BM * LDR * sizeof(unsigned short));

    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int wm = wave / WN, wn = wave % WN;
    const int li = lane & 31, kh = lane >> 5;

    // tile order: the workgroups of one XCD share a band of runs (rows of M^T)
    const int total = nrt * nct;
    int t = tile;
    if ((total & 7) == 0)
        t = (t & 7) * (total >> 3) + (t >> 3);
    const int rt = t / nct, ct = t % nct;
    if (skip && skip[rt])
        return;
    const int r0 = rt * BM;
    const int i0 = p0 + ct * BN;

    floatx16 acc[MB][NB];
#pragma unroll
    for (int a = 0; a < MB; ++a)
#pragma unroll
        for (int b = 0; b < NB; ++b)
#pragma unroll
            for (int v = 0; v < 16; ++v)
                acc[a][b][v] = 0.0f;

    ushortx8 ga[PF][LA], gb[PF][LB];
    // A chunk: run row, 8 spins; spins below p0 from the new buffer.  The
    // load is branch-free, so that the loads of a slab stay in flight while
    // the previous slab is multiplied: each chunk's buffer is selected (a
    // chunk straddling p0 is read from the old buffer).  When p0 is not a
    // multiple of 8 (BLEND), the straddling chunk's new-buffer copy is read
    // once at the start and its spins below p0 are patched in when that
    // chunk is staged into LDS.
    auto load_a = [&](ushortx8 &dst, int c, int k0) {
        const int row = c / CR, kc = k0 + (c % CR) * 8;
        const size_t off = (size_t)(r0 + row) * ldk + kc;
        dst = *reinterpret_cast<const ushortx8 *>((kc + 8 <= p0 ? Mnew : Mold) + off);
    };
    const int kst = p0 & ~7;  // start of the chunk that may straddle p0
    ushortx8 pre[LA];
    if constexpr (BLEND) {
#pragma unroll
        for (int q = 0; q < LA; ++q) {
            const int row = (tid + q * NT) / CR;
            pre[q] = *reinterpret_cast<const ushortx8 *>(Mnew + (size_t)(r0 + row) * ldk + kst);
        }
    }
    auto stage_a = [&](ushortx8 v, int q, int k0) -> ushortx8 {
        if constexpr (BLEND) {
            const int kc = k0 + ((tid + q * NT) % CR) * 8;
#pragma unroll
            for (int e = 0; e < 8; ++e)
                v[e] = (kc == kst && kst + e < p0) ? pre[q][e] : v[e];
        }
        return v;
    };
#define H_LOAD(RA, RB, k0)                                                                          \
    _Pragma("unroll") for (int q = 0; q < LA; ++q)                                                  \
    {                                                                                               \
        const int c_ = tid + q * NT;                                                                \
        if (c_ < CA)                                                                                \
            load_a((RA)[q], c_, (k0));                                                              \
    }                                                                                               \
    _Pragma("unroll") for (int q = 0; q < LB; ++q)                                                  \
    {                                                                                               \
        const int c_ = tid + q * NT;                                                                \
        if (c_ < CB)                                                                                \
            (RB)[q] = *reinterpret_cast<const ushortx8 *>(J + (size_t)(i0 + c_ / CR) * ldj + (k0) + (c_ % CR) * 8); \
    }
#define H_STORE(RA, RB, buf, k0)                                                                    \
    _Pragma("unroll") for (int q = 0; q < LA; ++q)                                                  \
    {                                                                                               \
        const int c_ = tid + q * NT;                                                                \
        if (c_ < CA)                                                                                \
            *reinterpret_cast<ushortx8 *>(&As[(buf)][c_ / CR][(c_ % CR) * 8]) = stage_a((RA)[q], q, (k0)); \
    }                                                                                               \
    _Pragma("unroll") for (int q = 0; q < LB; ++q)                                                  \
    {                                                                                               \
        const int c_ = tid + q * NT;                                                                \
        if (c_ < CB)                                                                                \
            *reinterpret_cast<ushortx8 *>(&Bs[(buf)][c_ / CR][(c_ % CR) * 8]) = (RB)[q];            \
    }

    // Slabs move global -> registers -> LDS.  Registers hold a ring of PF
    // slabs: at step kt the ring slot of slab kt (already in LDS) is refilled
    // with slab kt + PF, the step computes on slab kt, then slab kt + 1 goes
    // from its ring slot into the other LDS buffer.  A load thus has PF
    // compute steps to arrive.  The refill is unconditional (past the last
    // slab it re-reads the last one) so that the wait before each LDS store
    // covers only the older loads and the younger ones stay in flight.
    const int nk = kpad / BK;
#pragma unroll
    for (int s = 0; s < PF; ++s) {
        const int kl = s < nk ? s : nk - 1;
        H_LOAD(ga[s], gb[s], kl * BK);
    }
    H_STORE(ga[0], gb[0], 0, 0);
    __syncthreads();
    for (int kb = 0; kb < nk; kb += PF) {
#pragma unroll
        for (int s = 0; s < PF; ++s) {
            const int kt = kb + s;
            const int kl = kt + PF < nk ? kt + PF : nk - 1;
            H_LOAD(ga[s], gb[s], kl * BK);
            if (kt < nk) {
                const int cur = kt & 1;
#pragma unroll
                for (int ks = 0; ks < BK / 16; ++ks) {
                    bf16x8 fa[MB], fb[NB];
#pragma unroll
                    for (int a = 0; a < MB; ++a)
                        fa[a] = *reinterpret_cast<const bf16x8 *>(&As[cur][wm * TM + a * 32 + li][ks * 16 + kh * 8]);
#pragma unroll
                    for (int b = 0; b < NB; ++b)
                        fb[b] = *reinterpret_cast<const bf16x8 *>(&Bs[cur][wn * TN + b * 32 + li][ks * 16 + kh * 8]);
#pragma unroll
                    for (int a = 0; a < MB; ++a)
#pragma unroll
                        for (int b = 0; b < NB; ++b)
                            acc[a][b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(fa[a], fb[b], acc[a][b], 0, 0, 0);
                }
                if (kt + 1 < nk) {
                    H_STORE(ga[(s + 1) % PF], gb[(s + 1) % PF], cur ^ 1, (kt + 1) * BK);
                }
                __syncthreads();
            }
        }
    }
#undef H_LOAD
#undef H_STORE

    // epilogue: element (run = row, spin = column) of each 32 x 32 block; lane
    // l holds spin column l%32, register v holds run row 8*(v/4) + 4*(l/32) + v%4.
    // Every operand of a row block's update is loaded first, unconditionally
    // (rows below the padded run count and columns below the padded
    // dimension are in bounds), so the loads overlap instead of one round
    // trip per element.
    const bool damp = gamma != 1.0f;
    float hv[NB];
#pragma unroll
    for (int b = 0; b < NB; ++b)
        hv[b] = hhalf ? hhalf[i0 + wn * TN + b * 32 + li] : 0.0f;
#pragma unroll
    for (int a = 0; a < MB; ++a) {
        float itv[16];
        unsigned short ov[NB][16];
#pragma unroll
        for (int v = 0; v < 16; ++v) {
            const int run = r0 + wm * TM + a * 32 + 8 * (v >> 2) + 4 * kh + (v & 3);
            itv[v] = invT[run];
#pragma unroll
            for (int b = 0; b < NB; ++b)
                ov[b][v] = Mold[(size_t)run * ldk + i0 + wn * TN + b * 32 + li];
        }
        // The stores are unconditional too (a conditional store would make
        // the wait counts conservative again): a row past R writes its old
        // value back; a column past p1 belongs to a later phase of this
        // sweep, which overwrites it before anything reads it (columns past
        // N compute 0 from the zero padding of J and h).
#pragma unroll
        for (int v = 0; v < 16; ++v) {
            const int run = r0 + wm * TM + a * 32 + 8 * (v >> 2) + 4 * kh + (v & 3);
            const bool rok = run < R;
            const float it = rok ? itv[v] : -1.0f;  // < 0: frozen (finished run or padding row)
            float dl = 0.0f;
#pragma unroll
            for (int b = 0; b < NB; ++b) {
                const int spin = i0 + wn * TN + b * 32 + li;
                const float old = bf16_to_float(ov[b][v]);
                const float th = bf16_form_tanh((acc[a][b][v] + hv[b]) * it);
                const float upd = damp ? (1.0f - gamma) * old + gamma * th : th;
                const unsigned short nb16 = it >= 0.0f ? float_to_bf16(upd) : ov[b][v];
                Mnew[(size_t)run * ldk + spin] = nb16;
                const float dd = fabsf(bf16_to_float(nb16) - old);
                dl = (rok && spin < p1) ? fmaxf(dl, dd) : dl;
            }
            if (dmax) {
                // per-run maximum over the 32 spin lanes of this half-wave
#pragma unroll
                for (int m = 16; m >= 1; m >>= 1)
                    dl = fmaxf(dl, __shfl_xor(dl, m));
                if (li == 0 && rok)
                    atomicMax(&dmax[run], __float_as_uint(dl));
            }
        }
    }
}

template <int BM, int BN, int WM, int WN, int PF, int BK = HBK, bool BLEND = true>
__global__ __launch_bounds__(64 * WM * WN) void k_dense_phase_bf16(
    const unsigned short *__restrict__ J, int ldj, const unsigned short *__restrict__ Mold,
    unsigned short *__restrict__ Mnew, int ldk, int R, int p0, int p1, int nrt, int nct, int kpad,
    const float *__restrict__ invT, const float *__restrict__ hhalf, float gamma, uint32_t *__restrict__ dmax)
{
    __shared__ __attribute__((aligned(16))) unsigned char lds[bf16_phase_lds_bytes<BM, BN, BK>()];
    bf16_phase_tile<BM, BN, WM, WN, PF, BK, BLEND>(J, ldj, Mold, Mnew, ldk, R, p0, p1, nrt, nct, kpad, invT, hhalf,
                                                   gamma, dmax, lds, blockIdx.x);
}

}  // namespace mars
