// BF16 form of the dense path: conversion of J, state initialisation in the
// run-major bf16 layout, the phase launcher, and rounding into the padded
// spin operand shared with the fp32 form (exact energies are unchanged).
#include <algorithm>
#include <cstdlib>
#include <map>
#include <mutex>
#include <tuple>

#include "common_device.h"
#include "dense_batch_bf16.h"
#include "mars_internal.h"

namespace mars {

// Tile variants of the phase kernel (register prefetch ring of two slabs,
// one wave per 32 x 32 block).  Every variant reduces each output element
// over K in the same order (16-deep MFMA steps in increasing k, whatever the
// slab depth), so all of them produce bitwise identical results; they differ
// in how many workgroups a phase yields and how many barriers it takes.  128 x 128 x 16 waves with 128-deep
// slabs (half the barriers of 64-deep ones) is the fastest on the SK N=2000 x
// 4096-run shape and the default before the tuner has decided; smaller tiles
// fill the GPU on small instances.
typedef void (*Bf16PhaseFn)(const unsigned short *, int, const unsigned short *, unsigned short *, int, int, int,
                            int, int, int, int, const float *, const float *, float, uint32_t *);
// fn_aligned: the phase starts at a multiple of 8 spins (no 8-spin chunk
// straddles it); fn_blend: any start.
struct Bf16Variant {
    int bm, bn, bk, threads;
    Bf16PhaseFn fn_aligned, fn_blend;
};
#define BF16_VARIANT(BM, BN, WM, WN, PF, BK)                                                      \
    {                                                                                           \
        BM, BN, BK, 64 * WM * WN, k_dense_phase_bf16<BM, BN, WM, WN, PF, BK, false>,           \
            k_dense_phase_bf16<BM, BN, WM, WN, PF, BK, true>                                    \
    }
static const Bf16Variant kBf16Variants[] = {
    BF16_VARIANT(128, 128, 4, 4, 2, 128),
    BF16_VARIANT(64, 128, 2, 4, 2, 64),
    BF16_VARIANT(128, 64, 4, 2, 2, 64),
    BF16_VARIANT(64, 64, 2, 2, 2, 64),
    BF16_VARIANT(128, 128, 4, 4, 2, 64),
};
#undef BF16_VARIANT
constexpr int kNumBf16Variants = sizeof(kBf16Variants) / sizeof(kBf16Variants[0]);

__global__ void k_bf16_from_f32(const float *J, size_t n, unsigned short *Jb)
{
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (size_t)gridDim.x * blockDim.x)
        Jb[e] = float_to_bf16(J[e]);
}

mars_status ensure_bf16_couplings(Instance &I, hipStream_t s)
{
    if (I.Jbf)
        return MARS_OK;
    const size_t n = (size_t)I.Np * I.Np;
    hipError_t e = hipMalloc(&I.Jbf, n * sizeof(unsigned short));
    if (e != hipSuccess) {
        I.Jbf = nullptr;
        return hip_error(e, "hipMalloc bf16 couplings");
    }
    k_bf16_from_f32<<<2048, 256, 0, s>>>(I.J, n, I.Jbf);
    e = hipGetLastError();
    if (e != hipSuccess)
        return hip_error(e, "bf16 conversion");
    return MARS_OK;
}

int bf16_state_rows(int R) { return (R + 255) / 256 * 256; }

// M^T[r][i] = bf16(m0[i][r]) or the generator's draw (Algorithm 1's random start)
__global__ void k_bf16_init_state(uint64_t seed, int N, int R, int ldk, const float *m0, unsigned short *MT)
{
    const int r = blockIdx.y;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < N; i += gridDim.x * blockDim.x) {
        const float v = m0 ? m0[(size_t)i * R + r] : draw_m0(seed, r, i);
        MT[(size_t)r * ldk + i] = float_to_bf16(v);
    }
}

void launch_bf16_init_state(uint64_t seed, int N, int R, int ldk, const float *m0, unsigned short *MT, hipStream_t s)
{
    dim3 grid((N + 255) / 256, R);
    k_bf16_init_state<<<grid, 256, 0, s>>>(seed, N, R, ldk, m0, MT);
}

void launch_dense_phase_bf16(const Instance &I, const unsigned short *Mold, unsigned short *Mnew, int ldk, int R,
                             int p0, int p1, const float *invT, float gamma, uint32_t *dmax, int variant,
                             hipStream_t s)
{
    const Bf16Variant &v = kBf16Variants[(variant >= 0 && variant < kNumBf16Variants) ? variant : 0];
    const int nrt = (R + v.bm - 1) / v.bm;
    const int nct = (p1 - p0 + v.bn - 1) / v.bn;
    const int kpad = (I.N + v.bk - 1) / v.bk * v.bk;  // within the zero-padded Np columns
    hipLaunchKernelGGL((p0 % 8 == 0) ? v.fn_aligned : v.fn_blend, dim3(nrt * nct), dim3(v.threads), 0, s, I.Jbf,
                       I.Np, Mold, Mnew, ldk, R, p0, p1, nrt, nct, kpad, invT, I.has_h ? I.hhalf : nullptr, gamma,
                       dmax);
}

// Autotuner.  A shape class is (device, runs / 128, phase width / 128, N /
// 1024, capped at 8), rounded up.  The first solve of a class enqueues, on
// its own stream and before its first sweep, two launches of every variant
// on the first phase between timing events (the phase is idempotent: it
// reads the previous state and writes its own rows) and uses the default
// variant; a later solve of the class reads the events once they have
// completed and keeps the fastest variant for the process.  Nothing blocks
// the host.  MARS_BF16_TILE=<index> forces a variant.
struct TuneEntry {
    bool decided = false;
    int chosen = 0;
    hipEvent_t ev[kNumBf16Variants][2] = {};
};
static std::mutex g_tune_mu;
static std::map<std::tuple<int, int, int, int>, TuneEntry> g_tune_cache;

static void destroy_events(TuneEntry &t)
{
    for (auto &p : t.ev)
        for (auto &e : p)
            if (e) {
                (void)hipEventDestroy(e);
                e = nullptr;
            }
}

int bf16_phase_variant(const Instance &I, const unsigned short *Mold, unsigned short *Mnew, int ldk, int R, int p0,
                       int p1, const float *invT, float gamma, hipStream_t s)
{
    if (const char *f = std::getenv("MARS_BF16_TILE")) {
        const int v = std::atoi(f);
        if (v >= 0 && v < kNumBf16Variants)
            return v;
    }
    const auto key = std::make_tuple(I.device, (R + 127) / 128, (p1 - p0 + 127) / 128, std::min((I.N + 1023) / 1024, 8));
    std::lock_guard<std::mutex> g(g_tune_mu);
    auto it = g_tune_cache.find(key);
    if (it != g_tune_cache.end()) {
        TuneEntry &t = it->second;
        if (t.decided)
            return t.chosen;
        // pending: decide once every timing event has completed
        for (auto &p : t.ev)
            if (hipEventQuery(p[1]) != hipSuccess)
                return 0;
        float best_ms = 0.0f;
        for (int v = 0; v < kNumBf16Variants; ++v) {
            float ms = 0.0f;
            if (hipEventElapsedTime(&ms, t.ev[v][0], t.ev[v][1]) != hipSuccess) {
                (void)hipGetLastError();
                t.chosen = 0;
                break;
            }
            if (v == 0 || ms < best_ms) {
                best_ms = ms;
                t.chosen = v;
            }
        }
        destroy_events(t);
        t.decided = true;
        return t.chosen;
    }
    TuneEntry &t = g_tune_cache[key];
    bool ok = true;
    for (int v = 0; ok && v < kNumBf16Variants; ++v) {
        ok = hipEventCreate(&t.ev[v][0]) == hipSuccess && hipEventCreate(&t.ev[v][1]) == hipSuccess &&
             hipEventRecord(t.ev[v][0], s) == hipSuccess;
        for (int r = 0; ok && r < 2; ++r)
            launch_dense_phase_bf16(I, Mold, Mnew, ldk, R, p0, p1, invT, gamma, nullptr, v, s);
        ok = ok && hipGetLastError() == hipSuccess && hipEventRecord(t.ev[v][1], s) == hipSuccess;
    }
    if (!ok) {
        // timing unavailable: keep the default variant for this class
        (void)hipGetLastError();
        destroy_events(t);
        t.decided = true;
        t.chosen = 0;
    }
    return 0;
}

static_assert(kMaxBatch == kMaxBatchMembers, "grouped launch capacity");

struct BatchCaps {
    int n;
    int lslot[kMaxBatch], kmax[kMaxBatch];
};

__global__ void k_batch_advance(int *level, BatchCaps c)
{
    const int i = threadIdx.x;
    if (i < c.n) {
        const int k = level[c.lslot[i]];
        level[c.lslot[i]] = k < c.kmax[i] ? k + 1 : k;
    }
}

hipError_t launch_batch_sweep(const BatchMemberDesc *m, int n, int *level, hipStream_t s)
{
    if (n < 1 || n > kMaxBatch)
        return hipErrorInvalidValue;
    Bf16BatchArgs a;
    a.level = level;
    int maxB = 0;
    for (int i = 0; i < n; ++i)
        maxB = std::max(maxB, m[i].B);
    // tile shape of a phase launch: 128 x 128 (128-deep slabs) when the
    // members' tiles of that shape fill the chip, else 64 x 64 (four waves,
    // several workgroups per CU); both reduce every element in the same order,
    // so results do not depend on the choice.  MARS_BATCH_TILE=0|3 forces one.
    const char *fv = std::getenv("MARS_BATCH_TILE");
    const int forced = (fv && (fv[0] == '0' || fv[0] == '3') && !fv[1]) ? fv[0] - '0' : -1;
    for (int ph = 0; ph < maxB; ++ph) {
        int t128 = 0;
        for (int i = 0; i < n; ++i)
            if (ph < m[i].B && m[i].pb[ph + 1] > m[i].pb[ph])
                t128 += ((m[i].R + 127) / 128) * ((m[i].pb[ph + 1] - m[i].pb[ph] + 127) / 128);
        const bool small = forced >= 0 ? forced == 3 : t128 < 256;
        const int bm = small ? 64 : 128, bn = small ? 64 : 128, bk = small ? 64 : HBK;
        for (int i = 0; i < n; ++i) {
            const Instance &I = *m[i].I;
            Bf16BatchMember &d = a.mem[i];
            d.J = I.Jbf;
            d.Ma = m[i].Ma;
            d.Mb = m[i].Mb;
            d.table = m[i].table;
            d.hhalf = I.has_h ? I.hhalf : nullptr;
            d.ldk = I.Np;
            d.R = m[i].R;
            d.nrt = (m[i].R + bm - 1) / bm;
            d.kpad = (I.N + bk - 1) / bk * bk;
            d.ldt = m[i].ldt;
            d.kmax = m[i].kmax;
            d.lslot = m[i].lslot;
            d.gamma = m[i].gamma;
        }
        int ns = 0, tile0 = 0;
        for (int i = 0; i < n; ++i) {
            if (ph >= m[i].B || m[i].pb[ph + 1] <= m[i].pb[ph])
                continue;
            Bf16BatchSlot &sl = a.slot[ns++];
            sl.member = i;
            sl.p0 = m[i].pb[ph];
            sl.p1 = m[i].pb[ph + 1];
            sl.nct = (sl.p1 - sl.p0 + bn - 1) / bn;
            sl.tile0 = tile0;
            sl.blend = (sl.p0 % 8) != 0;
            tile0 += (a.mem[i].nrt * sl.nct + 7) / 8 * 8;  // next member starts on a multiple of 8
        }
        a.nslot = ns;
        if (ns == 0)
            continue;
        if (small)
            hipLaunchKernelGGL((k_dense_phase_bf16_batch<64, 64, 2, 2, 2, 64>), dim3(tile0), dim3(256), 0, s, a);
        else
            hipLaunchKernelGGL((k_dense_phase_bf16_batch<128, 128, 4, 4, 2, HBK>), dim3(tile0), dim3(1024), 0, s,
                               a);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess)
            return e;
    }
    BatchCaps c;
    c.n = n;
    for (int i = 0; i < n; ++i) {
        c.lslot[i] = m[i].lslot;
        c.kmax[i] = m[i].kmax;
    }
    hipLaunchKernelGGL(k_batch_advance, dim3(1), dim3(64), 0, s, level, c);
    return hipGetLastError();
}

template <int BM, int BN, int WM, int WN, int PF, int BK>
static hipError_t launch_persistent_shape(Bf16BatchPersistArgs &a, int widest, hipStream_t s)
{
    const void *fn = reinterpret_cast<const void *>(&k_dense_batch_persistent<BM, BN, WM, WN, PF, BK>);
    constexpr int threads = 64 * WM * WN;
    int dev = 0, per_cu = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess)
        return e;
    hipDeviceProp_t prop;
    if ((e = hipGetDeviceProperties(&prop, dev)) != hipSuccess)
        return e;
    if ((e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, threads, 0)) != hipSuccess)
        return e;
    // every workgroup resident at once (the grid barriers need all of them),
    // a multiple of 8 (a tile keeps its XCD), no more than the widest phase
    const int resident = per_cu * prop.multiProcessorCount / 8 * 8;
    if (resident < 8)
        return hipErrorInvalidConfiguration;
    const int grid = std::min(resident, (widest + 7) / 8 * 8);
    void *kargs[] = {&a};
    return hipLaunchCooperativeKernel(fn, dim3(grid), dim3(threads), kargs, 0, s);
}

static_assert(sizeof(Bf16BatchPersistArgs) <= 4096, "persistent step descriptors travel as kernel arguments");

hipError_t launch_batch_persistent(const BatchMemberDesc *m, int n, int *level, int sweeps, hipStream_t s)
{
    if (n < 1 || n > kMaxBatch || sweeps < 1)
        return hipErrorInvalidValue;
    int maxB = 0;
    for (int i = 0; i < n; ++i)
        maxB = std::max(maxB, m[i].B);
    if (maxB > kMaxPersistPhases)
        return hipErrorNotSupported;
    // one tile shape for the step: 128 x 128 when every phase's tiles of that
    // shape fill the chip, else 64 x 64 (bitwise the same results either way);
    // MARS_BATCH_TILE=0|3 forces one
    const char *fv = std::getenv("MARS_BATCH_TILE");
    const int forced = (fv && (fv[0] == '0' || fv[0] == '3') && !fv[1]) ? fv[0] - '0' : -1;
    int t128min = 1 << 30;
    for (int ph = 0; ph < maxB; ++ph) {
        int t128 = 0;
        for (int i = 0; i < n; ++i)
            if (ph < m[i].B && m[i].pb[ph + 1] > m[i].pb[ph])
                t128 += ((m[i].R + 127) / 128) * ((m[i].pb[ph + 1] - m[i].pb[ph] + 127) / 128);
        if (t128 > 0)
            t128min = std::min(t128min, t128);
    }
    const bool small = forced >= 0 ? forced == 3 : t128min < 256;
    const int bm = small ? 64 : 128, bn = small ? 64 : 128, bk = small ? 64 : HBK;
    Bf16BatchPersistArgs a;
    a.level = level;
    a.n = n;
    a.nph = maxB;
    a.sweeps = sweeps;
    for (int i = 0; i < n; ++i) {
        const Instance &I = *m[i].I;
        Bf16BatchMember &d = a.mem[i];
        d.J = I.Jbf;
        d.Ma = m[i].Ma;
        d.Mb = m[i].Mb;
        d.table = m[i].table;
        d.hhalf = I.has_h ? I.hhalf : nullptr;
        d.ldk = I.Np;
        d.R = m[i].R;
        d.nrt = (m[i].R + bm - 1) / bm;
        d.kpad = (I.N + bk - 1) / bk * bk;
        d.ldt = m[i].ldt;
        d.kmax = m[i].kmax;
        d.lslot = m[i].lslot;
        d.gamma = m[i].gamma;
        a.kmax[i] = m[i].kmax;
        a.lslot[i] = m[i].lslot;
    }
    int widest = 0;
    for (int ph = 0; ph < maxB; ++ph) {
        int ns = 0, tile0 = 0;
        for (int i = 0; i < n; ++i) {
            if (ph >= m[i].B || m[i].pb[ph + 1] <= m[i].pb[ph])
                continue;
            Bf16BatchSlot &sl = a.slot[ph][ns++];
            sl.member = i;
            sl.p0 = m[i].pb[ph];
            sl.p1 = m[i].pb[ph + 1];
            sl.nct = (sl.p1 - sl.p0 + bn - 1) / bn;
            sl.tile0 = tile0;
            sl.blend = (sl.p0 % 8) != 0;
            tile0 += (a.mem[i].nrt * sl.nct + 7) / 8 * 8;
        }
        a.nslot[ph] = ns;
        a.ntile[ph] = tile0;
        widest = std::max(widest, tile0);
    }
    if (widest == 0)
        return hipSuccess;
    return small ? launch_persistent_shape<64, 64, 2, 2, 2, 64>(a, widest, s)
                 : launch_persistent_shape<128, 128, 4, 4, 2, HBK>(a, widest, s);
}

// s = +1 if m >= 0 else -1 into the padded operand [ldr x Ke]; optional
// caller spins [R x N] and fp32 magnetisations [N x R]
__global__ void k_bf16_round(const unsigned short *MT, int ldk, int N, int R, int Ke, int ldr, int8_t *spad,
                             int8_t *spins, float *m_final)
{
    const int r = blockIdx.y;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < Ke; i += gridDim.x * blockDim.x) {
        int8_t v = 0;
        if (r < R && i < N) {
            const float m = bf16_to_float(MT[(size_t)r * ldk + i]);
            v = (m >= 0.0f) ? 1 : -1;
            if (spins)
                spins[(size_t)r * N + i] = v;
            if (m_final)
                m_final[(size_t)i * R + r] = m;
        }
        if (r < ldr)
            spad[(size_t)r * Ke + i] = v;
    }
}

void launch_bf16_round(const unsigned short *MT, int ldk, int N, int R, int Ke, int8_t *spad, int8_t *spins,
                       float *m_final, hipStream_t s)
{
    const int ldr = (R + 127) / 128 * 128;
    dim3 grid((Ke + 255) / 256, ldr);
    k_bf16_round<<<grid, 256, 0, s>>>(MT, ldk, N, R, Ke, ldr, spad, spins, m_final);
}

}  // namespace mars
