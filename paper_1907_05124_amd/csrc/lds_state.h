// Helpers of the LDS-resident solvers (lattice and sparse): storage types of
// the magnetisation, the fp32 tanh, and reads/writes of VEC consecutive runs.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "common_device.h"
#include "mars_internal.h"

namespace mars {

template <typename S>
struct LStore;
template <>
struct LStore<double> {
    typedef double C;
    __device__ static inline double ld(double v) { return v; }
    __device__ static inline double st(double v) { return v; }
};
template <>
struct LStore<float> {
    typedef float C;
    __device__ static inline float ld(float v) { return v; }
    __device__ static inline float st(float v) { return v; }
};
template <>
struct LStore<_Float16> {
    typedef float C;
    __device__ static inline float ld(_Float16 v) { return (float)v; }
    __device__ static inline _Float16 st(float v) { return (_Float16)v; }
};

__device__ inline double l_tanh(double x) { return tanh(x); }
// tanh(a) = 1 - 2 / (exp(2a) + 1) on |a| with the hardware exp2 and reciprocal,
// sign restored afterwards (exactly odd); absolute error ~1e-7
__device__ inline float l_tanh(float x)
{
    const float a = fabsf(x);
    const float e = __builtin_amdgcn_exp2f(a * 2.8853900817779268f);
    const float t = 1.0f - 2.0f * __builtin_amdgcn_rcpf(e + 1.0f);
    return copysignf(t, x);
}
__device__ inline double l_scale(double phi, double T, double invT) { return phi / T; }
__device__ inline float l_scale(float phi, double T, float invT) { return phi * invT; }
// Phi / T with the per-run factor of run_scale: a true division in fp64, a
// multiply by the rounded inverse in fp32
__device__ inline double l_apply(double phi, double T) { return phi / T; }
__device__ inline float l_apply(float phi, float invT) { return phi * invT; }

template <typename S, int VEC>
struct Pack {
    S v[VEC];
};

template <typename S, int VEC>
__device__ inline Pack<S, VEC> lds_get(const S *p)
{
    Pack<S, VEC> r;
    if constexpr (VEC == 4 && sizeof(S) == 4) {
        const float4 f = *reinterpret_cast<const float4 *>(p);
        r.v[0] = f.x;
        r.v[1] = f.y;
        r.v[2] = f.z;
        r.v[3] = f.w;
    } else if constexpr (VEC == 4 && sizeof(S) == 2) {
        const uint2 u = *reinterpret_cast<const uint2 *>(p);
        r.v[0] = __builtin_bit_cast(S, (unsigned short)(u.x & 0xffffu));
        r.v[1] = __builtin_bit_cast(S, (unsigned short)(u.x >> 16));
        r.v[2] = __builtin_bit_cast(S, (unsigned short)(u.y & 0xffffu));
        r.v[3] = __builtin_bit_cast(S, (unsigned short)(u.y >> 16));
    } else if constexpr (VEC == 2 && sizeof(S) == 2) {
        const uint32_t u = *reinterpret_cast<const uint32_t *>(p);
        r.v[0] = __builtin_bit_cast(S, (unsigned short)(u & 0xffffu));
        r.v[1] = __builtin_bit_cast(S, (unsigned short)(u >> 16));
    } else if constexpr (VEC == 2 && sizeof(S) == 4) {
        const float2 f = *reinterpret_cast<const float2 *>(p);
        r.v[0] = f.x;
        r.v[1] = f.y;
    } else {
#pragma unroll
        for (int e = 0; e < VEC; ++e)
            r.v[e] = p[e];
    }
    return r;
}

template <typename S, int VEC>
__device__ inline void lds_put(S *p, const Pack<S, VEC> &r)
{
    if constexpr (VEC == 4 && sizeof(S) == 4) {
        *reinterpret_cast<float4 *>(p) = make_float4(r.v[0], r.v[1], r.v[2], r.v[3]);
    } else if constexpr (VEC == 4 && sizeof(S) == 2) {
        auto b = [&](int e) { return (uint32_t)__builtin_bit_cast(unsigned short, r.v[e]); };
        *reinterpret_cast<uint2 *>(p) = make_uint2(b(0) | (b(1) << 16), b(2) | (b(3) << 16));
    } else if constexpr (VEC == 2 && sizeof(S) == 2) {
        const uint32_t u = (uint32_t)__builtin_bit_cast(unsigned short, r.v[0]) |
                           ((uint32_t)__builtin_bit_cast(unsigned short, r.v[1]) << 16);
        *reinterpret_cast<uint32_t *>(p) = u;
    } else if constexpr (VEC == 2 && sizeof(S) == 4) {
        *reinterpret_cast<float2 *>(p) = make_float2(r.v[0], r.v[1]);
    } else {
#pragma unroll
        for (int e = 0; e < VEC; ++e)
            p[e] = r.v[e];
    }
}

// Level bookkeeping of one run, kept in LDS and advanced by one thread at the
// end of each sweep: the run walks its own temperature levels (Algorithm 1),
// one sweep per level or, with max_sweeps > 1, sweeps until the largest
// change d falls below d_min.  The other threads only read T, invT and done.
struct RunState {
    LevelWalker lw;
    double invT64;  // 1/T of the current level
    float invT32;
    int done;
    int sw;       // sweeps at the current level
    int sweeps, levels, caps;

    __device__ void start(const RunSchedule &rs, double T0, bool live)
    {
        lw.start(rs, live ? T0 : 1.0);
        done = (!live || lw.done) ? 1 : 0;
        invT64 = done ? 1.0 : 1.0 / lw.T;
        invT32 = done ? 0.0f : (float)(1.0 / lw.T);
        sw = sweeps = levels = caps = 0;
    }
    // tT / tI: the run's row of the block's level table of 1/T in fp64 and
    // fp32 (geometric schedules, filled from the same walker before the first
    // sweep), or null
    __device__ void advance(const RunSchedule &rs, const double *tT, const float *tI)
    {
        ++levels;
        sw = 0;
        if (tT) {
            ++lw.k;
            if (lw.k >= lw.stop) {
                lw.done = true;
                done = 1;
                return;
            }
            invT64 = tT[lw.k - rs.first];
            invT32 = tI[lw.k - rs.first];
            return;
        }
        lw.next(rs);
        if (lw.done) {
            done = 1;
        } else {
            invT64 = 1.0 / lw.T;
            invT32 = (float)(1.0 / lw.T);
        }
    }
    // d: the run's largest change in the sweep (fp32 image), read only when
    // several sweeps per level are allowed.  spl: the run's row of per-level
    // sweep counts (entry = index of the level among those visited), cap
    // entries, or null
    __device__ void end_sweep(const RunSchedule &rs, float d, bool trackd, int max_sweeps, double d_min,
                              const double *tT, const float *tI, int32_t *spl, int cap)
    {
        if (done)
            return;
        ++sweeps;
        if (!trackd) {
            if (spl && levels < cap)
                spl[levels] = 1;
            advance(rs, tT, tI);
            return;
        }
        ++sw;
        const bool conv = (double)d < d_min;
        if (conv || sw >= max_sweeps) {
            if (!conv && max_sweeps > 1)
                ++caps;
            if (spl && levels < cap)
                spl[levels] = sw;
            advance(rs, tT, tI);
        }
    }
    __device__ void write_stats(int64_t *runstat, int run) const
    {
        runstat[(size_t)run * 4 + 0] = sweeps;
        runstat[(size_t)run * 4 + 1] = levels;
        runstat[(size_t)run * 4 + 2] = caps;
        runstat[(size_t)run * 4 + 3] = 0;
    }
};

// Block-wide vote at the top of a sweep of an LDS-resident solver: every
// thread contributes code bit 0 (one of its runs still anneals) and bit 1 (one
// of its runs has finished); the OR over the block comes back to every thread
// (every lane of the workgroup must call it, with the whole wave active),
// so the branches taken on it (leave the sweep loop; the fast update that
// needs every run live) are the same for the whole workgroup and every thread
// meets the same barriers.  One barrier per vote: the two words serve
// alternate votes, and the word of the next vote is cleared after this one's
// barrier, by which time every thread has read the previous vote from it (a
// sweep holds at least one more barrier between two votes).  words[0..1] must
// be zero before the first vote, k counts the votes.
__device__ inline unsigned block_vote(unsigned *words, unsigned k, unsigned code)
{
    unsigned *w = words + (k & 1u);
    // one LDS atomic per wave (the lanes' codes combined by two ballots)
    const unsigned wc = (__ballot(code & 1u) ? 1u : 0u) | (__ballot(code & 2u) ? 2u : 0u);
    if ((threadIdx.x & 63u) == 0u && wc)
        atomicOr(w, wc);
    __syncthreads();
    const unsigned v = *w;
    if (threadIdx.x == 0)
        words[(k + 1u) & 1u] = 0u;
    return v;
}

// Per-run LDS area of an LDS-resident solver: state, then the sweep's
// largest change (bit pattern of a non-negative float, for atomicMax).
constexpr size_t RUN_AREA_BYTES = sizeof(RunState) + sizeof(uint32_t);
static_assert(RUN_AREA_BYTES <= RUN_AREA_MAX, "per-run LDS area exceeds the launcher's reservation");

// tanh(Phi / T) from a per-run factor ts (run_tscale): fp32 folds the
// exp2 constant into the factor, ts = 2 log2(e) / T, and takes
// tanh(a) = 2 / (1 + exp(-2a)) - 1, which keeps the sign by itself (exp2 of
// a large argument is +inf and its reciprocal 0, so the ends are exactly -1
// and +1; absolute error ~1e-7 near 0, as for the form on |a|); fp64 divides
// by T
//
// ACC = 2 (fp32 storage): the form above has an absolute error of ~1e-7
// (the rounding of 2 / (1 + e) near 1), a large relative error where
// tanh(a) is small: it returns exactly 0 once |a| < ~3e-8, which would pin a
// magnetisation that decayed at a high temperature at 0 for the rest of the
// anneal (tanh keeps it tiny and lets it grow back once T falls below the
// instability), and it perturbs every small magnetisation by much more than
// fp32 rounding.  Below |a| = 0.625 tanh(a) = a q(a^2) instead, q a degree-4
// polynomial fitted for relative error (2.1e-7 with fp32 evaluation, against
// 2.8e-7 for the exp form above 0.625), so the result carries a relative
// error of a few fp32 units everywhere.  fp16 storage rounds to 2^-11 anyway
// and keeps the short form.
//
// ACC = 1 (fp16 storage of the sparse solver): only tanh(a) = a below
// |a| = 2^-12 (a^2/3 < 2^-25 relative), its magnitude floored at 2^-24 (the
// smallest fp16 subnormal) with the sign of a, so that a decayed value stays
// nonzero with its sign instead of becoming exactly 0: every value this
// returns converts to a nonzero fp16 (a zero field gives +2^-24, the state of
// an isolated spin; its rounded spin is +1 as for 0).  Values between 2^-25
// and 2^-24 round to 2^-24 anyway, so the floor only changes what would
// round to 0; a damped update, which can cancel to a smaller value, stores
// through lds_keep_sign.
template <int ACC = 0>
__device__ inline float l_tanh_run(float phi, float ts)
{
    const float x = -phi * ts;
    const float e = __builtin_amdgcn_exp2f(x);
    const float t = __builtin_fmaf(2.0f, __builtin_amdgcn_rcpf(1.0f + e), -1.0f);
    if constexpr (ACC == 2) {
        const float a = x * -0.34657359027997264f;  // x = -2 log2(e) a, so a = -x ln(2) / 2
        const float z = a * a;
        float q = __builtin_fmaf(z, 0.015050967f, -0.051821887f);
        q = __builtin_fmaf(z, q, 0.13304527f);
        q = __builtin_fmaf(z, q, -0.33331954f);
        q = __builtin_fmaf(z, q, 0.99999988f);
        return fabsf(a) < 0.625f ? a * q : t;
    } else if constexpr (ACC == 1) {
        const float a = x * -0.34657359027997264f;
        const float f = __builtin_copysignf(__builtin_fmaxf(fabsf(a), 0x1p-24f), a);
        return fabsf(a) < 0x1p-12f ? f : t;
    }
    return t;
}

// Store of a magnetisation that keeps its sign through fp16 underflow: a
// nonzero value below half the smallest fp16 subnormal (2^-24) would round to
// 0, losing the direction a decayed run grows back in once T falls below its
// instability; it is stored as +-2^-24 instead (needed after a damped
// update: an undamped one stores the fp16-storage tanh above, whose
// magnitude is never below 2^-24).  Other storage types store plainly.
template <typename S>
__device__ inline S lds_keep_sign(typename LStore<S>::C v)
{
    if constexpr (sizeof(S) == 2) {
        const _Float16 h = (_Float16)v;
        return (h == (_Float16)0.0f && v != 0.0f) ? (_Float16)copysignf(0x1p-24f, v) : h;
    } else {
        return LStore<S>::st(v);
    }
}
// fp64: a = Phi * (1/T) (within an ulp of Phi / T, without a division per
// update), tanh(a) = expm1(2|a|) / (expm1(2|a|) + 2) with the sign of a
// (accurate near 0 through expm1; a few ulp), a third of the instructions
// of the library tanh; |a| > 20 rounds to +-1 in double
template <int ACC = 0>
__device__ inline double l_tanh_run(double phi, double invT)
{
    const double a = phi * invT;
    const double x = fabs(a);
    const double e = expm1(2.0 * x);
    const double t = x > 20.0 ? 1.0 : e / (e + 2.0);
    return copysign(t, a);
}

template <typename C>
__device__ inline C run_tscale(const RunState &r);
template <>
__device__ inline float run_tscale<float>(const RunState &r) { return r.invT32 * 2.8853900817779268f; }
template <>
__device__ inline double run_tscale<double>(const RunState &r) { return r.invT64; }

}  // namespace mars
