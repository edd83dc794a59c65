// Device helpers shared by the library's kernels: the counter-based
// generator, temperature levels and exact integer-to-double conversion.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "../../include/mars.h"

namespace mars {

// SplitMix64 output function (Steele, Lea & Flood, OOPSLA 2014) evaluated at
// the counter c: the value the generator started at `seed` returns on its
// (c+1)-th call.  Stateless, so every (run, spin) draw is independent of the
// launch shape.
__host__ __device__ inline uint64_t splitmix64_at(uint64_t seed, uint64_t c)
{
    uint64_t z = seed + (c + 1ull) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// Initial magnetisation of spin i in run r (Algorithm 1: a uniform value in
// (-1, 1)): the top 24 bits k of stream 0 give (2k + 1 - 2^24) * 2^-24, an odd
// multiple of 2^-24 that is exact in float and never zero.
__device__ inline float draw_m0(uint64_t seed, int64_t r, int64_t i)
{
    uint64_t k = splitmix64_at(seed, ((uint64_t)r << 32) | (uint64_t)i) >> 40;
    return (float)(int32_t)(2 * (int64_t)k + 1 - (1 << 24)) * 0x1p-24f;
}

// Starting temperature of run r: T_lo + (T_hi - T_lo) * (k * 2^-24) from
// stream 1, each operation rounded separately (no fused multiply-add).
__device__ inline double draw_T0(uint64_t seed, int64_t r, double T_lo, double T_hi)
{
#pragma clang fp contract(off)
    uint64_t k = splitmix64_at(seed, (1ull << 62) | ((uint64_t)r << 32)) >> 40;
    double u = (double)k * 0x1p-24;
    double w = T_hi - T_lo;
    double t = w * u;
    return T_lo + t;
}

// Temperature levels of one run (Algorithm 1's scheduler):
//  linear:    T <- T0, then T <- T - c_step before each level, until T <= 0;
//  geometric: T_k = T0 exp((k/(K-1)) ln(T_end/T0)), k = 0..K-1.
// Only levels [first, first + count) are visited.
struct RunSchedule {
    int kind;
    double T_end, c_step;
    int steps;
    int first, count;  // count < 0: to the end
};

inline RunSchedule make_run_schedule(const mars_schedule &sc)
{
    RunSchedule r;
    r.kind = sc.kind;
    r.T_end = sc.T_end;
    r.c_step = sc.c_step;
    r.steps = sc.steps;
    r.first = sc.first_level < 0 ? 0 : sc.first_level;
    r.count = sc.level_count;
    return r;
}

// keeps a value opaque to the optimiser (no instruction is emitted): byte
// offsets stay plain additions instead of being re-derived at every use, and
// a load address is not related to the addresses of other iterations
__device__ __forceinline__ uint32_t opaque(uint32_t x)
{
    __asm__ volatile("" : "+v"(x));
    return x;
}
__device__ __forceinline__ float opaque(float x)
{
    __asm__ volatile("" : "+v"(x));
    return x;
}
// the same for a value that is uniform across the workgroup (kept in a
// scalar register)
__device__ __forceinline__ uint32_t opaque_uniform(uint32_t x)
{
    __asm__ volatile("" : "+s"(x));
    return x;
}

struct LevelWalker {
    double T0, lr, T;
    int k;      // level index in the run's schedule
    int stop;   // one past the last level to visit (geometric); linear uses T
    int left;   // levels left in range (linear, -1: unlimited)
    bool done;

    __host__ __device__ inline double geometric_T(const RunSchedule &s, int kk) const
    {
#pragma clang fp contract(off)
        if (s.steps == 1)
            return T0;
        double f = (double)kk / (double)(s.steps - 1);
        return T0 * exp(f * lr);
    }

    __host__ __device__ inline void start(const RunSchedule &s, double t0)
    {
#pragma clang fp contract(off)
        T0 = t0;
        done = false;
        k = s.first;
        if (s.kind == MARS_GEOMETRIC) {
            lr = log(s.T_end / T0);
            stop = s.steps;
            if (s.count >= 0 && s.first + s.count < stop)
                stop = s.first + s.count;
            if (k >= stop) {
                done = true;
                T = 0.0;
                return;
            }
            T = geometric_T(s, k);
        } else {
            lr = 0.0;
            left = s.count;
            double t = T0;
            for (int n = 0; n <= k; ++n) {
                t = t - s.c_step;
                if (!(t > 0.0))
                    break;
            }
            T = t;
            if (!(t > 0.0) || left == 0)
                done = true;
        }
    }

    __host__ __device__ inline void next(const RunSchedule &s)
    {
#pragma clang fp contract(off)
        ++k;
        if (s.kind == MARS_GEOMETRIC) {
            if (k >= stop) {
                done = true;
                return;
            }
            T = geometric_T(s, k);
        } else {
            if (left > 0)
                --left;
            T = T - s.c_step;
            if (!(T > 0.0) || left == 0)
                done = true;
        }
    }
};

// Round v * 2^e to the nearest double (ties to even).  v is an exact
// fixed-point sum, so this is the single rounding of the exact energy.
__device__ inline double i128_to_double_scaled(__int128 v, int e)
{
    if (v == 0)
        return 0.0;
    bool neg = v < 0;
    unsigned __int128 u = neg ? (unsigned __int128)0 - (unsigned __int128)v : (unsigned __int128)v;
    uint64_t hi = (uint64_t)(u >> 64), lo = (uint64_t)u;
    int top = hi ? 127 - __builtin_clzll(hi) : 63 - __builtin_clzll(lo);
    double d;
    if (top <= 52) {
        d = ldexp((double)lo, e);
    } else {
        int sh = top - 52;
        uint64_t sig = (uint64_t)(u >> sh);
        unsigned __int128 rem = u & (((unsigned __int128)1 << sh) - 1);
        unsigned __int128 half = (unsigned __int128)1 << (sh - 1);
        if (rem > half || (rem == half && (sig & 1)))
            ++sig;
        d = ldexp((double)sig, sh + e);
    }
    return neg ? -d : d;
}

}  // namespace mars
