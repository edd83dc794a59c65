// Periodic +-J lattices: a workgroup anneals a block of rpw runs from start
// to finish with their magnetisations in LDS, m[site * rpw + q], as the
// sparse solver does, specialised for the stencil:
//  * each thread updates one site for VEC consecutive runs, so the site's
//    address, neighbour offsets and bond byte are shared by VEC updates and
//    the VEC values of a neighbour arrive in one LDS read;
//  * the thread owns a fixed x half-column slot, walks rows (y, z) with a
//    constant stride and keeps the site index incrementally; neighbour
//    offsets along y and z are constants of the row;
//  * checkerboard phases (colour = parity of x + y + z) are independent sets,
//    updated in place with a barrier between them; the synchronous variant
//    writes a second copy and swaps.
#include <algorithm>
#include <cmath>
#include <type_traits>

#include "common_device.h"
#include "lds_state.h"
#include "mars_internal.h"

namespace mars {

typedef _Float16 half2_t __attribute__((ext_vector_type(2)));
typedef float float2_t __attribute__((ext_vector_type(2)));
// two floats rounded to the nearest halves, packed low / high
__device__ __forceinline__ uint32_t pack_halves(float lo, float hi)
{
    const half2_t h = __builtin_convertvector((float2_t){lo, hi}, half2_t);
    return __builtin_bit_cast(uint32_t, h);
}

template <typename S, int VEC, int DIM, bool JAC, bool TRACKD, bool HAS_H, bool DAMP>
__global__ __launch_bounds__(1024) void k_lattice_solve(GraphArgs a, int lg_rpw)
{
    typedef typename LStore<S>::C C;
    extern __shared__ __attribute__((aligned(16))) unsigned char smem_raw[];
    const int N = a.N;
    const int rpw = 1 << lg_rpw;
    S *m = reinterpret_cast<S *>(smem_raw);
    S *m2 = JAC ? m + (size_t)N * rpw : m;
    const size_t state_bytes = ((size_t)N * rpw * sizeof(S) * (JAC ? 2 : 1) + 15) & ~(size_t)15;
    RunState *rsl = reinterpret_cast<RunState *>(smem_raw + state_bytes);
    uint32_t *dq = reinterpret_cast<uint32_t *>(rsl + rpw);

    const int nq = rpw / VEC;               // run groups per workgroup
    const int qg = threadIdx.x % nq;
    const int q0 = qg * VEC;                // first run slot of this thread
    const int tq = threadIdx.x / nq;        // thread index within the run group
    const int Tq = blockDim.x / nq;
    const int run0 = blockIdx.x * rpw + q0;

    bool live[VEC];
#pragma unroll
    for (int e = 0; e < VEC; ++e)
        live[e] = run0 + e < a.R;

    // initial state (Algorithm 1: s_i := rand(-1, 1))
    for (int i = tq; i < N; i += Tq) {
        Pack<S, VEC> p;
#pragma unroll
        for (int e = 0; e < VEC; ++e) {
            C v = 0;
            if (live[e])
                v = a.m0 ? (C)(reinterpret_cast<const C *>(a.m0))[(size_t)i * a.R + run0 + e]
                         : (C)draw_m0(a.seed, run0 + e, i);
            p.v[e] = LStore<S>::st(v);
        }
        lds_put<S, VEC>(&m[((size_t)i << lg_rpw) + q0], p);
    }
    for (int q = threadIdx.x; q < rpw; q += blockDim.x) {
        const int r = blockIdx.x * rpw + q;
        rsl[q].start(a.rs, r < a.R ? a.T0[r] : 1.0, r < a.R);
        dq[q] = 0;
    }
    // geometric schedules: every level's 1/T (fp64 and fp32) of the block's
    // runs, computed side by side once, so that a level advance is a table read
    const int ttab = a.ttab;
    const size_t tab_off = (state_bytes + (size_t)rpw * RUN_AREA_BYTES + 7) & ~(size_t)7;
    double *tT = reinterpret_cast<double *>(smem_raw + tab_off);
    float *tI = reinterpret_cast<float *>(tT + (size_t)rpw * ttab);
    if (ttab) {
        __syncthreads();  // the runs' level walkers are set
        for (int i = threadIdx.x; i < rpw * ttab; i += blockDim.x) {
            const int q = i / ttab;
            const double T = rsl[q].lw.geometric_T(a.rs, a.rs.first + (i - q * ttab));
            tT[i] = 1.0 / T;
            tI[i] = (float)(1.0 / T);
        }
    }
    const C g = (C)a.damping;

    const int L0 = a.L0, L1 = a.L1, L2 = a.L2;
    const int plane = L0 * L1, vol = plane * L2;
    const int H = L0 / 2;
    const uint8_t *__restrict__ bonds = a.bondbits;
    int lgs = lg_rpw;  // log2 of the byte stride of one site
    for (int sz = (int)sizeof(S); sz > 1; sz >>= 1)
        ++lgs;
    // byte offset (mod 2^32) of a site displacement
    auto ob = [&](int d) -> uint32_t { return (uint32_t)d << lgs; };
    // Column walk (when the threads of a run group cover whole planes of one
    // colour): the thread owns the x slot xh of row y in every kz-th plane,
    // so its x and y neighbour offsets are fixed and only z wraps.  Otherwise
    // the thread walks rows with a constant stride.
    const bool cols = (Tq % (H * L1)) == 0;
    const int xh = tq % H;
    const int kz = cols ? Tq / (H * L1) : 0;
    const int cy = cols ? (tq / H) % L1 : 0;
    const int cz0 = cols ? tq / (H * L1) : 0;
    const int row0 = tq / H;
    const int drow = Tq / H;
    const int nrows = L1 * L2;
    const int dy = drow % L1, dz = drow / L1;
    // the lanes of a wave share cz0 when no boundary between walk columns of
    // different start planes falls inside a wave
    const bool zuni = cols && (nq >= 64 || (H * L1) % (64 / nq) == 0);
    // x offsets by parity p of x: p = 0 has x + 1 inside the row, p = 1 has x - 1
    const uint32_t oxp0 = ob(1), oxm0 = ob(xh > 0 ? -1 : L0 - 1);
    const uint32_t oxp1 = ob(xh < H - 1 ? 1 : 1 - L0), oxm1 = ob(-1);
    const uint32_t cyp = ob(cy + 1 < L1 ? L0 : L0 - plane), cym = ob(cy > 0 ? -L0 : plane - L0);

    // (16 bytes, 16-aligned: the dynamic area that holds the state follows the
    // static one, and the state's 16-byte reads need it 16-aligned)
    __shared__ __attribute__((aligned(16))) unsigned vote[4];
    if (threadIdx.x == 0)
        vote[0] = vote[1] = 0u;
    __syncthreads();
    unsigned v_first = 0u;
    for (unsigned nvote = 0;; ++nvote) {
        // the runs' level state, advanced at the end of the previous sweep
        C scale[VEC];
        bool done[VEC];
        unsigned code = 0;
#pragma unroll
        for (int e = 0; e < VEC; ++e) {
            scale[e] = run_tscale<C>(rsl[q0 + e]);
            done[e] = rsl[q0 + e].done != 0;
            code |= done[e] ? 2u : 1u;
        }
        // block-uniform: leave when no run of the block anneals; the fast
        // update only while every run of the block does
        // (with a known sweep count only the first sweep votes: it decides
        // whether the block has a run at all and whether every run anneals,
        // which holds until the last sweep)
        unsigned v;
        if (a.fixed_sweeps > 0 && nvote > 0) {
            v = nvote < (unsigned)a.fixed_sweeps ? v_first : 0u;
        } else {
            v = block_vote(vote, nvote, code);
            v_first = v;
        }
        if (!(v & 1u))
            break;
        const bool all = !(v & 2u);
        C dloc[VEC];
#pragma unroll
        for (int e = 0; e < VEC; ++e)
            dloc[e] = 0;
        const unsigned char *mb = reinterpret_cast<const unsigned char *>(m) + q0 * sizeof(S);
        unsigned char *wb = reinterpret_cast<unsigned char *>(JAC ? m2 : m) + q0 * sizeof(S);
        // update site v at LDS byte offset vb (from the thread's run slot);
        // o*: byte offsets of its neighbours along +x, -x, +y, -y, +z, -z
        // LIVE: every run of the thread is still annealing, so (undamped, no
        // convergence tracking) the old value is not needed
        auto site = [&](auto live, int v, uint32_t vb, uint32_t oxp, uint32_t oxm, uint32_t oyp, uint32_t oym,
                        uint32_t ozp, uint32_t ozm) {
            constexpr bool FAST = decltype(live)::value && !DAMP && !TRACKD;
            const uint32_t b = bonds[(unsigned)v];
            C phi[VEC];
            if constexpr (sizeof(S) == 2 && VEC == 2) {
                // packed pair of fp16 runs: one 32-bit read per neighbour; each
                // term is one mixed-precision fma of the stored half with the
                // bond's +-1.0f (exact product, one rounding: the same value as
                // converting and adding)
                auto rd = [&](uint32_t o) -> uint32_t {
                    return *reinterpret_cast<const uint32_t *>(mb + (uint32_t)(vb + o));
                };
                auto sgn = [&](int k) -> float {
                    return __uint_as_float(((uint32_t)__builtin_amdgcn_sbfe((int)b, k, 1) & 0x80000000u) | 0x3f800000u);
                };
                auto lo = [](uint32_t u) -> float {
                    return (float)__builtin_bit_cast(_Float16, (unsigned short)(u & 0xffffu));
                };
                auto hi = [](uint32_t u) -> float {
                    return (float)__builtin_bit_cast(_Float16, (unsigned short)(u >> 16));
                };
                const uint32_t u0 = rd(oxp), u1 = rd(oxm), u2 = rd(oyp), u3 = rd(oym);
                const float s0 = sgn(0), s1 = sgn(1), s2 = sgn(2), s3 = sgn(3);
                float p0 = lo(u0) * s0, p1 = hi(u0) * s0;
                p0 = __builtin_fmaf(lo(u1), s1, p0);
                p1 = __builtin_fmaf(hi(u1), s1, p1);
                p0 = __builtin_fmaf(lo(u2), s2, p0);
                p1 = __builtin_fmaf(hi(u2), s2, p1);
                p0 = __builtin_fmaf(lo(u3), s3, p0);
                p1 = __builtin_fmaf(hi(u3), s3, p1);
                if (DIM == 3) {
                    const uint32_t u4 = rd(ozp), u5 = rd(ozm);
                    const float s4 = sgn(4), s5 = sgn(5);
                    p0 = __builtin_fmaf(lo(u4), s4, p0);
                    p1 = __builtin_fmaf(hi(u4), s4, p1);
                    p0 = __builtin_fmaf(lo(u5), s5, p0);
                    p1 = __builtin_fmaf(hi(u5), s5, p1);
                }
                phi[0] = p0;
                phi[1] = p1;
            } else {
                auto get = [&](uint32_t o) {
                    return lds_get<S, VEC>(reinterpret_cast<const S *>(mb + (uint32_t)(vb + o)));
                };
                const Pack<S, VEC> t0 = get(oxp), t1 = get(oxm), t2 = get(oyp), t3 = get(oym);
                const C s0 = (b & 1) ? (C)-1 : (C)1, s1 = (b & 2) ? (C)-1 : (C)1;
                const C s2 = (b & 4) ? (C)-1 : (C)1, s3 = (b & 8) ? (C)-1 : (C)1;
#pragma unroll
                for (int e = 0; e < VEC; ++e) {
                    C f = s0 * LStore<S>::ld(t0.v[e]);
                    f += s1 * LStore<S>::ld(t1.v[e]);
                    f += s2 * LStore<S>::ld(t2.v[e]);
                    f += s3 * LStore<S>::ld(t3.v[e]);
                    phi[e] = f;
                }
                if (DIM == 3) {
                    const Pack<S, VEC> t4 = get(ozp), t5 = get(ozm);
                    const C s4 = (b & 16) ? (C)-1 : (C)1, s5 = (b & 32) ? (C)-1 : (C)1;
#pragma unroll
                    for (int e = 0; e < VEC; ++e)
                        phi[e] += s4 * LStore<S>::ld(t4.v[e]) + s5 * LStore<S>::ld(t5.v[e]);
                }
            }
            if (HAS_H) {
                C hh;
                if constexpr (sizeof(C) == 8)
                    hh = a.hhalf64[v];
                else
                    hh = a.hhalf32[v];
#pragma unroll
                for (int e = 0; e < VEC; ++e)
                    phi[e] += hh;
            }
            Pack<S, VEC> nw;
            if constexpr (FAST) {
#pragma unroll
                for (int e = 0; e < VEC; ++e)
                    nw.v[e] = LStore<S>::st(l_tanh_run<sizeof(S) == 4 ? 2 : 0>(phi[e], scale[e]));
                lds_put<S, VEC>(reinterpret_cast<S *>(wb + vb), nw);
                return;
            }
            const Pack<S, VEC> old = lds_get<S, VEC>(reinterpret_cast<const S *>(mb + vb));
#pragma unroll
            for (int e = 0; e < VEC; ++e) {
                const C th = l_tanh_run<sizeof(S) == 4 ? 2 : 0>(phi[e], scale[e]);
                const C o = LStore<S>::ld(old.v[e]);
                C n = DAMP ? ((C)1 - g) * o + g * th : th;
                n = done[e] ? o : n;  // a finished run keeps its state
                nw.v[e] = done[e] ? old.v[e] : LStore<S>::st(n);
                const C dd = n > o ? n - o : o - n;
                dloc[e] = dd > dloc[e] ? dd : dloc[e];
            }
            lds_put<S, VEC>(reinterpret_cast<S *>(wb + vb), nw);
        };
        // Column walk of a packed pair of fp16 runs on a 3D lattice with an
        // even walk step, every run of the thread annealing, undamped and
        // without convergence tracking: the common case of long anneals, cut
        // to the fewest vector instructions per site.
        //  * the six bond signs come as one word per site holding three pairs
        //    of fp16 sign bits (bits 15 - j and 31 - j for the bonds of axis
        //    j), so a pair of +-1.0 halves is one and-or (and a shift) and each
        //    term is one mixed-precision fma of two halves (exact product, one
        //    rounding: the value of converting and adding);
        //  * one byte-offset register walks the column, kept opaque so that
        //    each neighbour address is one addition;
        //  * with a walk step of two planes the +z neighbour of one site is the
        //    -z neighbour of the next, so its word is carried, not re-read;
        //  * when a plane of one colour spans whole waves, z is the same on
        //    every lane and the loop runs on scalar registers.
        // The terms are summed in the order of the general site update
        // (+x, -x, +y, -y, +z, -z), so both give the same bits.
        auto pair_walk = [&](auto uni, int p) {
          if constexpr (sizeof(S) == 2 && VEC == 2 && DIM == 3) {
            constexpr bool UNI = decltype(uni)::value;
            int z = cz0;
            if constexpr (UNI)
                z = __builtin_amdgcn_readfirstlane(z);
            int v = L0 * (cy + L1 * z) + 2 * xh + p;
            uint32_t vb = ob(v);
            const int dv = kz * plane;
            const uint32_t dvb = ob(dv);
            const uint32_t xp = opaque(p ? oxp1 : oxp0), xm = opaque(p ? oxm1 : oxm0);
            const uint32_t yp = opaque(cyp), ym = opaque(cym);
            const uint32_t zp = ob(plane), zm = ob(-plane), zpw = ob(plane - vol), zmw = ob(vol - plane);
            const bool carry = kz == 2;
            const uint32_t *__restrict__ sg = a.bondsgn;
            auto rd = [&](uint32_t o) -> uint32_t { return *reinterpret_cast<const uint32_t *>(mb + o); };
            auto lo = [](uint32_t u) -> float {
                return (float)__builtin_bit_cast(_Float16, (unsigned short)(u & 0xffffu));
            };
            auto hi = [](uint32_t u) -> float {
                return (float)__builtin_bit_cast(_Float16, (unsigned short)(u >> 16));
            };
            const float nzero = __uint_as_float(opaque(0x80000000u));  // -0 + x == x, also for x = +-0
            // the sign-pair constants in registers (one and-or per pair)
            const uint32_t smask = opaque(0x80008000u), sone = opaque_uniform(0x3c003c00u);
            uint32_t uzm = rd(vb + (z > 0 ? zm : zmw));
            uint32_t w = sg[v];
            for (; z < L2; z += kz) {
                const uint32_t wn = sg[v + dv];  // the next site's signs (the table holds 2N words)
                const uint32_t u0 = rd(vb + xp), u1 = rd(vb + xm), u2 = rd(vb + yp), u3 = rd(vb + ym);
                const uint32_t u4 = rd(vb + (z + 1 < L2 ? zp : zpw));
                const uint32_t u5 = carry ? uzm : rd(vb + (z > 0 ? zm : zmw));
                const uint32_t sx = (w & smask) | sone;
                const uint32_t sy = ((w << 1) & smask) | sone;
                const uint32_t sz = ((w << 2) & smask) | sone;
                float p0 = __builtin_fmaf(lo(u0), lo(sx), nzero);
                float p1 = __builtin_fmaf(hi(u0), lo(sx), nzero);
                p0 = __builtin_fmaf(lo(u1), hi(sx), p0);
                p1 = __builtin_fmaf(hi(u1), hi(sx), p1);
                p0 = __builtin_fmaf(lo(u2), lo(sy), p0);
                p1 = __builtin_fmaf(hi(u2), lo(sy), p1);
                p0 = __builtin_fmaf(lo(u3), hi(sy), p0);
                p1 = __builtin_fmaf(hi(u3), hi(sy), p1);
                p0 = __builtin_fmaf(lo(u4), lo(sz), p0);
                p1 = __builtin_fmaf(hi(u4), lo(sz), p1);
                p0 = __builtin_fmaf(lo(u5), hi(sz), p0);
                p1 = __builtin_fmaf(hi(u5), hi(sz), p1);
                if (HAS_H) {
                    const float hh = a.hhalf32[v];
                    p0 += hh;
                    p1 += hh;
                }
                // rounded to halves after the fp32 tanh (kept whole, so the
                // conversion stays one packed instruction)
                *reinterpret_cast<uint32_t *>(wb + vb) =
                    pack_halves(opaque(l_tanh_run(p0, scale[0])), opaque(l_tanh_run(p1, scale[1])));
                uzm = u4;
                w = wn;
                v += dv;
                vb = opaque(vb + dvb);
            }
          }
        };
        auto sweep = [&](auto live) {
            for (int c = 0; c < (JAC ? 1 : 2); ++c) {
                constexpr bool PAIR_WALK = sizeof(S) == 2 && VEC == 2 && DIM == 3 && !JAC &&
                                           decltype(live)::value && !DAMP && !TRACKD;
                if constexpr (PAIR_WALK) {
                    if (cols && (kz & 1) == 0) {
                        const int p = (c + cy + cz0) & 1;
                        if (zuni)
                            pair_walk(std::true_type{}, p);
                        else
                            pair_walk(std::false_type{}, p);
                        __syncthreads();
                        continue;
                    }
                }
                if (cols && !JAC && (kz & 1) == 0) {
                    // even walk step: the thread's x parity is fixed for the whole
                    // walk, so its site, x and y offsets are constants; only the
                    // first and last planes of the lattice wrap along z
                    const int p = (c + cy + cz0) & 1;
                    int v = L0 * (cy + L1 * cz0) + 2 * xh + p;
                    uint32_t vb = ob(v);
                    const int dv = kz * plane;
                    const uint32_t dvb = opaque(ob(dv));
                    const uint32_t xp = opaque(p ? oxp1 : oxp0), xm = opaque(p ? oxm1 : oxm0);
                    const uint32_t yp = opaque(cyp), ym = opaque(cym);
                    const uint32_t zp = opaque(ob(plane)), zm = opaque(ob(-plane));
                    for (int z = cz0; z < L2; z += kz, v += dv, vb += dvb) {
                        if (z > 0 && z + 1 < L2) {
                            site(live, v, vb, xp, xm, yp, ym, zp, zm);
                        } else {
                            const uint32_t ozp = z + 1 < L2 ? zp : ob(plane - vol);
                            const uint32_t ozm = z > 0 ? zm : ob(vol - plane);
                            site(live, v, vb, xp, xm, yp, ym, ozp, ozm);
                        }
                    }
                } else if (cols) {
                    // site and byte offset carried along the column
                    int v0 = L0 * (cy + L1 * cz0) + 2 * xh;
                    uint32_t vb0 = ob(v0);
                    const int dv = kz * plane;
                    const uint32_t dvb = ob(dv);
                    for (int z = cz0; z < L2; z += kz, v0 += dv, vb0 += dvb) {
                        const uint32_t ozp = ob(z + 1 < L2 ? plane : plane - vol);
                        const uint32_t ozm = ob(z > 0 ? -plane : vol - plane);
    #pragma unroll
                        for (int pp = 0; pp < (JAC ? 2 : 1); ++pp) {
                            const int p = JAC ? pp : ((c + cy + z) & 1);
                            site(live, v0 + p, vb0 + (p ? oxp0 : 0u), p ? oxp1 : oxp0, p ? oxm1 : oxm0, cyp, cym, ozp, ozm);
                        }
                    }
                } else {
                    int y = row0 % L1, z = row0 / L1;
                    for (int rw = row0; rw < nrows; rw += drow) {
                        const uint32_t oyp = ob(y + 1 < L1 ? L0 : L0 - plane), oym = ob(y > 0 ? -L0 : plane - L0);
                        const uint32_t ozp = ob(z + 1 < L2 ? plane : plane - vol);
                        const uint32_t ozm = ob(z > 0 ? -plane : vol - plane);
    #pragma unroll
                        for (int pp = 0; pp < (JAC ? 2 : 1); ++pp) {
                            const int p = JAC ? pp : ((c + y + z) & 1);
                            const int v = L0 * rw + 2 * xh + p;
                            site(live, v, ob(v), p ? oxp1 : oxp0, p ? oxm1 : oxm0, oyp, oym, ozp, ozm);
                        }
                        y += dy;
                        z += dz;
                        if (y >= L1) {
                            y -= L1;
                            ++z;
                        }
                    }
                }
                __syncthreads();
            }
        };
        if (all)
            sweep(std::true_type{});
        else
            sweep(std::false_type{});
        if (JAC) {
            S *tmp = m;
            m = m2;
            m2 = tmp;
        }
        if (TRACKD) {
#pragma unroll
            for (int e = 0; e < VEC; ++e)
                if (!done[e])
                    atomicMax(&dq[q0 + e], __float_as_uint((float)dloc[e]));
            __syncthreads();
        }
        // each run's level advance (an fp64 exp and divide on geometric
        // schedules) on its own lane of the first wave, side by side
        for (int q = threadIdx.x; q < rpw; q += blockDim.x) {
            rsl[q].end_sweep(a.rs, __uint_as_float(dq[q]), TRACKD, a.max_sweeps, a.d_min,
                             ttab ? tT + (size_t)q * ttab : nullptr, ttab ? tI + (size_t)q * ttab : nullptr,
                             a.spl ? a.spl + (size_t)(blockIdx.x * rpw + q) * a.spl_cap : nullptr, a.spl_cap);
            dq[q] = 0;
        }
        // Keep this barrier.  Without it (the run-owning lanes feeding the
        // next sweep's vote directly) a build hung the GPU on a 2D fp32
        // lattice with 200 runs: the compiler split the sweep loop into a
        // nest in which owner and non-owner lanes of one wave took different
        // paths through the code holding the barriers.
        __syncthreads();
    }

    // outputs: rounded spins (s = +1 if m >= 0), optional final magnetisation
    for (int i = tq; i < N; i += Tq) {
        const Pack<S, VEC> p = lds_get<S, VEC>(&m[((size_t)i << lg_rpw) + q0]);
#pragma unroll
        for (int e = 0; e < VEC; ++e) {
            if (!live[e])
                continue;
            const C v = LStore<S>::ld(p.v[e]);
            a.spins[(size_t)(run0 + e) * N + i] = (v >= (C)0) ? 1 : -1;
            if (a.m_final)
                reinterpret_cast<C *>(a.m_final)[(size_t)i * a.R + run0 + e] = v;
        }
    }
    if (tq == 0)
#pragma unroll
        for (int e = 0; e < VEC; ++e)
            if (live[e])
                rsl[q0 + e].write_stats(a.runstat, run0 + e);
}

template <typename S, int VEC, int DIM, bool HAS_H, bool DAMP>
static void (*lat_pick3(bool jac, bool trackd))(GraphArgs, int)
{
    if (jac)
        return trackd ? k_lattice_solve<S, VEC, DIM, true, true, HAS_H, DAMP>
                      : k_lattice_solve<S, VEC, DIM, true, false, HAS_H, DAMP>;
    return trackd ? k_lattice_solve<S, VEC, DIM, false, true, HAS_H, DAMP>
                  : k_lattice_solve<S, VEC, DIM, false, false, HAS_H, DAMP>;
}

template <typename S, int VEC, bool HAS_H>
static void (*lat_pick(int dim, bool jac, bool trackd, bool damp))(GraphArgs, int)
{
    if (damp)
        return dim == 3 ? lat_pick3<S, VEC, 3, HAS_H, true>(jac, trackd) : lat_pick3<S, VEC, 2, HAS_H, true>(jac, trackd);
    return dim == 3 ? lat_pick3<S, VEC, 3, HAS_H, false>(jac, trackd) : lat_pick3<S, VEC, 2, HAS_H, false>(jac, trackd);
}

template <typename S, int VEC>
static hipError_t lat_launch(const GraphArgs &a, int lg_rpw, bool jac, bool trackd, dim3 grid, dim3 block,
                             size_t lds, hipStream_t s)
{
    const bool has_h = a.hhalf32 != nullptr;
    const bool damp = a.damping != 1.0;
    void (*fn)(GraphArgs, int) = has_h ? lat_pick<S, VEC, true>(a.dim, jac, trackd, damp)
                                       : lat_pick<S, VEC, false>(a.dim, jac, trackd, damp);
    if (lds > 65536) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(fn),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess)
            return e;
    }
    hipLaunchKernelGGL(fn, grid, block, lds, s, a, lg_rpw);
    return hipGetLastError();
}

// esz: bytes per stored magnetisation; rpw: runs per workgroup (power of two)
hipError_t launch_lattice_solve(const GraphArgs &a, int esz, int rpw, bool jac, bool trackd, hipStream_t s)
{
    int lg = 0;
    while ((1 << lg) < rpw)
        ++lg;
    const int vec = (rpw >= 2 && esz <= 4) ? 2 : 1;
    const int nq = rpw / vec;
    const int H = a.L0 / 2;
    const int N = a.N;
    const size_t per_run = (size_t)N * esz * (jac ? 2 : 1);
    const size_t base_lds = (((size_t)rpw * per_run + 15) & ~(size_t)15) + rpw * RUN_AREA_BYTES;
    // threads per run group, at most 1024 per workgroup: whole planes of one
    // colour (H x L1 sites) when one fits, so that threads walk columns along
    // z; otherwise a multiple of the half-row length H, no more than one per
    // site of a colour
    int Tq;
    const int P = H * a.L1;
    if (P <= 1024 / nq) {
        Tq = P * std::min(a.L2, (1024 / nq) / P);
    } else {
        Tq = std::min(1024 / nq, std::max(H, (N / 2 + H - 1) / H * H));
        Tq = std::max(H, Tq / H * H);
    }
    if (Tq * nq > 1024)
        return hipErrorInvalidConfiguration;
    dim3 grid((a.R + rpw - 1) / rpw), block(Tq * nq);
    GraphArgs b = a;
    b.ttab = level_table_fit(a.ttab, rpw, base_lds, Tq * nq, grid.x);
    const size_t lds = base_lds + level_table_bytes(rpw, b.ttab);
    if (esz == 8)
        return lat_launch<double, 1>(b, lg, jac, trackd, grid, block, lds, s);
    if (esz == 4)
        return vec == 2 ? lat_launch<float, 2>(b, lg, jac, trackd, grid, block, lds, s)
                        : lat_launch<float, 1>(b, lg, jac, trackd, grid, block, lds, s);
    return vec == 2 ? lat_launch<_Float16, 2>(b, lg, jac, trackd, grid, block, lds, s)
                    : lat_launch<_Float16, 1>(b, lg, jac, trackd, grid, block, lds, s);
}

}  // namespace mars
