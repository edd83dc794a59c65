// Sparse (CSR-defined) instances: a workgroup anneals a block of rpw runs
// from start to finish with their magnetisations in LDS, m[slot * rpw + q],
// in the sliced-ELL labelling built at creation (colour classes contiguous,
// each sorted by degree and padded to whole slices of SELL_H slots).
//  * A colour class is an independent set (no coupling inside it), so its
//    slots are updated in place; classes run in colour order with a barrier
//    between them (sequential dynamics in colour order).  The synchronous
//    variant writes a second copy and swaps after each sweep.
//  * Each thread updates one slot for VEC consecutive runs: one entry read
//    (neighbour slot and weight) serves VEC terms, and the VEC values of a
//    neighbour arrive in one LDS read.
//  * The threads of a wave cover consecutive slots, so their entry reads
//    (column j of a slice) are consecutive words.
//  * Missing entries of a slice point at the all-zero row nslot, so every
//    lane of a slice runs the same number of terms; slice widths are whole
//    groups of SELL_W entries, read together before their terms are summed.
//  * With +-1 weights the weight is rebuilt as +-1.0f from the entry's sign
//    bit (one bit operation) instead of an integer-to-float conversion.
#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <type_traits>

#include "common_device.h"
#include "lds_state.h"
#include "mars_internal.h"

namespace mars {

template <typename C, bool UNIT>
__device__ inline C entry_weight(uint32_t cb)
{
    if constexpr (UNIT)
        return (C)__uint_as_float((cb & 0x80000000u) | 0x3f800000u);
    else
        return (C)((int32_t)cb >> 24);
}

template <typename S, int VEC, bool JAC, bool TRACKD, bool HAS_H, bool UNIT, bool DAMP>
__global__ __launch_bounds__(1024) void k_sparse_solve(GraphArgs a, int lg_rpw)
{
    typedef typename LStore<S>::C C;
    extern __shared__ __attribute__((aligned(16))) unsigned char smem_raw[];
    const int N = a.N;
    const int ns = a.nslot;
    const int rows = ns + 1;  // row ns: all zeros
    const int rpw = 1 << lg_rpw;
    S *m = reinterpret_cast<S *>(smem_raw);
    S *m2 = JAC ? m + (size_t)rows * rpw : m;
    const size_t state_bytes = ((size_t)rows * rpw * sizeof(S) * (JAC ? 2 : 1) + 15) & ~(size_t)15;
    RunState *rsl = reinterpret_cast<RunState *>(smem_raw + state_bytes);
    uint32_t *dq = reinterpret_cast<uint32_t *>(rsl + rpw);

    const int nq = rpw / VEC;
    const int qg = threadIdx.x % nq;
    const int q0 = qg * VEC;
    const int tq = threadIdx.x / nq;
    const int Tq = blockDim.x / nq;
    const int run0 = blockIdx.x * rpw + q0;

    // initial state (Algorithm 1: s_i := rand(-1, 1)); padding slots and the
    // zero row hold 0 in both copies
    for (int i = tq; i < rows; i += Tq) {
        const int v = i < ns ? a.perm[i] : -1;
        Pack<S, VEC> p;
#pragma unroll
        for (int e = 0; e < VEC; ++e) {
            C x = 0;
            if (v >= 0 && run0 + e < a.R)
                x = a.m0 ? (C)(reinterpret_cast<const C *>(a.m0))[(size_t)v * a.R + run0 + e]
                         : (C)draw_m0(a.seed, run0 + e, v);
            p.v[e] = LStore<S>::st(x);
        }
        lds_put<S, VEC>(&m[((size_t)i << lg_rpw) + q0], p);
        if (JAC)
            lds_put<S, VEC>(&m2[((size_t)i << lg_rpw) + q0], p);
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
    int lgs = lg_rpw;  // log2 of the byte stride of one slot's row
    for (int sz = (int)sizeof(S); sz > 1; sz >>= 1)
        ++lgs;
    const uint32_t *__restrict__ colsell = a.colsell;
    const bool long_rows = a.long_rows != 0;
    const int32_t *__restrict__ meta = a.sl_meta;

    // (16 bytes, 16-aligned: the dynamic area that holds the state follows the
    // static one, and the state's 16-byte reads need it 16-aligned)
    __shared__ __attribute__((aligned(16))) unsigned vote[4];
    if (threadIdx.x == 0)
        vote[0] = vote[1] = 0u;
    __syncthreads();
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
        const unsigned v = block_vote(vote, nvote, code);
        if (!(v & 1u))
            break;
        const bool all = !(v & 2u);
        C dloc[VEC];
#pragma unroll
        for (int e = 0; e < VEC; ++e)
            dloc[e] = 0;
        auto sweep = [&](auto live) {
            constexpr bool FAST = decltype(live)::value && !DAMP && !TRACKD;
            const int nph = JAC ? 1 : a.nphase;
            for (int c = 0; c < nph; ++c) {
                // the synchronous sweep visits every slot (padding slots are inert:
                // no terms, zero field, state 0)
                const int sb = JAC ? 0 : a.cls[2 * c];
                const int sn = JAC ? ns : a.cls[2 * c + 1];
                const unsigned char *mb = reinterpret_cast<const unsigned char *>(m) + q0 * sizeof(S);
                unsigned char *wb = reinterpret_cast<unsigned char *>(JAC ? m2 : m) + q0 * sizeof(S);
                // the slice record (offset, width) of the thread's next slot is
                // read while the current one is computed (index clamped to the
                // class's last slot: in bounds, unused past the end)
                const int2 *rec = reinterpret_cast<const int2 *>(meta);
                const unsigned last = (unsigned)min(sb + max(sn, 1) - 1, ns - 1);
                int2 rc = rec[min((unsigned)(sb + tq), last) / SELL_H];
                for (int it = tq; it < sn; it += Tq) {
                    const int slot = sb + it;
                    const int2 rn = rec[min((unsigned)(slot + Tq), last) / SELL_H];
                    const int off = rc.x;
                    const int w = rc.y;
                    rc = rn;
                    // the slot's entry groups: 16 contiguous bytes each, one
                    // slice (SELL_H slots) apart
                    const uint4 *gp = reinterpret_cast<const uint4 *>(colsell + off) + ((unsigned)slot % SELL_H);
                    C phi[VEC];
#pragma unroll
                    for (int e = 0; e < VEC; ++e)
                        phi[e] = 0;
                    // w is a multiple of SELL_W: whole groups, no remainder loop.
                    // A +-1 entry holds only its sign above the slot (bit 31,
                    // shifted out with the byte offset: lgs >= 1), an int8
                    // entry its weight byte in bits 24-31
                    constexpr uint32_t colmask = UNIT ? 0xffffffffu : 0xffffffu;
                    auto group = [&](const uint4 cb) {
                        const uint32_t ent[SELL_W] = {cb.x, cb.y, cb.z, cb.w};
#pragma unroll
                        for (int u = 0; u < SELL_W; ++u) {
                            const C wt = entry_weight<C, UNIT>(ent[u]);
                            const Pack<S, VEC> t =
                                lds_get<S, VEC>(reinterpret_cast<const S *>(mb + ((ent[u] & colmask) << lgs)));
#pragma unroll
                            for (int e = 0; e < VEC; ++e)
                                phi[e] += wt * LStore<S>::ld(t.v[e]);
                        }
                    };
                    if (!long_rows) {
                        for (int j = 0, g = 0; j < w; j += SELL_W, ++g)
                            group(gp[g * SELL_H]);
                    } else if (w > 0) {
                        // long rows (high average degree): entry groups are
                        // read ahead of the one being summed; reads run up to
                        // two groups past the slice, into the next slice or
                        // the table's padding (in bounds, unused), and a slice
                        // without entries reads nothing
                        uint4 cb = gp[0], n1 = gp[SELL_H];
                        for (int j = 0, g = 2; j < w; j += SELL_W, ++g) {
                            // (an opaque index keeps the read ahead: otherwise
                            // it is turned back into a read of the current
                            // group at its use)
                            const uint4 n2 = gp[opaque((uint32_t)g * SELL_H)];
                            group(cb);
                            cb = n1;
                            n1 = n2;
                        }
                    }
                    if (HAS_H) {
                        C hh;
                        if constexpr (sizeof(C) == 8)
                            hh = a.hhalf64[slot];
                        else
                            hh = a.hhalf32[slot];
#pragma unroll
                        for (int e = 0; e < VEC; ++e)
                            phi[e] += hh;
                    }
                    const uint32_t o_slot = (uint32_t)slot << lgs;
                    Pack<S, VEC> nw;
                    if constexpr (FAST) {
                        // every run of the thread still anneals, undamped, no
                        // convergence tracking: the old value is not needed
#pragma unroll
                        for (int e = 0; e < VEC; ++e)
                            nw.v[e] = lds_keep_sign<S>(l_tanh_run<sizeof(S) == 4 ? 2 : 1>(phi[e], scale[e]));
                        lds_put<S, VEC>(reinterpret_cast<S *>(wb + o_slot), nw);
                        continue;
                    }
                    const Pack<S, VEC> old = lds_get<S, VEC>(reinterpret_cast<const S *>(mb + o_slot));
#pragma unroll
                    for (int e = 0; e < VEC; ++e) {
                        const C th = l_tanh_run<sizeof(S) == 4 ? 2 : 1>(phi[e], scale[e]);
                        const C o = LStore<S>::ld(old.v[e]);
                        C n = DAMP ? ((C)1 - g) * o + g * th : th;
                        n = done[e] ? o : n;  // a finished run keeps its state
                        nw.v[e] = done[e] ? old.v[e] : lds_keep_sign<S>(n);
                        const C dd = n > o ? n - o : o - n;
                        dloc[e] = dd > dloc[e] ? dd : dloc[e];
                    }
                    lds_put<S, VEC>(reinterpret_cast<S *>(wb + o_slot), nw);
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

    // outputs in the caller's labels: rounded spins (s = +1 if m >= 0) and the
    // optional final magnetisation
    for (int i = tq; i < ns; i += Tq) {
        const int v = a.perm[i];
        if (v < 0)
            continue;
        const Pack<S, VEC> p = lds_get<S, VEC>(&m[((size_t)i << lg_rpw) + q0]);
#pragma unroll
        for (int e = 0; e < VEC; ++e) {
            if (run0 + e >= a.R)
                continue;
            const C x = LStore<S>::ld(p.v[e]);
            a.spins[(size_t)(run0 + e) * N + v] = (x >= (C)0) ? 1 : -1;
            if (a.m_final)
                reinterpret_cast<C *>(a.m_final)[(size_t)v * a.R + run0 + e] = x;
        }
    }
    if (tq == 0)
#pragma unroll
        for (int e = 0; e < VEC; ++e)
            if (run0 + e < a.R)
                rsl[q0 + e].write_stats(a.runstat, run0 + e);
}

typedef void (*SparseFn)(GraphArgs, int);

template <typename S, int VEC, bool HAS_H, bool UNIT, bool DAMP>
static SparseFn sp_pick(bool jac, bool trackd)
{
    if (jac)
        return trackd ? k_sparse_solve<S, VEC, true, true, HAS_H, UNIT, DAMP>
                      : k_sparse_solve<S, VEC, true, false, HAS_H, UNIT, DAMP>;
    return trackd ? k_sparse_solve<S, VEC, false, true, HAS_H, UNIT, DAMP>
                  : k_sparse_solve<S, VEC, false, false, HAS_H, UNIT, DAMP>;
}

template <typename S, int VEC, bool DAMP>
static SparseFn sp_pick_hu(bool has_h, bool unit, bool jac, bool trackd)
{
    if (has_h)
        return unit ? sp_pick<S, VEC, true, true, DAMP>(jac, trackd) : sp_pick<S, VEC, true, false, DAMP>(jac, trackd);
    return unit ? sp_pick<S, VEC, false, true, DAMP>(jac, trackd) : sp_pick<S, VEC, false, false, DAMP>(jac, trackd);
}

template <typename S, int VEC>
static SparseFn sp_pick_d(bool damp, bool has_h, bool unit, bool jac, bool trackd)
{
    return damp ? sp_pick_hu<S, VEC, true>(has_h, unit, jac, trackd) : sp_pick_hu<S, VEC, false>(has_h, unit, jac, trackd);
}

// esz: bytes per stored magnetisation; rpw: runs per workgroup (power of two);
// Tq: threads per run group; vec: runs per thread (1, 2 or 4, dividing rpw)
hipError_t launch_sparse_solve(const GraphArgs &a, int esz, int rpw, int Tq, int vec, bool jac, bool trackd,
                               bool unit, hipStream_t s)
{
    int lg = 0;
    while ((1 << lg) < rpw)
        ++lg;
    const bool has_h = a.hhalf32 != nullptr;
    const bool damp = a.damping != 1.0;
    SparseFn fn;
    if (esz == 8)
        fn = sp_pick_d<double, 1>(damp, has_h, unit, jac, trackd);
    else if (esz == 4)
        fn = vec == 4   ? sp_pick_d<float, 4>(damp, has_h, unit, jac, trackd)
             : vec == 2 ? sp_pick_d<float, 2>(damp, has_h, unit, jac, trackd)
                        : sp_pick_d<float, 1>(damp, has_h, unit, jac, trackd);
    else
        fn = vec == 4   ? sp_pick_d<_Float16, 4>(damp, has_h, unit, jac, trackd)
             : vec == 2 ? sp_pick_d<_Float16, 2>(damp, has_h, unit, jac, trackd)
                        : sp_pick_d<_Float16, 1>(damp, has_h, unit, jac, trackd);
    const size_t rows = (size_t)a.nslot + 1;
    const size_t base_lds = ((rows * rpw * esz * (jac ? 2 : 1) + 15) & ~(size_t)15) + rpw * RUN_AREA_BYTES;
    const int nq = rpw / (esz == 8 ? 1 : vec);
    if (Tq * nq > 1024 || Tq < 1)
        return hipErrorInvalidConfiguration;
    GraphArgs b = a;
    b.ttab = level_table_fit(a.ttab, rpw, base_lds, Tq * nq, (a.R + rpw - 1) / rpw);
    const size_t lds = base_lds + level_table_bytes(rpw, b.ttab);
    if (lds > 65536) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(fn),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess)
            return e;
    }
    dim3 grid((a.R + rpw - 1) / rpw), block(Tq * nq);
    hipLaunchKernelGGL(fn, grid, block, lds, s, b, lg);
    return hipGetLastError();
}

}  // namespace mars
