// Sparse instances whose one-run state does not fit in LDS: the same
// colour-phased update as the LDS-resident solver (sparse_solve.h), with the
// magnetisations in device memory, m[slot * ldr + r] (row = slot in the
// sliced-ELL labelling, runs contiguous, row nslot all zeros), and one
// cooperative launch for the whole anneal:
//  * a phase is a grid-stride loop over (slot of the class, group of VEC
//    runs) items, run groups fastest, so the lanes of a wave read
//    consecutive runs of one neighbour row (coalesced gathers); the items go
//    chunk by chunk of runs, sized so that the state of a chunk's runs fits
//    well inside the MALL, where a row segment read by one neighbour stays
//    for the others (random graphs have no locality to exploit otherwise);
//  * a grid barrier separates the phases (a class reads the values the
//    classes before it wrote in the same sweep), and two more end a sweep:
//    after the per-run level advance, and after the vote that ends the anneal;
//  * the paper's stopping rule needs, per run, only whether some change in
//    the sweep reached d_min (d < d_min is decided on the largest change): a
//    per-run flag set by the first update that reaches it replaces a max over
//    every spin-update.
// The synchronous (one-phase) variant writes a second copy and swaps.
#include <hip/hip_cooperative_groups.h>

#include <algorithm>

#include "sparse_solve.h"

namespace cg = cooperative_groups;

namespace mars {

constexpr int kGlobalThreads = 1024;

template <typename S, int VEC>
__global__ __launch_bounds__(kGlobalThreads) void k_sparse_global(SparseGlobalArgs g)
{
    typedef typename LStore<S>::C C;
    cg::grid_group grid = cg::this_grid();
    const GraphArgs &a = g.a;
    const int N = a.N;
    const int ns = a.nslot;
    const int rows = ns + 1;
    const int ldr = g.ldr;
    const int ngr = ldr / VEC;
    const int ngc = g.ngc;  // run groups per chunk of a phase's items
    const int nchunk = (ngr + ngc - 1) / ngc;
    const size_t G = (size_t)gridDim.x * blockDim.x;
    const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    S *m = reinterpret_cast<S *>(g.m);
    S *m2 = g.jac ? reinterpret_cast<S *>(g.m2) : m;
    C *tsc = reinterpret_cast<C *>(g.tscale);
    const bool trackd = a.max_sweeps > 1;
    const C gam = (C)a.damping;
    const bool damp = a.damping != 1.0;

    if (t == 0) {
        g.live[0] = 0u;
        g.live[1] = 0u;
    }
    // initial state (Algorithm 1: s_i := rand(-1, 1)); padding slots, padded
    // runs and the zero row hold 0 in both copies
    for (size_t idx = t; idx < (size_t)rows * ngr; idx += G) {
        const int i = (int)(idx / ngr);
        const int r0 = (int)(idx % ngr) * VEC;
        const int v = i < ns ? a.perm[i] : -1;
        Pack<S, VEC> p;
#pragma unroll
        for (int e = 0; e < VEC; ++e) {
            C x = 0;
            if (v >= 0 && r0 + e < a.R)
                x = a.m0 ? (C)(reinterpret_cast<const C *>(a.m0))[(size_t)v * a.R + r0 + e]
                         : (C)draw_m0(a.seed, r0 + e, v);
            p.v[e] = LStore<S>::st(x);
        }
        lds_put<S, VEC>(&m[(size_t)i * ldr + r0], p);
        if (g.jac)
            lds_put<S, VEC>(&m2[(size_t)i * ldr + r0], p);
    }
    grid.sync();  // the vote words are clear
    // the runs' level state; padded runs start finished
    for (size_t r = t; r < (size_t)ldr; r += G) {
        RunState &q = reinterpret_cast<RunState *>(g.rs)[r];
        q.start(a.rs, r < (size_t)a.R ? a.T0[r] : 1.0, r < (size_t)a.R);
        tsc[r] = run_tscale<C>(q);
        g.rdone[r] = q.done;
        g.flag[r] = 0u;
        if (!q.done)
            atomicOr(&g.live[0], 1u);
    }
    grid.sync();

    const uint32_t colmask = g.unit ? 0x7fffffffu : 0xffffffu;
    const int2 *rec = reinterpret_cast<const int2 *>(a.sl_meta);
    for (unsigned k = 0;; ++k) {
        if (__hip_atomic_load(&g.live[k & 1u], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0u)
            break;
        if (t == 0)
            g.live[(k + 1u) & 1u] = 0u;  // read by every thread only after the next barrier
        const int nph = g.jac ? 1 : a.nphase;
        for (int c = 0; c < nph; ++c) {
            const int sb = g.jac ? 0 : a.cls[2 * c];
            const int sn = g.jac ? ns : a.cls[2 * c + 1];
            // items run-chunk by run-chunk (all slots of the class for ngc run
            // groups, then the next ngc): the rows' segments a chunk gathers
            // stay in the MALL while its items run
            const size_t per_chunk = (size_t)sn * ngc;
            for (size_t idx = t; idx < per_chunk * nchunk; idx += G) {
                const size_t chunk = idx / per_chunk;
                const size_t rem = idx - chunk * per_chunk;
                const int slot = sb + (int)(rem / ngc);
                const int rg = (int)(chunk * ngc + rem % ngc);
                if (rg >= ngr)
                    continue;
                const int r0 = rg * VEC;
                C scale[VEC];
                bool done[VEC];
#pragma unroll
                for (int e = 0; e < VEC; ++e) {
                    scale[e] = tsc[r0 + e];
                    done[e] = g.rdone[r0 + e] != 0;
                }
                const int2 rc = rec[slot / SELL_H];
                const uint4 *gp = reinterpret_cast<const uint4 *>(a.colsell + rc.x) + (slot % SELL_H);
                C phi[VEC];
#pragma unroll
                for (int e = 0; e < VEC; ++e)
                    phi[e] = 0;
                for (int j = 0, gi = 0; j < rc.y; j += SELL_W, ++gi) {
                    const uint4 cb = gp[(size_t)gi * SELL_H];
                    const uint32_t ent[SELL_W] = {cb.x, cb.y, cb.z, cb.w};
#pragma unroll
                    for (int u = 0; u < SELL_W; ++u) {
                        const C wt = g.unit ? entry_weight<C, true>(ent[u]) : entry_weight<C, false>(ent[u]);
                        const Pack<S, VEC> nb = lds_get<S, VEC>(&m[(size_t)(ent[u] & colmask) * ldr + r0]);
#pragma unroll
                        for (int e = 0; e < VEC; ++e)
                            phi[e] += wt * LStore<S>::ld(nb.v[e]);
                    }
                }
                if (a.hhalf32) {
                    C hh;
                    if constexpr (sizeof(C) == 8)
                        hh = a.hhalf64[slot];
                    else
                        hh = a.hhalf32[slot];
#pragma unroll
                    for (int e = 0; e < VEC; ++e)
                        phi[e] += hh;
                }
                const size_t o = (size_t)slot * ldr + r0;
                const Pack<S, VEC> old = lds_get<S, VEC>(&m[o]);
                Pack<S, VEC> nw;
#pragma unroll
                for (int e = 0; e < VEC; ++e) {
                    const C th = l_tanh_run<sizeof(S) == 4 ? 2 : 1>(phi[e], scale[e]);
                    const C ov = LStore<S>::ld(old.v[e]);
                    C n = damp ? ((C)1 - gam) * ov + gam * th : th;
                    n = done[e] ? ov : n;  // a finished run keeps its state
                    nw.v[e] = done[e] ? old.v[e] : (damp ? lds_keep_sign<S>(n) : LStore<S>::st(n));
                    if (trackd && !done[e]) {
                        // the sweep's largest change reaches d_min iff one of
                        // its changes does (the comparison in the precision
                        // the LDS solvers decide it in)
                        const C dd = n > ov ? n - ov : ov - n;
                        if (!((double)(float)dd < a.d_min) &&
                            __hip_atomic_load(&g.flag[r0 + e], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0u)
                            atomicOr(&g.flag[r0 + e], 1u);
                    }
                }
                lds_put<S, VEC>(&m2[o], nw);
            }
            grid.sync();
        }
        if (g.jac) {
            S *tmp = m;
            m = m2;
            m2 = tmp;
        }
        // each run's level advance
        for (size_t r = t; r < (size_t)a.R; r += G) {
            RunState &q = reinterpret_cast<RunState *>(g.rs)[r];
            q.end_sweep(a.rs, g.flag[r] ? __builtin_huge_valf() : 0.0f, trackd, a.max_sweeps, a.d_min, nullptr, nullptr,
                        a.spl ? a.spl + r * a.spl_cap : nullptr, a.spl_cap);
            g.flag[r] = 0u;
            tsc[r] = run_tscale<C>(q);
            g.rdone[r] = q.done;
            if (!q.done)
                atomicOr(&g.live[(k + 1u) & 1u], 1u);
        }
        grid.sync();
    }

    // outputs in the caller's labels: rounded spins (s = +1 if m >= 0) and the
    // optional final magnetisation
    for (size_t idx = t; idx < (size_t)ns * ngr; idx += G) {
        const int i = (int)(idx / ngr);
        const int r0 = (int)(idx % ngr) * VEC;
        const int v = a.perm[i];
        if (v < 0)
            continue;
        const Pack<S, VEC> p = lds_get<S, VEC>(&m[(size_t)i * ldr + r0]);
#pragma unroll
        for (int e = 0; e < VEC; ++e) {
            if (r0 + e >= a.R)
                continue;
            const C x = LStore<S>::ld(p.v[e]);
            a.spins[(size_t)(r0 + e) * N + v] = (x >= (C)0) ? 1 : -1;
            if (a.m_final)
                reinterpret_cast<C *>(a.m_final)[(size_t)v * a.R + r0 + e] = x;
        }
    }
    for (size_t r = t; r < (size_t)a.R; r += G)
        reinterpret_cast<RunState *>(g.rs)[r].write_stats(a.runstat, (int)r);
}

hipError_t launch_sparse_global(const SparseGlobalArgs &args, int esz, hipStream_t s)
{
    const void *fn = esz == 8   ? reinterpret_cast<const void *>(&k_sparse_global<double, 1>)
                     : esz == 4 ? reinterpret_cast<const void *>(&k_sparse_global<float, 4>)
                                : reinterpret_cast<const void *>(&k_sparse_global<_Float16, 4>);
    int dev = 0, per_cu = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess)
        return e;
    hipDeviceProp_t prop;
    if ((e = hipGetDeviceProperties(&prop, dev)) != hipSuccess)
        return e;
    if ((e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, kGlobalThreads, 0)) != hipSuccess)
        return e;
    if (per_cu < 1)
        return hipErrorInvalidConfiguration;
    // every resident workgroup (the grid barriers need all of them at once),
    // no more than the widest item loop needs
    const int vec = esz == 8 ? 1 : 4;
    const size_t items = (size_t)(args.a.nslot + 1) * (args.ldr / vec);
    const int grid = (int)std::max<size_t>(1, std::min<size_t>((items + kGlobalThreads - 1) / kGlobalThreads,
                                                               (size_t)per_cu * prop.multiProcessorCount));
    SparseGlobalArgs a = args;
    void *kargs[] = {&a};
    return hipLaunchCooperativeKernel(fn, dim3(grid), dim3(kGlobalThreads), kargs, 0, s);
}

}  // namespace mars
