// Sparse (CSR-defined) instances: the launcher of the LDS-resident solver
// (kernel in sparse_solve.h) and its one-lane-per-slot instances; the
// lane-split instances are in k_sparse_split.hip.
#include <algorithm>
#include <cmath>
#include <cstdlib>

#include "sparse_solve.h"

namespace mars {

// esz: bytes per stored magnetisation; rpw: runs per workgroup (power of two);
// Tq: slots in flight per run group; vec: runs per lane group (1, 2 or 4,
// dividing rpw); lps: lanes per (slot, run group) (1, or 2 or 4 dividing vec
// with fp32 fields)
hipError_t plan_sparse_solve(const GraphArgs &a, int esz, int rpw, int Tq, int vec, int lps, bool jac, bool trackd,
                             bool unit, SparsePlan *plan)
{
    int lg = 0;
    while ((1 << lg) < rpw)
        ++lg;
    const bool has_h = a.hhalf32 != nullptr;
    const bool damp = a.damping != 1.0;
    SparseFn fn = nullptr, gfn = nullptr;
    if (lps > 1) {
        fn = sparse_split_kernel(esz, vec, lps, damp, has_h, unit, jac, trackd, false);
        gfn = sparse_split_kernel(esz, vec, lps, damp, has_h, unit, jac, trackd, true);
    } else if (esz == 8) {
        fn = sp_pick_d<double, 1, 1>(damp, has_h, unit, jac, trackd);
        gfn = sp_pick_group<double, 1, 1>(damp, has_h, unit, jac, trackd);
    } else if (esz == 4) {
        fn = vec == 4   ? sp_pick_d<float, 4, 1>(damp, has_h, unit, jac, trackd)
             : vec == 2 ? sp_pick_d<float, 2, 1>(damp, has_h, unit, jac, trackd)
                        : sp_pick_d<float, 1, 1>(damp, has_h, unit, jac, trackd);
        gfn = vec == 4   ? sp_pick_group<float, 4, 1>(damp, has_h, unit, jac, trackd)
              : vec == 2 ? sp_pick_group<float, 2, 1>(damp, has_h, unit, jac, trackd)
                         : sp_pick_group<float, 1, 1>(damp, has_h, unit, jac, trackd);
    } else {
        fn = vec == 4   ? sp_pick_d<_Float16, 4, 1>(damp, has_h, unit, jac, trackd)
             : vec == 2 ? sp_pick_d<_Float16, 2, 1>(damp, has_h, unit, jac, trackd)
                        : sp_pick_d<_Float16, 1, 1>(damp, has_h, unit, jac, trackd);
        gfn = vec == 4   ? sp_pick_group<_Float16, 4, 1>(damp, has_h, unit, jac, trackd)
              : vec == 2 ? sp_pick_group<_Float16, 2, 1>(damp, has_h, unit, jac, trackd)
                         : sp_pick_group<_Float16, 1, 1>(damp, has_h, unit, jac, trackd);
    }
    if (!fn)
        return hipErrorInvalidValue;
    const size_t rows = (size_t)a.nslot + 1;
    const size_t base_lds = ((rows * rpw * esz * (jac ? 2 : 1) + 15) & ~(size_t)15) + rpw * RUN_AREA_BYTES;
    const int nq = rpw / (esz == 8 ? 1 : vec);
    const int threads = Tq * nq * lps;
    if (threads > 1024 || Tq < 1 || threads % 64 != 0)
        return hipErrorInvalidConfiguration;
    plan->fn = reinterpret_cast<const void *>(fn);
    plan->gfn = reinterpret_cast<const void *>(gfn);
    plan->args = a;
    plan->args.ttab = level_table_fit(a.ttab, rpw, base_lds, threads, (a.R + rpw - 1) / rpw);
    plan->lg = lg;
    plan->blocks = (a.R + rpw - 1) / rpw;
    plan->threads = threads;
    plan->lds = base_lds + level_table_bytes(rpw, plan->args.ttab);
    return hipSuccess;
}

// Launches solves with one kernel: one plan alone (no descriptor), or several
// of the same kernel through the group descriptor (host_desc is filled and
// copied to dev_desc on the stream; both stay untouched until the launch has
// run).
hipError_t launch_sparse_plans(const SparsePlan *plans, int n, GraphGroup *host_desc, GraphGroup *dev_desc,
                               hipStream_t s)
{
    if (n < 1 || n > GRAPH_GROUP_MAX)
        return hipErrorInvalidValue;
    int blocks = 0, threads = 0;
    size_t lds = 0;
    // one solve: its own kernel; several: the group instantiation they share
    const void *kfn = n == 1 ? plans[0].fn : plans[0].gfn;
    for (int k = 0; k < n; ++k) {
        if (!kfn || (n > 1 && plans[k].gfn != kfn))
            return hipErrorInvalidValue;
        blocks += plans[k].blocks;
        threads = std::max(threads, plans[k].threads);
        lds = std::max(lds, plans[k].lds);
    }
    SparseFn fn = reinterpret_cast<SparseFn>(const_cast<void *>(kfn));
    if (lds > 65536) {
        hipError_t e = hipFuncSetAttribute(kfn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess)
            return e;
    }
    const GraphGroup *grp = nullptr;
    if (n > 1) {
        if (!host_desc || !dev_desc)
            return hipErrorInvalidValue;
        host_desc->count = n;
        host_desc->first[0] = 0;
        for (int k = 0; k < n; ++k) {
            host_desc->first[k + 1] = host_desc->first[k] + plans[k].blocks;
            host_desc->lg[k] = plans[k].lg;
            host_desc->args[k] = plans[k].args;
        }
        hipError_t e = hipMemcpyAsync(dev_desc, host_desc, sizeof(GraphGroup), hipMemcpyHostToDevice, s);
        if (e != hipSuccess)
            return e;
        grp = dev_desc;
    }
    hipLaunchKernelGGL(fn, dim3(blocks), dim3(threads), lds, s, plans[0].args, plans[0].lg, grp);
    return hipGetLastError();
}

hipError_t launch_sparse_solve(const GraphArgs &a, int esz, int rpw, int Tq, int vec, int lps, bool jac,
                               bool trackd, bool unit, hipStream_t s)
{
    SparsePlan p;
    hipError_t e = plan_sparse_solve(a, esz, rpw, Tq, vec, lps, jac, trackd, unit, &p);
    if (e != hipSuccess)
        return e;
    return launch_sparse_plans(&p, 1, nullptr, nullptr, s);
}

}  // namespace mars
