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
hipError_t launch_sparse_solve(const GraphArgs &a, int esz, int rpw, int Tq, int vec, int lps, bool jac,
                               bool trackd, bool unit, hipStream_t s)
{
    int lg = 0;
    while ((1 << lg) < rpw)
        ++lg;
    const bool has_h = a.hhalf32 != nullptr;
    const bool damp = a.damping != 1.0;
    SparseFn fn = nullptr;
    if (lps > 1)
        fn = sparse_split_kernel(esz, vec, lps, damp, has_h, unit, jac, trackd);
    else if (esz == 8)
        fn = sp_pick_d<double, 1, 1>(damp, has_h, unit, jac, trackd);
    else if (esz == 4)
        fn = vec == 4   ? sp_pick_d<float, 4, 1>(damp, has_h, unit, jac, trackd)
             : vec == 2 ? sp_pick_d<float, 2, 1>(damp, has_h, unit, jac, trackd)
                        : sp_pick_d<float, 1, 1>(damp, has_h, unit, jac, trackd);
    else
        fn = vec == 4   ? sp_pick_d<_Float16, 4, 1>(damp, has_h, unit, jac, trackd)
             : vec == 2 ? sp_pick_d<_Float16, 2, 1>(damp, has_h, unit, jac, trackd)
                        : sp_pick_d<_Float16, 1, 1>(damp, has_h, unit, jac, trackd);
    if (!fn)
        return hipErrorInvalidValue;
    const size_t rows = (size_t)a.nslot + 1;
    const size_t base_lds = ((rows * rpw * esz * (jac ? 2 : 1) + 15) & ~(size_t)15) + rpw * RUN_AREA_BYTES;
    const int nq = rpw / (esz == 8 ? 1 : vec);
    const int threads = Tq * nq * lps;
    if (threads > 1024 || Tq < 1 || threads % 64 != 0)
        return hipErrorInvalidConfiguration;
    GraphArgs b = a;
    b.ttab = level_table_fit(a.ttab, rpw, base_lds, threads, (a.R + rpw - 1) / rpw);
    const size_t lds = base_lds + level_table_bytes(rpw, b.ttab);
    if (lds > 65536) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(fn),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess)
            return e;
    }
    dim3 grid((a.R + rpw - 1) / rpw), block(threads);
    hipLaunchKernelGGL(fn, grid, block, lds, s, b, lg);
    return hipGetLastError();
}

}  // namespace mars
