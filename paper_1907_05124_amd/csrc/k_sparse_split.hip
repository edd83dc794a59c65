// Lane-split instances of the sparse solver (sparse_solve.h): two or four
// lanes per (slot, run group) with four runs per group, fp32 and fp16
// storage.  A translation unit of their own so that they compile beside the
// one-lane instances.
#include "sparse_solve.h"

namespace mars {

SparseFn sparse_split_kernel(int esz, int vec, int lps, bool damp, bool has_h, bool unit, bool jac, bool trackd,
                             bool group)
{
    if (vec != 4 || (lps != 2 && lps != 4))
        return nullptr;
    if (group) {
        if (esz == 4)
            return lps == 4 ? sp_pick_group<float, 4, 4>(damp, has_h, unit, jac, trackd)
                            : sp_pick_group<float, 4, 2>(damp, has_h, unit, jac, trackd);
        if (esz == 2)
            return lps == 4 ? sp_pick_group<_Float16, 4, 4>(damp, has_h, unit, jac, trackd)
                            : sp_pick_group<_Float16, 4, 2>(damp, has_h, unit, jac, trackd);
        return nullptr;
    }
    if (esz == 4)
        return lps == 4 ? sp_pick_d<float, 4, 4>(damp, has_h, unit, jac, trackd)
                        : sp_pick_d<float, 4, 2>(damp, has_h, unit, jac, trackd);
    if (esz == 2)
        return lps == 4 ? sp_pick_d<_Float16, 4, 4>(damp, has_h, unit, jac, trackd)
                        : sp_pick_d<_Float16, 4, 2>(damp, has_h, unit, jac, trackd);
    return nullptr;
}

}  // namespace mars
