// The batched solver's phase kernel: one launch covers one update phase of
// several dense instances (BF16 form), built on the single-instance tile of
// dense_phase_bf16.h (device code; included by the library's BF16 unit).
#pragma once

#include <hip/hip_cooperative_groups.h>

#include "dense_phase_bf16.h"

namespace mars {

// One phase of several dense instances in one launch (the batched solver).
// Member descriptors and the phase's slots travel as kernel arguments and
// stay fixed while the batch's membership is unchanged; a member's level k
// is read from device memory (advanced by k_batch_advance after each
// sweep), and with it the buffer roles (level k reads Ma if k is even, Mb if
// odd, and writes the other) and the 1/T row.  A captured sweep therefore
// replays unchanged.  Slot i owns workgroups [tile0_i, tile0_i + nrt * nct);
// tile0 is a multiple of 8, so that a workgroup's position inside its
// member's grid keeps the XCD it would have alone (the gaps exit at once).
struct Bf16BatchMember {
    const unsigned short *J;
    unsigned short *Ma, *Mb;
    const float *table;  // 1/T: row k at table + k * ldt
    const float *hhalf;
    int ldk, R, nrt, kpad, ldt, kmax, lslot;  // lslot: index of the member's level counter
    float gamma;
};

struct Bf16BatchSlot {
    int member, p0, p1, nct, tile0, blend;  // blend: p0 is not a multiple of 8
};

constexpr int kMaxBatch = 16;  // members per batch (descriptors travel as kernel arguments)
struct Bf16BatchArgs {
    const int *level;  // [kMaxBatch] level counters
    int nslot;
    Bf16BatchSlot slot[kMaxBatch];
    Bf16BatchMember mem[kMaxBatch];
};

template <int BM, int BN, int WM, int WN, int PF, int BK>
__global__ __launch_bounds__(64 * WM * WN) void k_dense_phase_bf16_batch(Bf16BatchArgs a)
{
    __shared__ __attribute__((aligned(16))) unsigned char lds[bf16_phase_lds_bytes<BM, BN, BK>()];
    const int g = blockIdx.x;
    int i = 0;
    while (i + 1 < a.nslot && a.slot[i + 1].tile0 <= g)
        ++i;
    const Bf16BatchSlot sl = a.slot[i];
    const Bf16BatchMember &m = a.mem[sl.member];
    const int t = g - sl.tile0;
    if (t >= m.nrt * sl.nct)
        return;
    const int k = a.level[m.lslot];
    if (k >= m.kmax)
        return;  // finished member (its last levels ran in earlier sweeps)
    const unsigned short *cur = (k & 1) ? m.Mb : m.Ma;
    unsigned short *nxt = (k & 1) ? m.Ma : m.Mb;
    const float *invT = m.table + (size_t)k * m.ldt;
    if (sl.blend)
        bf16_phase_tile<BM, BN, WM, WN, PF, BK, true>(m.J, m.ldk, cur, nxt, m.ldk, m.R, sl.p0, sl.p1, m.nrt, sl.nct,
                                                      m.kpad, invT, m.hhalf, m.gamma, nullptr, lds, t);
    else
        bf16_phase_tile<BM, BN, WM, WN, PF, BK, false>(m.J, m.ldk, cur, nxt, m.ldk, m.R, sl.p0, sl.p1, m.nrt, sl.nct,
                                                       m.kpad, invT, m.hhalf, m.gamma, nullptr, lds, t);
}

// The batched solver's whole step as one persistent launch: `sweeps` sweeps
// of every member, each a sequence of phases, the tiles of a phase spread
// over the (co-resident, cooperatively launched) workgroups by a grid stride,
// and a grid barrier after each phase (the next phase reads the
// magnetisations this one wrote).  A member anneals one level per sweep until
// its last, so its level at sweep sw of the step is min(k0 + sw, kmax) from
// the level k0 it starts the step at; the counters are written once, at the
// end.  Per tile the same arithmetic as the one-launch-per-phase kernel above,
// in the same order, so results are identical bit for bit.  The grid is a
// multiple of 8 workgroups, so a tile keeps the XCD it has there.
constexpr int kMaxPersistPhases = 4;  // phase indices per persistent step (descriptors are kernel arguments)
struct Bf16BatchPersistArgs {
    int *level;  // [kMaxBatch] level counters
    int n, nph, sweeps;
    int kmax[kMaxBatch], lslot[kMaxBatch];
    int nslot[kMaxPersistPhases], ntile[kMaxPersistPhases];
    Bf16BatchSlot slot[kMaxPersistPhases][kMaxBatch];
    Bf16BatchMember mem[kMaxBatch];
};

template <int BM, int BN, int WM, int WN, int PF, int BK>
__global__ __launch_bounds__(64 * WM * WN) void k_dense_batch_persistent(Bf16BatchPersistArgs a)
{
    __shared__ __attribute__((aligned(16))) unsigned char lds[bf16_phase_lds_bytes<BM, BN, BK>()];
    cooperative_groups::grid_group grid = cooperative_groups::this_grid();
    for (int sw = 0; sw < a.sweeps; ++sw) {
        for (int ph = 0; ph < a.nph; ++ph) {
            const int ns = a.nslot[ph];
            for (int g = blockIdx.x; g < a.ntile[ph]; g += gridDim.x) {
                int i = 0;
                while (i + 1 < ns && a.slot[ph][i + 1].tile0 <= g)
                    ++i;
                const Bf16BatchSlot sl = a.slot[ph][i];
                const Bf16BatchMember &m = a.mem[sl.member];
                const int t = g - sl.tile0;
                if (t >= m.nrt * sl.nct)
                    continue;
                const int k = min(a.level[m.lslot] + sw, m.kmax);
                if (k >= m.kmax)
                    continue;
                const unsigned short *cur = (k & 1) ? m.Mb : m.Ma;
                unsigned short *nxt = (k & 1) ? m.Ma : m.Mb;
                const float *invT = m.table + (size_t)k * m.ldt;
                if (sl.blend)
                    bf16_phase_tile<BM, BN, WM, WN, PF, BK, true>(m.J, m.ldk, cur, nxt, m.ldk, m.R, sl.p0, sl.p1, m.nrt,
                                                                  sl.nct, m.kpad, invT, m.hhalf, m.gamma, nullptr, lds,
                                                                  t);
                else
                    bf16_phase_tile<BM, BN, WM, WN, PF, BK, false>(m.J, m.ldk, cur, nxt, m.ldk, m.R, sl.p0, sl.p1,
                                                                   m.nrt, sl.nct, m.kpad, invT, m.hhalf, m.gamma,
                                                                   nullptr, lds, t);
            }
            grid.sync();
        }
    }
    // every workgroup's last read of the counters precedes the last barrier
    if (blockIdx.x == 0 && threadIdx.x < a.n) {
        int *lv = a.level + a.lslot[threadIdx.x];
        *lv = min(*lv + a.sweeps, a.kmax[threadIdx.x]);
    }
}

}  // namespace mars
