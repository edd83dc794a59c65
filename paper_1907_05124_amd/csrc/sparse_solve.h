// The sparse (CSR-defined) solver kernel: a workgroup anneals a block of rpw
// runs from start to finish with their magnetisations in LDS,
// m[slot * rpw + q], in the sliced-ELL labelling built at creation (colour
// classes contiguous, each sorted by degree and padded to whole slices of
// SELL_H slots).
//  * A colour class is an independent set (no coupling inside it), so its
//    slots are updated in place; classes run in colour order with a barrier
//    between them (sequential dynamics in colour order).  The synchronous
//    variant writes a second copy and swaps after each sweep.
//  * VEC consecutive runs share each entry read (neighbour slot and weight),
//    and the VEC values of a neighbour arrive in one LDS read.
//  * LPS lanes share one (slot, run group): lane p of the group sums the
//    entry groups p, p + LPS, ...; the partial fields are combined by a
//    reduce-scatter over the group's lanes (DPP moves), after which lane p
//    holds the whole field of runs p, p + LPS, ... and updates those.  With
//    two lanes per slot and at least eight run groups, the two parts of a
//    slot sit eight lanes apart (exchange by a rotation of the 16-lane row),
//    so that eight consecutive lanes read eight consecutive 16-byte pieces of
//    one neighbour's row (measured faster than adjacent pairs on long rows,
//    though the LDS bank-conflict share did not change).  Otherwise the lanes
//    of a group are adjacent within a quad.  Long rows on narrow colour classes (few slots per phase, tens of
//    terms per slot) otherwise leave most lanes idle, each of the busy ones
//    summing a long serial chain; the split shortens the chain and the update
//    (tanh) is still evaluated once per spin-update.
//  * The lanes of a wave cover consecutive slots, so their entry reads
//    (column j of a slice) are consecutive words.
//  * Missing entries of a slice point at the all-zero row nslot, so every
//    lane of a slice runs the same number of terms; slice widths are whole
//    groups of SELL_W entries, read together before their terms are summed.
//  * With +-1 weights the weight is rebuilt as +-1.0f from the entry's sign
//    bit (one bit operation) instead of an integer-to-float conversion.
#pragma once

#include <hip/hip_runtime.h>

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

// value of the lane whose index differs in bit 0 (X = 1) or bit 1 (X = 2),
// within the lane's quad (DPP quad permutation), or in bit 3 (X = 8: a
// rotation of the lane's 16-lane row by eight); both lanes active
template <int X>
__device__ __forceinline__ float lane_xor(float v)
{
    static_assert(X == 1 || X == 2 || X == 8, "DPP exchange distance");
    constexpr int ctrl = X == 1 ? 0xB1 : X == 2 ? 0x4E : 0x128;  // quad_perm [1,0,3,2] / [2,3,0,1] / row_ror:8
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), ctrl, 0xf, 0xf, false));
}

// Reduce-scatter of the VEC partial fields over the LPS lanes of a group:
// afterwards own[k] is the field of run part + LPS * k summed over the group's
// lanes.  Each sum is formed by one lane in a fixed order ((p0 + p1) + (p2 +
// p3) for four lanes), so the result does not depend on scheduling.  far:
// the two lanes of a pair are eight apart instead of adjacent (LPS = 2).
template <int VEC, int LPS>
__device__ __forceinline__ void split_reduce(const float (&phi)[VEC], float (&own)[VEC / LPS], int part, bool far)
{
    if constexpr (LPS == 1) {
#pragma unroll
        for (int e = 0; e < VEC; ++e)
            own[e] = phi[e];
    } else {
        // bit 0 of the lane: keep the runs e with (e & 1) == b, send the rest
        const bool b = (part & 1) != 0;
        float half[VEC / 2];
#pragma unroll
        for (int j = 0; j < VEC / 2; ++j) {
            const float keep = b ? phi[2 * j + 1] : phi[2 * j];
            const float send = b ? phi[2 * j] : phi[2 * j + 1];
            half[j] = keep + (far ? lane_xor<8>(send) : lane_xor<1>(send));  // run 2j + b
        }
        if constexpr (LPS == 2) {
#pragma unroll
            for (int j = 0; j < VEC / 2; ++j)
                own[j] = half[j];
        } else {
            static_assert(LPS == 4 && VEC == 4, "four lanes per slot split four runs");
            // bit 1: keep run b + 2c
            const bool c = (part & 2) != 0;
            const float keep = c ? half[1] : half[0];
            const float send = c ? half[0] : half[1];
            own[0] = keep + lane_xor<2>(send);
        }
    }
}

// The anneal of one block of runs: a = the solve's arguments, 2^lg_rpw runs
// per workgroup, bid = the block's index within the solve.
template <typename S, int VEC, int LPS, bool JAC, bool TRACKD, bool HAS_H, bool UNIT, bool DAMP>
__device__ __forceinline__ void sparse_solve_block(const GraphArgs &a, int lg_rpw, int bid)
{
    typedef typename LStore<S>::C C;
    static_assert(LPS == 1 || (sizeof(C) == 4 && VEC % LPS == 0), "lane split needs fp32 fields and LPS | VEC");
    constexpr int OWN = VEC / LPS;  // runs each lane updates
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
    // initial state and outputs: a thread per (slot, run group)
    const int q0_io = (threadIdx.x % nq) * VEC;
    const int tq_io = threadIdx.x / nq;
    const int Tq_io = blockDim.x / nq;
    const int run0_io = bid * rpw + q0_io;
    // sweeps: LPS lanes per (slot, run group), LPS * nq consecutive lanes
    // per slot; two lanes per slot with at least eight run groups: lane bits
    // [run group mod 8 | part | run group / 8 | slot], else [part | run group
    // | slot]
    const int tid = (int)threadIdx.x;
    const bool far = LPS == 2 && nq >= 8;
    const int part = LPS == 1 ? 0 : far ? (tid >> 3) & 1 : tid % LPS;
    const int q0 = (far ? (tid & 7) | (((tid >> 4) & (nq / 8 - 1)) << 3) : (tid / LPS) % nq) * VEC;
    const int tq = tid / (LPS * nq);
    const int Tq = blockDim.x / (LPS * nq);

    // initial state (Algorithm 1: s_i := rand(-1, 1)); padding slots and the
    // zero row hold 0 in both copies
    for (int i = tq_io; i < rows; i += Tq_io) {
        const int v = i < ns ? a.perm[i] : -1;
        Pack<S, VEC> p;
#pragma unroll
        for (int e = 0; e < VEC; ++e) {
            C x = 0;
            if (v >= 0 && run0_io + e < a.R)
                x = a.m0 ? (C)(reinterpret_cast<const C *>(a.m0))[(size_t)v * a.R + run0_io + e]
                         : (C)draw_m0(a.seed, run0_io + e, v);
            p.v[e] = LStore<S>::st(x);
        }
        lds_put<S, VEC>(&m[((size_t)i << lg_rpw) + q0_io], p);
        if (JAC)
            lds_put<S, VEC>(&m2[((size_t)i << lg_rpw) + q0_io], p);
    }
    for (int q = threadIdx.x; q < rpw; q += blockDim.x) {
        const int r = bid * rpw + q;
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
    unsigned v_first = 0u;
    for (unsigned nvote = 0;; ++nvote) {
        // the level state of the lane's runs (part + LPS k of its group),
        // advanced at the end of the previous sweep
        C scale[OWN];
        bool done[OWN];
        unsigned code = 0;
#pragma unroll
        for (int k = 0; k < OWN; ++k) {
            const RunState &rk = rsl[q0 + part + LPS * k];
            scale[k] = run_tscale<C>(rk);
            done[k] = rk.done != 0;
            code |= done[k] ? 2u : 1u;
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
        C dloc[OWN];
#pragma unroll
        for (int k = 0; k < OWN; ++k)
            dloc[k] = 0;
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
                // the slice record (offset, width) of the group's next slot is
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
                    // slice (SELL_H slots) apart; this lane's are part,
                    // part + LPS, ...
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
                    // a group's neighbour values (one LDS read per entry),
                    // then its terms
                    struct GroupVals {
                        Pack<S, VEC> t[SELL_W];
                        uint32_t ent[SELL_W];
                    };
                    auto fetch = [&](const uint4 cb) {
                        GroupVals gv;
                        gv.ent[0] = cb.x;
                        gv.ent[1] = cb.y;
                        gv.ent[2] = cb.z;
                        gv.ent[3] = cb.w;
#pragma unroll
                        for (int u = 0; u < SELL_W; ++u)
                            gv.t[u] = lds_get<S, VEC>(reinterpret_cast<const S *>(mb + ((gv.ent[u] & colmask) << lgs)));
                        return gv;
                    };
                    auto terms = [&](const GroupVals &gv) {
#pragma unroll
                        for (int u = 0; u < SELL_W; ++u) {
                            const C wt = entry_weight<C, UNIT>(gv.ent[u]);
#pragma unroll
                            for (int e = 0; e < VEC; ++e)
                                phi[e] += wt * LStore<S>::ld(gv.t[u].v[e]);
                        }
                    };
                    auto group = [&](const uint4 cb) { terms(fetch(cb)); };
                    if (!long_rows) {
                        for (int j = part * SELL_W, gi = part; j < w; j += LPS * SELL_W, gi += LPS)
                            group(gp[gi * SELL_H]);
                    } else if (w > 0) {
                        // long rows (high average degree): entry groups are
                        // read ahead of the one being summed; reads run up to
                        // SPARSE_READ_AHEAD of the lane's groups (that many
                        // times LPS groups) past the slice, into the next
                        // slice or the table's padding (in bounds, unused),
                        // and a slice without entries reads nothing
                        static_assert(SPARSE_READ_AHEAD == 2, "the read-ahead below is two groups deep");
                        uint4 cb = gp[part * SELL_H], n1 = gp[(part + LPS) * SELL_H];
                        for (int j = part * SELL_W, gi = part + 2 * LPS; j < w; j += LPS * SELL_W, gi += LPS) {
                            // (an opaque index keeps the read ahead: otherwise
                            // it is turned back into a read of the current
                            // group at its use)
                            const uint4 n2 = gp[opaque((uint32_t)gi * SELL_H)];
                            group(cb);
                            cb = n1;
                            n1 = n2;
                        }
                    }
                    C own[OWN];
                    if constexpr (LPS == 1) {
#pragma unroll
                        for (int e = 0; e < VEC; ++e)
                            own[e] = phi[e];
                    } else {
                        split_reduce<VEC, LPS>(phi, own, part, far);
                    }
                    if (HAS_H) {
                        C hh;
                        if constexpr (sizeof(C) == 8)
                            hh = a.hhalf64[slot];
                        else
                            hh = a.hhalf32[slot];
#pragma unroll
                        for (int k = 0; k < OWN; ++k)
                            own[k] += hh;
                    }
                    const uint32_t o_slot = (uint32_t)slot << lgs;
                    constexpr int TA = sizeof(S) == 4 ? 2 : 1;  // tanh accuracy of the storage
                    if constexpr (LPS == 1) {
                        Pack<S, VEC> nw;
                        if constexpr (FAST) {
                            // every run of the thread still anneals, undamped, no
                            // convergence tracking: the old value is not needed
#pragma unroll
                            for (int e = 0; e < VEC; ++e)
                                nw.v[e] = LStore<S>::st(l_tanh_run<TA>(own[e], scale[e]));
                            lds_put<S, VEC>(reinterpret_cast<S *>(wb + o_slot), nw);
                            continue;
                        }
                        const Pack<S, VEC> old = lds_get<S, VEC>(reinterpret_cast<const S *>(mb + o_slot));
#pragma unroll
                        for (int e = 0; e < VEC; ++e) {
                            const C th = l_tanh_run<TA>(own[e], scale[e]);
                            const C o = LStore<S>::ld(old.v[e]);
                            C n = DAMP ? ((C)1 - g) * o + g * th : th;
                            n = done[e] ? o : n;  // a finished run keeps its state
                            nw.v[e] = done[e] ? old.v[e] : (DAMP ? lds_keep_sign<S>(n) : LStore<S>::st(n));
                            const C dd = n > o ? n - o : o - n;
                            dloc[e] = dd > dloc[e] ? dd : dloc[e];
                        }
                        lds_put<S, VEC>(reinterpret_cast<S *>(wb + o_slot), nw);
                    } else {
                        // each lane writes its own runs' elements of the row
#pragma unroll
                        for (int k = 0; k < OWN; ++k) {
                            const uint32_t o_e = o_slot + (uint32_t)((part + LPS * k) * sizeof(S));
                            const C th = l_tanh_run<TA>(own[k], scale[k]);
                            if constexpr (FAST) {
                                *reinterpret_cast<S *>(wb + o_e) = LStore<S>::st(th);
                            } else {
                                const S os = *reinterpret_cast<const S *>(mb + o_e);
                                const C o = LStore<S>::ld(os);
                                C n = DAMP ? ((C)1 - g) * o + g * th : th;
                                n = done[k] ? o : n;
                                *reinterpret_cast<S *>(wb + o_e) = done[k] ? os : (DAMP ? lds_keep_sign<S>(n) : LStore<S>::st(n));
                                const C dd = n > o ? n - o : o - n;
                                dloc[k] = dd > dloc[k] ? dd : dloc[k];
                            }
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
            for (int k = 0; k < OWN; ++k)
                if (!done[k])
                    atomicMax(&dq[q0 + part + LPS * k], __float_as_uint((float)dloc[k]));
            __syncthreads();
        }
        // each run's level advance (an fp64 exp and divide on geometric
        // schedules) on its own lane of the first wave, side by side
        for (int q = threadIdx.x; q < rpw; q += blockDim.x) {
            rsl[q].end_sweep(a.rs, __uint_as_float(dq[q]), TRACKD, a.max_sweeps, a.d_min,
                             ttab ? tT + (size_t)q * ttab : nullptr, ttab ? tI + (size_t)q * ttab : nullptr,
                             a.spl ? a.spl + (size_t)(bid * rpw + q) * a.spl_cap : nullptr, a.spl_cap);
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
    for (int i = tq_io; i < ns; i += Tq_io) {
        const int v = a.perm[i];
        if (v < 0)
            continue;
        const Pack<S, VEC> p = lds_get<S, VEC>(&m[((size_t)i << lg_rpw) + q0_io]);
#pragma unroll
        for (int e = 0; e < VEC; ++e) {
            if (run0_io + e >= a.R)
                continue;
            const C x = LStore<S>::ld(p.v[e]);
            a.spins[(size_t)(run0_io + e) * N + v] = (x >= (C)0) ? 1 : -1;
            if (a.m_final)
                reinterpret_cast<C *>(a.m_final)[(size_t)v * a.R + run0_io + e] = x;
        }
    }
    if (tq_io == 0)
#pragma unroll
        for (int e = 0; e < VEC; ++e)
            if (run0_io + e < a.R)
                rsl[q0_io + e].write_stats(a.runstat, run0_io + e);
}

// One solve (GROUP false: a_one, lg_one, the block index), or the solves of
// a group (GROUP true: each owns consecutive blocks; a block finds its solve
// in the descriptor).  The two are separate instantiations so that a single
// solve reads its arguments straight from the kernel arguments.
template <typename S, int VEC, int LPS, bool JAC, bool TRACKD, bool HAS_H, bool UNIT, bool DAMP, bool GROUP>
__global__ __launch_bounds__(1024) void k_sparse_solve(GraphArgs a_one, int lg_one, const GraphGroup *grp)
{
    if constexpr (!GROUP) {
        sparse_solve_block<S, VEC, LPS, JAC, TRACKD, HAS_H, UNIT, DAMP>(a_one, lg_one, blockIdx.x);
    } else {
        int k = 0;
        while (k + 1 < grp->count && (int)blockIdx.x >= grp->first[k + 1])
            ++k;
        sparse_solve_block<S, VEC, LPS, JAC, TRACKD, HAS_H, UNIT, DAMP>(grp->args[k], grp->lg[k],
                                                                         (int)blockIdx.x - grp->first[k]);
    }
}

typedef void (*SparseFn)(GraphArgs, int, const GraphGroup *);

template <typename S, int VEC, int LPS, bool HAS_H, bool UNIT, bool DAMP>
static SparseFn sp_pick(bool jac, bool trackd)
{
    if (jac)
        return trackd ? k_sparse_solve<S, VEC, LPS, true, true, HAS_H, UNIT, DAMP, false>
                      : k_sparse_solve<S, VEC, LPS, true, false, HAS_H, UNIT, DAMP, false>;
    return trackd ? k_sparse_solve<S, VEC, LPS, false, true, HAS_H, UNIT, DAMP, false>
                  : k_sparse_solve<S, VEC, LPS, false, false, HAS_H, UNIT, DAMP, false>;
}

template <typename S, int VEC, int LPS, bool DAMP>
static SparseFn sp_pick_hu(bool has_h, bool unit, bool jac, bool trackd)
{
    if (has_h)
        return unit ? sp_pick<S, VEC, LPS, true, true, DAMP>(jac, trackd)
                    : sp_pick<S, VEC, LPS, true, false, DAMP>(jac, trackd);
    return unit ? sp_pick<S, VEC, LPS, false, true, DAMP>(jac, trackd)
                : sp_pick<S, VEC, LPS, false, false, DAMP>(jac, trackd);
}

template <typename S, int VEC, int LPS>
static SparseFn sp_pick_d(bool damp, bool has_h, bool unit, bool jac, bool trackd)
{
    return damp ? sp_pick_hu<S, VEC, LPS, true>(has_h, unit, jac, trackd)
                : sp_pick_hu<S, VEC, LPS, false>(has_h, unit, jac, trackd);
}

// group instantiations: the phased, undamped update (what a serving stream
// runs), with or without the paper's stopping rule, field and +-1 weights;
// null otherwise (such solves launch alone)
template <typename S, int VEC, int LPS>
static SparseFn sp_pick_group(bool damp, bool has_h, bool unit, bool jac, bool trackd)
{
    if (damp || jac)
        return nullptr;
    if (has_h)
        return unit ? (trackd ? k_sparse_solve<S, VEC, LPS, false, true, true, true, false, true>
                              : k_sparse_solve<S, VEC, LPS, false, false, true, true, false, true>)
                    : (trackd ? k_sparse_solve<S, VEC, LPS, false, true, true, false, false, true>
                              : k_sparse_solve<S, VEC, LPS, false, false, true, false, false, true>);
    return unit ? (trackd ? k_sparse_solve<S, VEC, LPS, false, true, false, true, false, true>
                          : k_sparse_solve<S, VEC, LPS, false, false, false, true, false, true>)
                : (trackd ? k_sparse_solve<S, VEC, LPS, false, true, false, false, false, true>
                          : k_sparse_solve<S, VEC, LPS, false, false, false, false, false, true>);
}

// the split kernels (LPS = 2 or 4; fp32 and fp16 storage, four runs per
// lane group), instantiated in their own translation unit; null for other
// combinations (group: the group instantiation, or null)
SparseFn sparse_split_kernel(int esz, int vec, int lps, bool damp, bool has_h, bool unit, bool jac, bool trackd,
                             bool group);

}  // namespace mars
