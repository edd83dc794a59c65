// The paper's scheduler on dense instances (Algorithm 1's repeat ... until:
// sweeps at one temperature until the largest change d falls below d_min,
// per run) as ONE cooperative launch: every workgroup takes phase tiles,
// then the runs' level states advance on the device, and a grid barrier
// separates the steps, so the whole anneal is enqueued at once and the host
// never waits for it.  Runs leave at different sweeps; a 128-run block whose
// runs have all finished, and whose values both state buffers already hold,
// is left out of the products from then on.
#include <hip/hip_cooperative_groups.h>

#include "common_device.h"
#include "dense_phase.h"
#include "dense_phase_bf16.h"
#include "mars_internal.h"

namespace mars {

namespace cg = cooperative_groups;

// bf16 tile of the launch: 128 runs x 128 spins, 16 waves, 128-deep slabs
// (the tuner's default; every variant gives the same bits)
constexpr int PB_BM = 128, PB_BN = 128, PB_WM = 4, PB_WN = 4, PB_PF = 2, PB_BK = 128;

// The sweep loop shared by both forms: phase(b, p0, p1, reads_b) runs one
// phase's tiles of this workgroup (reads_b: the state to read is buffer B),
// copy_b_to_a() moves the final state into buffer A.
template <typename Phase, typename Copy>
__device__ void paper_loop(const DensePaperArgs &a, Phase phase, Copy copy_b_to_a)
{
    cg::grid_group grid = cg::this_grid();
    const int gtid = blockIdx.x * blockDim.x + threadIdx.x;
    const int gsz = gridDim.x * blockDim.x;
    const long long cap = (long long)a.kmax * a.max_sweeps + 1;
    bool in_b = false;  // the current state is in buffer A (false) or B
    for (long long sw = 0; sw < cap; ++sw) {
        for (int b = 0; b < a.B; ++b) {
            const int p0 = a.pb[b], p1 = a.pb[b + 1];
            if (p1 <= p0)
                continue;
            phase(p0, p1, in_b);
            grid.sync();
        }
        in_b = !in_b;
        // level state of every run; active runs counted per 128-run block
        const int par = (int)(sw & 1);
        for (int r = gtid; r < a.R; r += gsz)
            if (dense_advance_one(r, a.table, a.table64, a.ldt, a.nlev, a.max_sweeps, a.d_min, a.invT_cur,
                                  a.invT64_cur, a.state, a.runstat, a.dmax, a.spl, a.spl_cap)) {
                atomicAdd(&a.active[par], 1u);
                atomicAdd(&a.cnt[par * a.ntr + (r >> 7)], 1);
            }
        grid.sync();
        const unsigned act = __hip_atomic_load(&a.active[par], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        // a block is left out once it has had no active run at two advances in
        // a row: the sweep after its last run finished copied every value of
        // the block into the other buffer too.  The other parity's counters
        // were last read before this sweep's first barrier and are next
        // written after the next one.
        for (int q = gtid; q < a.ntr; q += gsz) {
            const int f = a.cnt[par * a.ntr + q] == 0 ? a.frozen[q] + 1 : 0;
            a.frozen[q] = f;
            a.skip[q] = f >= 2 ? 1 : 0;
            a.cnt[(par ^ 1) * a.ntr + q] = 0;
        }
        if (gtid == 0)
            a.active[par ^ 1] = 0u;
        grid.sync();
        if (act == 0u)
            break;
    }
    if (in_b)
        copy_b_to_a(gtid, gsz);
}

__global__ __launch_bounds__(1024) void k_dense_paper_f32(DensePaperArgs a)
{
    const int kpad = (a.N + DBK - 1) / DBK * DBK;
    auto phase = [&](int p0, int p1, bool in_b) {
        const float *cur = in_b ? a.Mb : a.Ma;
        float *nxt = in_b ? a.Ma : a.Mb;
        const int a0 = p0 & ~3;
        const int nrt = (p1 - a0 + DBM - 1) / DBM;
        const int nct = a.ldm / DBN;
        for (int t = blockIdx.x; t < nrt * nct; t += gridDim.x) {
            dense_phase_f32_tile<4, 4, 2, false>(a.J, a.ldj, cur, nxt, a.ldm, a.R, p0, p1, a0, nrt, nct, kpad,
                                                 a.invT_cur, a.invT64_cur, a.hhalf, a.gamma, a.dmax, nullptr, t,
                                                 a.skip);
            __syncthreads();
        }
    };
    auto copy = [&](int gtid, int gsz) {
        const size_t n = (size_t)a.Np * a.ldm;
        for (size_t e = gtid; e < n; e += gsz)
            a.Ma[e] = a.Mb[e];
    };
    paper_loop(a, phase, copy);
}

__global__ __launch_bounds__(1024) void k_dense_paper_bf16(DensePaperArgs a)
{
    __shared__ __attribute__((aligned(16))) unsigned char lds[bf16_phase_lds_bytes<PB_BM, PB_BN, PB_BK>()];
    const int kpad = (a.N + PB_BK - 1) / PB_BK * PB_BK;
    auto phase = [&](int p0, int p1, bool in_b) {
        const unsigned short *cur = in_b ? a.Bb : a.Ba;
        unsigned short *nxt = in_b ? a.Ba : a.Bb;
        const int nrt = (a.R + PB_BM - 1) / PB_BM;
        const int nct = (p1 - p0 + PB_BN - 1) / PB_BN;
        for (int t = blockIdx.x; t < nrt * nct; t += gridDim.x) {
            if (p0 % 8 == 0)
                bf16_phase_tile<PB_BM, PB_BN, PB_WM, PB_WN, PB_PF, PB_BK, false>(
                    a.Jb, a.Np, cur, nxt, a.Np, a.R, p0, p1, nrt, nct, kpad, a.invT_cur, a.hhalf, a.gamma, a.dmax,
                    lds, t, a.skip);
            else
                bf16_phase_tile<PB_BM, PB_BN, PB_WM, PB_WN, PB_PF, PB_BK, true>(
                    a.Jb, a.Np, cur, nxt, a.Np, a.R, p0, p1, nrt, nct, kpad, a.invT_cur, a.hhalf, a.gamma, a.dmax,
                    lds, t, a.skip);
            __syncthreads();
        }
    };
    auto copy = [&](int gtid, int gsz) {
        const size_t n = (size_t)a.ldr * a.Np;
        for (size_t e = gtid; e < n; e += gsz)
            a.Ba[e] = a.Bb[e];
    };
    paper_loop(a, phase, copy);
}

hipError_t launch_dense_paper(const DensePaperArgs &args, bool bf16, hipStream_t s)
{
    const void *fn = bf16 ? reinterpret_cast<const void *>(&k_dense_paper_bf16)
                          : reinterpret_cast<const void *>(&k_dense_paper_f32);
    int dev = 0, per_cu = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess)
        return e;
    hipDeviceProp_t prop;
    if ((e = hipGetDeviceProperties(&prop, dev)) != hipSuccess)
        return e;
    if ((e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, 1024, 0)) != hipSuccess)
        return e;
    if (per_cu < 1)
        return hipErrorInvalidConfiguration;
    // as many workgroups as the largest phase has tiles, within what is resident at once
    int tiles = 1;
    for (int b = 0; b < args.B; ++b) {
        const int p0 = args.pb[b], p1 = args.pb[b + 1];
        if (p1 <= p0)
            continue;
        const int t = bf16 ? ((args.R + PB_BM - 1) / PB_BM) * ((p1 - p0 + PB_BN - 1) / PB_BN)
                           : ((p1 - (p0 & ~3) + DBM - 1) / DBM) * (args.ldm / DBN);
        tiles = std::max(tiles, t);
    }
    const int grid = std::min(tiles, per_cu * prop.multiProcessorCount);
    DensePaperArgs a = args;
    void *kargs[] = {&a};
    return hipLaunchCooperativeKernel(fn, dim3(grid), dim3(1024), kargs, 0, s);
}

}  // namespace mars
