// Lattices and sparse graphs: a workgroup anneals a block of `rpw` runs from
// start to finish with their magnetisations resident in LDS.  Runs never
// interact (every descent of the method is independent), so no grid-wide
// synchronisation is needed and the state never touches HBM between the
// initial draw and the final write.  This file chooses the launch shape; the
// kernels are in k_lattice.hip (stencil) and k_sparse.hip (sliced ELL).
#include <algorithm>
#include <cstdlib>

#include "common_device.h"
#include "lds_state.h"
#include "mars_internal.h"

namespace mars {

// A schedule with no temperature level leaves every run at its initial state
// (Algorithm 1 with an empty temperature loop): spins = sign of m0 as stored,
// no sweeps.  Separate from the solver kernels so that their launches are
// all whole anneals.
template <typename S>
__global__ void k_graph_start_only(int N, int R, uint64_t seed, const void *m0, void *m_final, int8_t *spins,
                                   int64_t *runstat)
{
    typedef typename LStore<S>::C C;
    const int run = blockIdx.y;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < N; i += gridDim.x * blockDim.x) {
        const C x = m0 ? (reinterpret_cast<const C *>(m0))[(size_t)i * R + run] : (C)draw_m0(seed, run, i);
        const C xs = LStore<S>::ld(LStore<S>::st(x));
        spins[(size_t)run * N + i] = (xs >= (C)0) ? 1 : -1;
        if (m_final)
            reinterpret_cast<C *>(m_final)[(size_t)i * R + run] = xs;
    }
    if (blockIdx.x == 0 && threadIdx.x < 4)
        runstat[(size_t)run * 4 + threadIdx.x] = 0;
}

static int env_int(const char *name, int dflt)
{
    const char *v = std::getenv(name);
    return (v && *v) ? std::atoi(v) : dflt;
}

static size_t graph_esz(int precision)
{
    return precision == MARS_FP64 ? 8 : precision == MARS_FP32 ? 4 : precision == MARS_FP16 ? 2 : 0;
}

static constexpr size_t kLdsCap = 160 * 1024 - 1024;

// sparse instances run with their state in device memory when one run's state
// does not fit in LDS, or when MARS_GRAPH_GLOBAL=1 (tests of that path at
// sizes the oracle handles)
static bool sparse_global(const Instance &I, const mars_schedule &sc)
{
    const size_t esz = graph_esz(sc.precision);
    const size_t rows = I.kind == KIND_LATTICE ? (size_t)I.N : (size_t)I.nslot + 1;
    const size_t per_run = rows * esz * (sc.update == MARS_JACOBI ? 2 : 1);
    return per_run + 16 + RUN_AREA_MAX > kLdsCap || env_int("MARS_GRAPH_GLOBAL", 0) == 1;
}

bool graph_uses_global(const Instance &I, const mars_schedule &sc)
{
    return graph_esz(sc.precision) != 0 && sparse_global(I, sc);
}

static size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

// layout of the device memory of the sparse solver beyond LDS
struct GlobalLayout {
    size_t m, m2, rs, tscale, rdone, flag, live, total;
    int ldr;
};
static GlobalLayout global_layout(const Instance &I, const mars_schedule &sc, int R)
{
    GlobalLayout L;
    const size_t esz = graph_esz(sc.precision);
    const int vec = esz == 8 ? 1 : 4;
    L.ldr = (R + vec - 1) / vec * vec;
    const size_t state = align256(((size_t)I.nslot + 1) * L.ldr * esz);
    L.m = 0;
    L.m2 = state;
    L.rs = L.m2 + (sc.update == MARS_JACOBI ? state : 0);
    L.tscale = L.rs + align256(sizeof(RunState) * L.ldr);
    L.rdone = L.tscale + align256((esz == 8 ? 8 : 4) * (size_t)L.ldr);
    L.flag = L.rdone + align256(sizeof(int32_t) * L.ldr);
    L.live = L.flag + align256(sizeof(uint32_t) * L.ldr);
    L.total = L.live + 256;
    return L;
}

size_t graph_global_bytes(const Instance &I, const mars_schedule &sc, int R)
{
    if (graph_esz(sc.precision) == 0 || !sparse_global(I, sc))
        return 0;
    return global_layout(I, sc, R).total;
}

// Enqueues the solve's anneal, or, for a sparse solve on the LDS-resident
// solver when `plan` is given, fills *plan for a shared launch and enqueues
// nothing (plan->fn stays null when the solve was enqueued).
static mars_status graph_solve_or_plan(const Instance &I, const GraphSolve &g, hipStream_t s, SparsePlan *plan)
{
    const mars_schedule &sc = *g.sc;
    const bool jac = sc.update == MARS_JACOBI;
    const bool trackd = sc.max_sweeps > 1;
    size_t esz;
    switch (sc.precision) {
    case MARS_FP64: esz = 8; break;
    case MARS_FP32: esz = 4; break;
    case MARS_FP16: esz = 2; break;
    default: return set_error(MARS_E_UNSUPPORTED, "lattice/sparse instances support fp64, fp32 and fp16 storage");
    }
    const bool lat = I.kind == KIND_LATTICE;
    const int N = I.N;
    const size_t rows = lat ? (size_t)N : (size_t)I.nslot + 1;
    const size_t per_run = rows * esz * (jac ? 2 : 1);
    const size_t lds_cap = kLdsCap;
    const bool global = sparse_global(I, sc);
    if (!global && per_run + 16 + RUN_AREA_MAX > lds_cap)
        return set_error(MARS_E_UNSUPPORTED, "the state of one run does not fit in LDS");
    if (global && (!g.gscratch || (lat && !I.lat_sell)))
        return set_error(MARS_E_ARG, "the sparse solver beyond LDS needs its device memory and encodings");
    // runs per workgroup: as many as fit the LDS budget while at least one
    // workgroup per CU (256) remains; more runs per workgroup give each phase
    // more independent (spin, run) items per barrier
    int rpw = 1;
    while (!global && rpw < 64 && (size_t)(2 * rpw) * (per_run + RUN_AREA_MAX) + 16 <= lds_cap &&
           2 * rpw * 256 <= g.R)
        rpw *= 2;
    // MARS_SPARSE_RPW=<power of two> overrides for sparse instances (tuning),
    // within the LDS budget
    if (!lat && !global) {
        const int want_rpw = env_int("MARS_SPARSE_RPW", 0);
        if (want_rpw >= 1 && want_rpw <= 64 && (want_rpw & (want_rpw - 1)) == 0 &&
            (size_t)want_rpw * (per_run + RUN_AREA_MAX) + 16 <= lds_cap)
            rpw = want_rpw;
    }

    GraphArgs a;
    a.N = N;
    a.nphase = I.ncolours;
    a.nslot = I.nslot;
    a.perm = I.perm;
    a.sl_meta = I.sl_meta;
    a.colsell = I.colsell;
    a.long_rows = (!lat && I.nnz >= 16LL * N) ? 1 : 0;
    a.cls = I.cls;
    a.dim = I.dim;
    a.L0 = I.L[0];
    a.L1 = I.L[1];
    a.L2 = I.dim == 3 ? I.L[2] : 1;
    a.bondbits = I.bondbits;
    a.bondsgn = I.bondsgn;
    if (lat) {
        a.hhalf32 = I.has_h ? I.hhalf : nullptr;
        a.hhalf64 = I.has_h ? I.hhalf64 : nullptr;
    } else {
        a.hhalf32 = I.has_h ? I.hperm : nullptr;
        a.hhalf64 = I.has_h ? I.hperm64 : nullptr;
    }
    a.rs = make_run_schedule(sc);
    // geometric schedules: the levels from first to the walker's stop, the
    // length of the block's level table (kept by the launcher if it fits)
    a.ttab = 0;
    if (a.rs.kind == MARS_GEOMETRIC) {
        int stop = a.rs.steps;
        if (a.rs.count >= 0 && a.rs.first + a.rs.count < stop)
            stop = a.rs.first + a.rs.count;
        a.ttab = std::max(0, stop - a.rs.first);
    }
    // one sweep per level on a geometric schedule: every live run anneals
    // exactly one sweep per level of the same level range, so a block's sweep
    // count is known and its per-sweep vote can be left out
    a.fixed_sweeps = (a.rs.kind == MARS_GEOMETRIC && !trackd) ? a.ttab : 0;
    a.max_sweeps = sc.max_sweeps;
    a.d_min = sc.d_min;
    a.damping = sc.damping;
    a.seed = g.seed;
    a.R = g.R;
    a.rpw = rpw;
    a.m0 = g.m0;
    a.T0 = g.T0;
    a.m_final = g.m_final;
    a.spins = g.spins;
    a.runstat = g.runstat;
    a.spl = g.spl;
    a.spl_cap = g.spl ? g.spl_cap : 0;

    hipError_t e;
    const RunSchedule rs = make_run_schedule(sc);
    if (rs.kind == MARS_GEOMETRIC && (rs.first >= rs.steps || rs.count == 0)) {
        dim3 grid((N + 255) / 256, g.R);
        if (esz == 8)
            k_graph_start_only<double><<<grid, 256, 0, s>>>(N, g.R, g.seed, g.m0, g.m_final, g.spins, g.runstat);
        else if (esz == 4)
            k_graph_start_only<float><<<grid, 256, 0, s>>>(N, g.R, g.seed, g.m0, g.m_final, g.spins, g.runstat);
        else
            k_graph_start_only<_Float16><<<grid, 256, 0, s>>>(N, g.R, g.seed, g.m0, g.m_final, g.spins, g.runstat);
        e = hipGetLastError();
        if (e != hipSuccess)
            return hip_error(e, "graph start-only launch");
        return MARS_OK;
    }
    if (global) {
        const GlobalLayout L = global_layout(I, sc, g.R);
        unsigned char *base = static_cast<unsigned char *>(g.gscratch);
        SparseGlobalArgs ga;
        ga.a = a;
        // the field by slot (for a lattice: over its sparse encodings)
        ga.a.hhalf32 = I.has_h ? I.hperm : nullptr;
        ga.a.hhalf64 = I.has_h ? I.hperm64 : nullptr;
        ga.m = base + L.m;
        ga.m2 = base + L.m2;
        ga.ldr = L.ldr;
        {
            // a chunk's state (every row, its runs) within 64 MB, a quarter of
            // the MALL; MARS_SPARSE_CHUNK_RUNS overrides (tuning)
            const int vecg = esz == 8 ? 1 : 4;
            const size_t row_group = ((size_t)I.nslot + 1) * vecg * esz;
            size_t ngc = std::max<size_t>(1, ((size_t)64 << 20) / row_group);
            const int want = env_int("MARS_SPARSE_CHUNK_RUNS", 0);
            if (want > 0)
                ngc = std::max<size_t>(1, (size_t)want / vecg);
            // equal chunks (no nearly empty last chunk)
            const size_t ngr = (size_t)L.ldr / vecg;
            const size_t nchunk = (ngr + std::min(ngc, ngr) - 1) / std::min(ngc, ngr);
            ga.ngc = (int)((ngr + nchunk - 1) / nchunk);
        }
        ga.rs = base + L.rs;
        ga.tscale = base + L.tscale;
        ga.rdone = reinterpret_cast<int32_t *>(base + L.rdone);
        ga.flag = reinterpret_cast<uint32_t *>(base + L.flag);
        ga.live = reinterpret_cast<uint32_t *>(base + L.live);
        ga.jac = jac ? 1 : 0;
        ga.unit = I.unit ? 1 : 0;
        e = launch_sparse_global(ga, (int)esz, s);
        if (e != hipSuccess)
            return hip_error(e, "sparse solve launch (state in device memory)");
        return MARS_OK;
    }
    if (lat) {
        e = launch_lattice_solve(a, (int)esz, rpw, jac, trackd, s);
        if (e != hipSuccess)
            return hip_error(e, "lattice solve launch");
        return MARS_OK;
    }
    // runs per thread (fp32/fp16): four when the block has at least four
    // runs, else two when it has two (each entry group read and decoded once
    // for all of them); MARS_SPARSE_VEC=1|2|4 overrides (tuning)
    int vec = esz > 4 ? 1 : rpw >= 4 ? 4 : rpw >= 2 ? 2 : 1;
    const int want = env_int("MARS_SPARSE_VEC", 0);
    if (esz <= 4 && (want == 1 || want == 2 || want == 4) && want <= rpw)
        vec = want;
    const int nq = rpw / vec;
    // lanes per (slot, run group): a long row is split over two lanes (fp32
    // fields, four runs per group).  On ER N = 800 (48 terms per row, ~40
    // slots per colour class, 32 runs per workgroup) one lane per slot keeps
    // about a third of the workgroup's lanes busy in a phase; two lanes per
    // slot took the solve from 14.1 to 11.7 ms, four (which need two passes
    // over a 40-slot class at 1024 lanes) to 18.5 ms.  MARS_SPARSE_LPS=1|2|4
    // overrides (tuning)
    int lps = (esz <= 4 && vec == 4 && a.long_rows) ? 2 : 1;
    const int want_lps = env_int("MARS_SPARSE_LPS", 0);
    if (esz <= 4 && vec == 4 && (want_lps == 1 || want_lps == 2 || want_lps == 4))
        lps = want_lps;
    // slots in flight per run group: no more than the widest phase has slots
    // (rounded up to whole waves), at most 1024 lanes per workgroup
    int widest = 1;
    if (jac) {
        widest = I.nslot;
    } else {
        for (int c = 0; c < I.ncolours; ++c)
            widest = std::max(widest, I.h_cls[2 * c + 1]);
    }
    // MARS_SPARSE_THREADS=<64..1024, power of two> caps the workgroup (tuning)
    int cap = 1024;
    const int want_thr = env_int("MARS_SPARSE_THREADS", 0);
    if (want_thr >= 64 && want_thr <= 1024 && (want_thr & (want_thr - 1)) == 0)
        cap = want_thr;
    int Tq = std::min(cap / (nq * lps), (widest + 63) / 64 * 64);
    Tq = std::max(Tq, std::max(1, 64 / (nq * lps)));
    if (plan) {
        e = plan_sparse_solve(a, (int)esz, rpw, Tq, vec, lps, jac, trackd, I.unit, plan);
        if (e != hipSuccess)
            return hip_error(e, "sparse solve plan");
        return MARS_OK;
    }
    e = launch_sparse_solve(a, (int)esz, rpw, Tq, vec, lps, jac, trackd, I.unit, s);
    if (e != hipSuccess)
        return hip_error(e, "sparse solve launch");
    return MARS_OK;
}

mars_status launch_graph_solve(const Instance &I, const GraphSolve &g, hipStream_t s)
{
    return graph_solve_or_plan(I, g, s, nullptr);
}

mars_status plan_graph_solve(const Instance &I, const GraphSolve &g, hipStream_t s, SparsePlan *plan)
{
    plan->fn = nullptr;
    return graph_solve_or_plan(I, g, s, plan);
}

}  // namespace mars
