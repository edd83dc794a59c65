// Lattices and sparse graphs: a workgroup anneals a block of `rpw` runs from
// start to finish with their magnetisations resident in LDS.  Runs never
// interact (section MARS: every descent is independent), so no grid-wide
// synchronisation is needed and the state never touches HBM between the
// initial draw and the final write.
//
// LDS layout: m[i * rpw + q] = magnetisation of spin i in the block's run q,
// so the rpw lanes that update spin i for the block's rpw runs read each
// neighbour's values from consecutive addresses.
//
// Phases (colour classes) are independent sets: a lattice sublattice or a
// greedy colour class.  A phase's spins have no couplings among themselves,
// so they are updated in place; the next phase sees the new values, which is
// sequential dynamics in colour order.  The synchronous variant keeps a
// second copy and swaps after each sweep.
#include <algorithm>
#include <cmath>

#include "common_device.h"
#include "mars_internal.h"

namespace mars {

template <typename S>
struct StoreOps;
template <>
struct StoreOps<double> {
    typedef double C;
    __device__ static inline double ld(double v) { return v; }
    __device__ static inline double st(double v) { return v; }
};
template <>
struct StoreOps<float> {
    typedef float C;
    __device__ static inline float ld(float v) { return v; }
    __device__ static inline float st(float v) { return v; }
};
template <>
struct StoreOps<_Float16> {
    typedef float C;
    __device__ static inline float ld(_Float16 v) { return (float)v; }
    __device__ static inline _Float16 st(float v) { return (_Float16)v; }
};

// tanh: the library routine in fp64; in fp32 the identity
// tanh(a) = 1 - 2 / (exp(2a) + 1) on |a| with the hardware exp2 and reciprocal
// (absolute error ~1e-7, far below the fp32 form's 1e-5 bar and the fp16
// storage step), sign restored afterwards so that tanh stays exactly odd.
__device__ inline double mf_tanh(double x) { return tanh(x); }
__device__ inline float mf_tanh(float x)
{
    const float a = fabsf(x);
    const float e = __builtin_amdgcn_exp2f(a * 2.8853900817779268f);  // exp(2a) = 2^(2a / ln 2)
    const float t = 1.0f - 2.0f * __builtin_amdgcn_rcpf(e + 1.0f);
    return copysignf(t, x);
}
// Phi / T: a true division in fp64 (the reference arithmetic), a multiply by
// the rounded inverse in fp32.
__device__ inline double scale_T(double phi, double T, double invT) { return phi / T; }
__device__ inline float scale_T(float phi, double T, float invT) { return phi * invT; }

struct GraphArgs {
    int N;
    // csr
    const int32_t *rowptr;
    const uint32_t *colval;
    const int32_t *phase_ptr;
    const int32_t *phase_vert;
    int nphase;
    // lattice
    int dim, L0, L1, L2;
    const uint8_t *bondbits;
    // field
    const float *hhalf32;
    const double *hhalf64;
    // schedule
    RunSchedule rs;
    int max_sweeps;
    double d_min;
    double damping;
    // runs
    uint64_t seed;
    int R;
    int rpw;
    const void *m0;
    const double *T0;
    void *m_final;
    int8_t *spins;
    int64_t *runstat;
};

template <typename C>
__device__ inline C hhalf_of(const GraphArgs &a, int i);
template <>
__device__ inline double hhalf_of<double>(const GraphArgs &a, int i) { return a.hhalf64 ? a.hhalf64[i] : 0.0; }
template <>
__device__ inline float hhalf_of<float>(const GraphArgs &a, int i) { return a.hhalf32 ? a.hhalf32[i] : 0.0f; }

// IS_LAT: lattice (neighbours from coordinates) or CSR.  JAC: synchronous
// update.  TRACKD: several sweeps per level, ended by d < d_min.
template <bool IS_LAT, typename S, bool JAC, bool TRACKD, bool HAS_H>
__global__ __launch_bounds__(1024) void k_graph_solve(GraphArgs a)
{
    typedef typename StoreOps<S>::C C;
    extern __shared__ unsigned char smem_raw[];
    const int N = a.N;
    const int rpw = a.rpw;
    S *m = reinterpret_cast<S *>(smem_raw);
    S *m2 = JAC ? m + (size_t)N * rpw : m;
    const size_t state_bytes = ((size_t)N * rpw * sizeof(S) * (JAC ? 2 : 1) + 15) & ~(size_t)15;
    uint32_t *dq = reinterpret_cast<uint32_t *>(smem_raw + state_bytes);

    const int q = threadIdx.x % rpw;  // run slot in the block
    const int tq = threadIdx.x / rpw;  // thread index within the run
    const int Tq = blockDim.x / rpw;   // threads per run
    const int run = blockIdx.x * rpw + q;
    const bool live = (tq < Tq) && (run < a.R);

    // initial state (Algorithm 1: s_i := rand(-1, 1))
    for (int i = tq; i < N; i += Tq) {
        C v = 0;
        if (live) {
            if (a.m0)
                v = (C)(reinterpret_cast<const C *>(a.m0))[(size_t)i * a.R + run];
            else
                v = (C)draw_m0(a.seed, run, i);
        }
        m[i * rpw + q] = StoreOps<S>::st(v);
    }
    if (TRACKD && threadIdx.x < rpw)
        dq[threadIdx.x] = 0;

    LevelWalker lw;
    lw.start(a.rs, live ? a.T0[run] : 1.0);
    bool done = !live || lw.done;
    C invT = done ? (C)0 : (C)(1.0 / lw.T);
    double Tcur = done ? 1.0 : lw.T;
    long long n_sweeps = 0, n_levels = 0, n_caps = 0;
    int sw_level = 0;
    const C g = (C)a.damping;
    const bool damp = a.damping != 1.0;

    // lattice iteration constants: item index -> (xh, row) with xh = L0/2 slots
    const int H = IS_LAT ? a.L0 / 2 : 1;
    const int xh = IS_LAT ? tq % H : 0;
    const int row0 = IS_LAT ? tq / H : 0;
    const int drow = IS_LAT ? Tq / H : 0;
    const int nrows = IS_LAT ? a.L1 * a.L2 : 0;
    const int plane = a.L0 * a.L1;

    __syncthreads();
    for (;;) {
        const bool act = !done;
        if (!__syncthreads_or(act))
            break;
        C dloc = 0;
        const int nph = IS_LAT ? 2 : a.nphase;
        for (int c = 0; c < nph; ++c) {
            if (IS_LAT) {
                // colour c = parity of x + y + z; rows (y, z) enumerated with y fastest
                const int dy = drow % a.L1, dz = drow / a.L1;
                int y = row0 % a.L1, z = row0 / a.L1;
                for (int rw = row0; rw < nrows; rw += drow) {
                    const int par = JAC ? 0 : ((c + y + z) & 1);
                    // JAC visits both parities in one phase
                    for (int pp = 0; pp < (JAC ? 2 : 1); ++pp) {
                        const int x = 2 * xh + (JAC ? pp : par);
                        const int v = x + a.L0 * (y + a.L1 * z);
                        const C old = StoreOps<S>::ld(m[v * rpw + q]);
                        C nw = old;
                        if (act) {
                            const int vxp = (x + 1 < a.L0) ? v + 1 : v + 1 - a.L0;
                            const int vxm = (x > 0) ? v - 1 : v - 1 + a.L0;
                            const int vyp = (y + 1 < a.L1) ? v + a.L0 : v + a.L0 - plane;
                            const int vym = (y > 0) ? v - a.L0 : v - a.L0 + plane;
                            const uint8_t b = a.bondbits[v];
                            C phi = 0;
                            C t0 = StoreOps<S>::ld(m[vxp * rpw + q]);
                            C t1 = StoreOps<S>::ld(m[vxm * rpw + q]);
                            C t2 = StoreOps<S>::ld(m[vyp * rpw + q]);
                            C t3 = StoreOps<S>::ld(m[vym * rpw + q]);
                            phi += (b & 1) ? -t0 : t0;
                            phi += (b & 2) ? -t1 : t1;
                            phi += (b & 4) ? -t2 : t2;
                            phi += (b & 8) ? -t3 : t3;
                            if (a.dim == 3) {
                                const int vol = plane * a.L2;
                                const int vzp = (z + 1 < a.L2) ? v + plane : v + plane - vol;
                                const int vzm = (z > 0) ? v - plane : v - plane + vol;
                                C t4 = StoreOps<S>::ld(m[vzp * rpw + q]);
                                C t5 = StoreOps<S>::ld(m[vzm * rpw + q]);
                                phi += (b & 16) ? -t4 : t4;
                                phi += (b & 32) ? -t5 : t5;
                            }
                            if (HAS_H)
                                phi += hhalf_of<C>(a, v);
                            const C th = mf_tanh(scale_T(phi, Tcur, invT));
                            nw = damp ? ((C)1 - g) * old + g * th : th;
                            const C dd = nw > old ? nw - old : old - nw;
                            dloc = dd > dloc ? dd : dloc;
                        }
                        if (JAC)
                            m2[v * rpw + q] = StoreOps<S>::st(nw);
                        else
                            m[v * rpw + q] = StoreOps<S>::st(nw);
                    }
                    y += dy;
                    z += dz;
                    if (y >= a.L1) {
                        y -= a.L1;
                        ++z;
                    }
                }
            } else {
                const int pbeg = JAC ? 0 : a.phase_ptr[c];
                const int pend = JAC ? N : a.phase_ptr[c + 1];
                for (int it = pbeg + tq; it < pend; it += Tq) {
                    const int v = JAC ? it : a.phase_vert[it];
                    const C old = StoreOps<S>::ld(m[v * rpw + q]);
                    C nw = old;
                    if (act) {
                        C phi = 0;
                        const int kb = a.rowptr[v], ke = a.rowptr[v + 1];
                        for (int k = kb; k < ke; ++k) {
                            const uint32_t cv = a.colval[k];
                            const int u = (int)(cv >> 8);
                            const C w = (C)(int8_t)(cv & 0xff);
                            phi += w * StoreOps<S>::ld(m[u * rpw + q]);
                        }
                        if (HAS_H)
                            phi += hhalf_of<C>(a, v);
                        const C th = mf_tanh(scale_T(phi, Tcur, invT));
                        nw = damp ? ((C)1 - g) * old + g * th : th;
                        const C dd = nw > old ? nw - old : old - nw;
                        dloc = dd > dloc ? dd : dloc;
                    }
                    if (JAC)
                        m2[v * rpw + q] = StoreOps<S>::st(nw);
                    else
                        m[v * rpw + q] = StoreOps<S>::st(nw);
                }
            }
            __syncthreads();
            if (JAC)
                break;  // one phase holds every spin
        }
        if (JAC) {
            S *tmp = m;
            m = m2;
            m2 = tmp;
        }
        // level bookkeeping (identical in every thread of a run)
        if (TRACKD) {
            if (act)
                atomicMax(&dq[q], __float_as_uint((float)dloc));
            __syncthreads();
            const float d = __uint_as_float(dq[q]);
            __syncthreads();
            if (tq == 0)
                dq[q] = 0;
            if (act) {
                ++n_sweeps;
                ++sw_level;
                // the fp32 image of d is compared with d_min; d is computed in
                // the storage's arithmetic
                const bool conv = (double)d < a.d_min;
                if (conv || sw_level >= a.max_sweeps) {
                    if (!conv && a.max_sweeps > 1)
                        ++n_caps;
                    ++n_levels;
                    sw_level = 0;
                    lw.next(a.rs);
                    if (lw.done)
                        done = true;
                    else {
                        Tcur = lw.T;
                        invT = (C)(1.0 / lw.T);
                    }
                }
            }
        } else if (act) {
            ++n_sweeps;
            ++n_levels;
            lw.next(a.rs);
            if (lw.done)
                done = true;
            else {
                Tcur = lw.T;
                invT = (C)(1.0 / lw.T);
            }
        }
    }

    // outputs: rounded spins (s = +1 if m >= 0), optional final magnetisation
    if (live) {
        for (int i = tq; i < N; i += Tq) {
            const C v = StoreOps<S>::ld(m[i * rpw + q]);
            a.spins[(size_t)run * N + i] = (v >= (C)0) ? 1 : -1;
            if (a.m_final)
                reinterpret_cast<C *>(a.m_final)[(size_t)i * a.R + run] = v;
        }
        if (tq == 0) {
            a.runstat[(size_t)run * 4 + 0] = n_sweeps;
            a.runstat[(size_t)run * 4 + 1] = n_levels;
            a.runstat[(size_t)run * 4 + 2] = n_caps;
            a.runstat[(size_t)run * 4 + 3] = 0;
        }
    }
}

template <bool IS_LAT, typename S, bool HAS_H>
static void (*pick(bool jac, bool trackd))(GraphArgs)
{
    if (jac)
        return trackd ? k_graph_solve<IS_LAT, S, true, true, HAS_H> : k_graph_solve<IS_LAT, S, true, false, HAS_H>;
    return trackd ? k_graph_solve<IS_LAT, S, false, true, HAS_H> : k_graph_solve<IS_LAT, S, false, false, HAS_H>;
}

template <bool IS_LAT, typename S>
static hipError_t launch_one(const GraphArgs &a, bool jac, bool trackd, dim3 grid, dim3 block, size_t lds,
                             hipStream_t s)
{
    const bool has_h = a.hhalf32 != nullptr;
    void (*fn)(GraphArgs) = has_h ? pick<IS_LAT, S, true>(jac, trackd) : pick<IS_LAT, S, false>(jac, trackd);
    if (lds > 65536) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(fn),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess)
            return e;
    }
    hipLaunchKernelGGL(fn, grid, block, lds, s, a);
    return hipGetLastError();
}

mars_status launch_graph_solve(const Instance &I, const GraphSolve &g, hipStream_t s)
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
    const int N = I.N;
    const size_t per_run = (size_t)N * esz * (jac ? 2 : 1);
    const size_t lds_cap = 160 * 1024 - 1024;
    if (per_run + 64 > lds_cap)
        return set_error(MARS_E_UNSUPPORTED, "the state of one run does not fit in LDS (N too large for this kernel)");
    // runs per workgroup: as many as fit the LDS budget while at least one
    // workgroup per CU (256) remains; more runs per workgroup give each phase
    // more independent (spin, run) items per barrier
    int rpw = 1;
    while (rpw < 64 && (size_t)(2 * rpw) * per_run + 256 <= lds_cap && 2 * rpw * 256 <= g.R)
        rpw *= 2;
    // threads per run: at most 1024 per workgroup and no more than the
    // largest phase has spins (lattice: N/2; sparse: the largest colour class)
    int Tq = 1024 / rpw;
    int widest = N;
    if (!jac) {
        if (I.kind == KIND_LATTICE) {
            widest = (N + 1) / 2;
        } else {
            widest = 1;
            for (size_t c = 0; c + 1 < I.h_phase_ptr.size(); ++c)
                widest = std::max(widest, I.h_phase_ptr[c + 1] - I.h_phase_ptr[c]);
        }
    }
    Tq = std::max(1, std::min(Tq, (widest + 63) / 64 * 64));
    if (I.kind == KIND_LATTICE) {
        const int H = I.L[0] / 2;
        if (Tq < H) {
            while (rpw > 1 && 1024 / rpw < H)
                rpw /= 2;
            Tq = 1024 / rpw;
            if (Tq < H)
                Tq = H;
        }
        Tq = (Tq / H) * H;
    }
    if (Tq < 1)
        Tq = 1;
    const int nthreads = Tq * rpw;
    if (nthreads > 1024)
        return set_error(MARS_E_UNSUPPORTED, "lattice row too long for one workgroup");
    const size_t lds = (((size_t)rpw * per_run + 15) & ~(size_t)15) + 64 * sizeof(uint32_t);

    GraphArgs a;
    a.N = N;
    a.rowptr = I.rowptr;
    a.colval = I.colval;
    a.phase_ptr = I.phase_ptr;
    a.phase_vert = I.phase_vert;
    a.nphase = I.ncolours;
    a.dim = I.dim;
    a.L0 = I.L[0];
    a.L1 = I.L[1];
    a.L2 = I.dim == 3 ? I.L[2] : 1;
    a.bondbits = I.bondbits;
    a.hhalf32 = I.has_h ? I.hhalf : nullptr;
    a.hhalf64 = I.has_h ? I.hhalf64 : nullptr;
    a.rs = make_run_schedule(sc);
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

    dim3 grid((g.R + rpw - 1) / rpw), block(nthreads);
    hipError_t e;
    const bool lat = I.kind == KIND_LATTICE;
    if (esz == 8)
        e = lat ? launch_one<true, double>(a, jac, trackd, grid, block, lds, s)
                : launch_one<false, double>(a, jac, trackd, grid, block, lds, s);
    else if (esz == 4)
        e = lat ? launch_one<true, float>(a, jac, trackd, grid, block, lds, s)
                : launch_one<false, float>(a, jac, trackd, grid, block, lds, s);
    else
        e = lat ? launch_one<true, _Float16>(a, jac, trackd, grid, block, lds, s)
                : launch_one<false, _Float16>(a, jac, trackd, grid, block, lds, s);
    if (e != hipSuccess)
        return hip_error(e, "graph solve launch");
    return MARS_OK;
}

}  // namespace mars
