// Dense couplings: the local fields of one update phase for a block of runs
// are one product  Phi[P, runs] = J[P, :] * M[:, runs]  (Algorithm 1's
// Phi_i = sum_j J_ij s_j for every spin i of the phase and every run), done
// on the matrix cores, with the annealing update fused into the epilogue.
//
// State layout: M is [Np x ldm] fp32, row i = spin i, column r = run r (runs
// contiguous); rows >= N and columns >= R are zero and never written.
// A sweep ping-pongs between two such buffers: the phase with rows [p0, p1)
// reads rows < p0 from `Mnew` (already updated in this sweep) and all other
// rows from `Mold`, and writes its own rows to `Mnew`.  After the last phase
// `Mnew` holds the whole new state.
#include <cmath>

#include "common_device.h"
#include "dense_phase.h"
#include "mars_internal.h"

namespace mars {


// ---------------------------------------------------------------------------
// initial state
// ---------------------------------------------------------------------------

__global__ void k_dense_init_state(uint64_t seed, int N, int R, int ldm, const float *m0, float *M)
{
    int r = blockIdx.x * blockDim.x + threadIdx.x;
    int i = blockIdx.y;
    if (r >= R)
        return;
    M[(size_t)i * ldm + r] = m0 ? m0[(size_t)i * R + r] : draw_m0(seed, r, i);
}

void launch_dense_init_state(uint64_t seed, int N, int R, int ldm, const float *m0, float *M, hipStream_t s)
{
    dim3 grid((R + 255) / 256, N);
    k_dense_init_state<<<grid, 256, 0, s>>>(seed, N, R, ldm, m0, M);
}

// ---------------------------------------------------------------------------
// one update phase: fp32 matrix-core product + fused tanh update
// ---------------------------------------------------------------------------
//
// 16 waves (4 x 4) per 128 x 128 tile, each wave one 32 x 32 MFMA block, slab
// loads issued two slabs ahead (the shape measured fastest for this problem:
// four waves per SIMD keep the matrix pipe fed across LDS reads and barriers).
constexpr int DWM = 4, DWN = 4, DPF = 2;

void launch_dense_phase_f32(const Instance &I, const float *Mold, float *Mnew, int ldm, int R, int p0, int p1,
                            const float *invT, const double *invT64, float gamma, uint32_t *dmax, hipStream_t s)
{
    const int a0 = p0 & ~3;
    const int nrt = (p1 - a0 + DBM - 1) / DBM;
    const int nct = ldm / DBN;
    const int kpad = (I.N + DBK - 1) / DBK * DBK;
    k_dense_phase_f32<DWM, DWN, DPF, false><<<nrt * nct, 64 * DWM * DWN, 0, s>>>(
        I.J, I.Np, Mold, Mnew, ldm, R, p0, p1, a0, nrt, nct, kpad, invT, invT64, I.has_h ? I.hhalf : nullptr, gamma,
        dmax, nullptr);
}

// ---------------------------------------------------------------------------
// sequential update (every spin its own phase, in index order)
// ---------------------------------------------------------------------------

// One block of SEQ_NB consecutive spins [p0, p1): phi holds their fields from
// the state at the start of the block (J M + h/2, old values for the block's
// own spins).  Each thread updates one run's spins in index order and adds
// the change of each updated spin to the fields of the later ones,
// J_ki (m_i^new - m_i^old), so every spin sees its predecessors' new values:
// the sequential dynamics that the paper's GPU description assigns spin by
// spin.  The block's couplings are staged in LDS (read as broadcasts).
__global__ __launch_bounds__(64) void k_dense_seq_block(const float *__restrict__ J, int ldj,
                                                        const float *__restrict__ phi, const float *__restrict__ Mold,
                                                        float *__restrict__ Mnew, int ldm, int R, int p0, int p1,
                                                        const float *__restrict__ invT, float gamma,
                                                        uint32_t *__restrict__ dmax)
{
    __shared__ float Jb[SEQ_NB][SEQ_NB + 1];
    const int n = p1 - p0;
    for (int e = threadIdx.x; e < SEQ_NB * SEQ_NB; e += blockDim.x) {
        const int k = e / SEQ_NB, i = e % SEQ_NB;
        Jb[k][i] = (k < n && i < n) ? J[(size_t)(p0 + k) * ldj + p0 + i] : 0.0f;
    }
    __syncthreads();
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= R)
        return;
    const float it = invT[r];  // < 0: frozen run
    const bool damp = gamma != 1.0f;
    float c[SEQ_NB];
#pragma unroll
    for (int k = 0; k < SEQ_NB; ++k)
        c[k] = 0.0f;
    float dl = 0.0f;
#pragma unroll
    for (int i = 0; i < SEQ_NB; ++i) {
        if (i < n) {
            const size_t at = (size_t)(p0 + i) * ldm + r;
            const float old = Mold[at];
            float nw = old;
            if (it >= 0.0f) {
                const float th = tanhf((phi[at] + c[i]) * it);
                nw = damp ? (1.0f - gamma) * old + gamma * th : th;
            }
            Mnew[at] = nw;
            const float d = nw - old;
            dl = fmaxf(dl, fabsf(d));
#pragma unroll
            for (int k = i + 1; k < SEQ_NB; ++k)
                c[k] += Jb[k][i] * d;
        }
    }
    if (dmax)
        atomicMax(&dmax[r], __float_as_uint(dl));
}

void launch_dense_seq_block(const Instance &I, const float *Mold, float *Mnew, float *phi, int ldm, int R, int p0,
                            int p1, const float *invT, float gamma, uint32_t *dmax, hipStream_t s)
{
    const int a0 = p0 & ~3;
    const int nrt = (p1 - a0 + DBM - 1) / DBM;
    const int nct = ldm / DBN;
    const int kpad = (I.N + DBK - 1) / DBK * DBK;
    k_dense_phase_f32<DWM, DWN, DPF, true><<<nrt * nct, 64 * DWM * DWN, 0, s>>>(
        I.J, I.Np, Mold, Mnew, ldm, R, p0, p1, a0, nrt, nct, kpad, invT, nullptr, I.has_h ? I.hhalf : nullptr, gamma,
        dmax, phi);
    k_dense_seq_block<<<(R + 63) / 64, 64, 0, s>>>(I.J, I.Np, phi, Mold, Mnew, ldm, R, p0, p1, invT, gamma, dmax);
}

// ---------------------------------------------------------------------------
// rounding, output copies, run statistics
// ---------------------------------------------------------------------------

// s_i = +1 if m_i >= 0 else -1 (Algorithm 1's continuous spins rounded), written
// to the zero-padded run-major operand of the energy product [ldr x Ke] and,
// when requested, to the caller's [R x N] spins and [N x R] magnetisations.
// A 64 x 64 tile goes through LDS so that both the spin-major reads and the
// run-major writes are coalesced.
__global__ __launch_bounds__(256) void k_dense_round(const float *M, int ldm, int N, int R, int Ke, int ldr,
                                                     int8_t *spad, int8_t *spins, float *m_final)
{
    __shared__ int8_t t[64][65];
    const int i0 = blockIdx.y * 64, r0 = blockIdx.x * 64;
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;  // 64 x 4
    for (int y = ty; y < 64; y += 4) {
        const int i = i0 + y, r = r0 + tx;
        int8_t v = 0;
        if (i < N && r < R) {
            const float m = M[(size_t)i * ldm + r];
            v = (m >= 0.0f) ? 1 : -1;
            if (m_final)
                m_final[(size_t)i * R + r] = m;
        }
        t[y][tx] = v;
    }
    __syncthreads();
    for (int y = ty; y < 64; y += 4) {
        const int r = r0 + y, i = i0 + tx;
        if (r < ldr && i < Ke) {
            const int8_t v = t[tx][y];
            spad[(size_t)r * Ke + i] = v;
            if (spins && r < R && i < N)
                spins[(size_t)r * N + i] = v;
        }
    }
}

void launch_dense_round(const float *M, int ldm, int N, int R, int Ke, int8_t *spad, int8_t *spins, float *m_final,
                        hipStream_t s)
{
    const int ldr = (R + 127) / 128 * 128;
    dim3 grid((ldr + 63) / 64, (Ke + 63) / 64);
    k_dense_round<<<grid, 256, 0, s>>>(M, ldm, N, R, Ke, ldr, spad, spins, m_final);
}

// one sweep per level: sweeps = levels = nlev, no cap hits
__global__ void k_dense_runstat(int R, const int32_t *nlev, int64_t *runstat)
{
    int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= R)
        return;
    runstat[(size_t)r * 4 + 0] = nlev[r];
    runstat[(size_t)r * 4 + 1] = nlev[r];
    runstat[(size_t)r * 4 + 2] = 0;
    runstat[(size_t)r * 4 + 3] = 0;
}

void launch_dense_runstat(int R, const int32_t *nlev, int64_t *runstat, hipStream_t s)
{
    k_dense_runstat<<<(R + 255) / 256, 256, 0, s>>>(R, nlev, runstat);
}

// ---------------------------------------------------------------------------
// several sweeps per level (Algorithm 1's repeat-until): per-run level state
// ---------------------------------------------------------------------------
//
// state[2r] = level index, state[2r+1] = sweeps done at this level (or -1
// once the run has finished its levels).  invT_cur[r] is the inverse
// temperature of the run's current level, -1 for a finished run (its
// magnetisations are then left unchanged by the phase kernel).

__global__ void k_dense_advance_init(int R, const float *table, const double *table64, const int32_t *nlev,
                                     float *invT_cur, double *invT64_cur, int32_t *state, int64_t *runstat,
                                     uint32_t *dmax)
{
    int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= R)
        return;
    const bool any = nlev[r] > 0;
    invT_cur[r] = any ? table[r] : -1.0f;
    if (table64)
        invT64_cur[r] = any ? table64[r] : -1.0;
    state[2 * r] = 0;
    state[2 * r + 1] = any ? 0 : -1;
    runstat[(size_t)r * 4 + 0] = 0;
    runstat[(size_t)r * 4 + 1] = 0;
    runstat[(size_t)r * 4 + 2] = 0;
    runstat[(size_t)r * 4 + 3] = 0;
    dmax[r] = 0u;
}

void launch_dense_advance_init(int R, const float *table, const double *table64, const int32_t *nlev,
                               float *invT_cur, double *invT64_cur, int32_t *state, int64_t *runstat, uint32_t *dmax,
                               hipStream_t s)
{
    k_dense_advance_init<<<(R + 255) / 256, 256, 0, s>>>(R, table, table64, nlev, invT_cur, invT64_cur, state,
                                                          runstat, dmax);
}

// After a sweep: every run's level state (dense_advance_one); active counts
// the runs still annealing.
__global__ void k_dense_advance(int R, const float *table, const double *table64, int ldt, const int32_t *nlev,
                                int max_sweeps, double d_min, float *invT_cur, double *invT64_cur, int32_t *state,
                                int64_t *runstat, uint32_t *dmax, uint32_t *active, int32_t *spl, int cap)
{
    int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= R)
        return;
    if (dense_advance_one(r, table, table64, ldt, nlev, max_sweeps, d_min, invT_cur, invT64_cur, state, runstat, dmax,
                          spl, cap))
        atomicAdd(active, 1u);
}

void launch_dense_advance(int R, const float *table, const double *table64, int ldt, const int32_t *nlev,
                          int max_sweeps, double d_min, float *invT_cur, double *invT64_cur, int32_t *state,
                          int64_t *runstat, uint32_t *dmax, uint32_t *active, int32_t *spl, int cap, hipStream_t s)
{
    k_dense_advance<<<(R + 255) / 256, 256, 0, s>>>(R, table, table64, ldt, nlev, max_sweeps, d_min, invT_cur,
                                                     invT64_cur, state, runstat, dmax, active, spl, cap);
}

// One sweep per level: every visited level of run r ran one sweep.
__global__ void k_dense_spl_ones(int R, const int32_t *nlev, int32_t *spl, int cap)
{
    const int r = blockIdx.y;
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (r < R && k < cap)
        spl[(size_t)r * cap + k] = k < nlev[r] ? 1 : 0;
}

void launch_dense_spl_ones(int R, const int32_t *nlev, int32_t *spl, int cap, hipStream_t s)
{
    dim3 grid((cap + 255) / 256, R);
    k_dense_spl_ones<<<grid, 256, 0, s>>>(R, nlev, spl, cap);
}

// ---------------------------------------------------------------------------
// exact energies (eq. (2)) of run-major spins
// ---------------------------------------------------------------------------
//
// Every coupling and field value is an integer multiple of 2^emin; the dense
// energy uses Jfix = J * 2^-emin, split into int8 digits whose products with
// the spins run on the int8 matrix cores (k_energy.hip).

__global__ void k_dense_fixpoint(const float *J, int ldj, int N, int emin, int64_t *Jfix)
{
    size_t n = (size_t)N * N;
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (size_t)gridDim.x * blockDim.x) {
        size_t i = e / N, j = e % N;
        float v = (i == j) ? 0.0f : J[i * ldj + j];
        Jfix[e] = (int64_t)ldexp((double)v, -emin);
    }
}

void launch_dense_fixpoint(const Instance &I, hipStream_t s)
{
    k_dense_fixpoint<<<2048, 256, 0, s>>>(I.J, I.Np, I.N, I.emin, I.Jfix);
}

// ---------------------------------------------------------------------------
// exact energies for the sparse and lattice instances
// ---------------------------------------------------------------------------

constexpr int GENT = 256;

__global__ __launch_bounds__(GENT) void k_graph_energy(int kind, int N, const int32_t *__restrict__ rowptr,
                                                       const uint32_t *__restrict__ colval, int dim, int L0,
                                                       int L1, int L2, const uint8_t *__restrict__ bondbits,
                                                       const int64_t *__restrict__ hfix, int emin,
                                                       const int8_t *__restrict__ spins, double *E)
{
    __shared__ long long red[GENT];
    const int r = blockIdx.x;
    const int8_t *s = spins + (size_t)r * N;
    long long acc = 0;
    const int shift = -emin;  // couplings are integers, emin <= 0
    for (int i = threadIdx.x; i < N; i += GENT) {
        long long phi = 0;
        if (kind == KIND_CSR) {
            for (int k = rowptr[i]; k < rowptr[i + 1]; ++k) {
                uint32_t cv = colval[k];
                int u = (int)(cv >> 8);
                int v = (int)(int8_t)(cv & 0xff);
                phi += (s[u] > 0) ? v : -v;
            }
        } else {
            int x = i % L0, y = (i / L0) % L1, z = i / (L0 * L1);
            uint8_t b = bondbits[i];
            int nb[6];
            nb[0] = i - x + (x + 1) % L0;
            nb[1] = i - x + (x + L0 - 1) % L0;
            nb[2] = i + ((y + 1) % L1 - y) * L0;
            nb[3] = i + ((y + L1 - 1) % L1 - y) * L0;
            nb[4] = i + ((z + 1) % L2 - z) * L0 * L1;
            nb[5] = i + ((z + L2 - 1) % L2 - z) * L0 * L1;
            for (int q = 0; q < 2 * dim; ++q) {
                int v = (b >> q & 1) ? -1 : 1;
                phi += (s[nb[q]] > 0) ? v : -v;
            }
        }
        long long f = phi << shift;
        if (hfix)
            f += hfix[i];
        acc += (s[i] > 0) ? f : -f;
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int w = GENT / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w)
            red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0)
        E[r] = i128_to_double_scaled(-(__int128)red[0], emin);
}

void launch_graph_energy(const Instance &I, const int8_t *spins, int R, double *E, hipStream_t s)
{
    k_graph_energy<<<R, GENT, 0, s>>>(I.kind, I.N, I.rowptr, I.colval, I.dim, I.L[0], I.L[1], I.L[2], I.bondbits,
                                      I.has_h ? I.hfix : nullptr, I.emin, spins, E);
}

}  // namespace mars
