// Kernels shared by every instance type: starting temperatures, temperature
// level tables, best-of-runs reduction and the spins of the best run.
#include <cfloat>
#include <cmath>

#include "common_device.h"
#include "mars_internal.h"

namespace mars {

__global__ void k_fill_u32(uint32_t *p, uint32_t v, size_t n)
{
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    size_t stride = (size_t)gridDim.x * blockDim.x;
    for (; i < n; i += stride)
        p[i] = v;
}

void launch_fill_u32(uint32_t *p, uint32_t v, size_t n, hipStream_t s)
{
    if (n == 0)
        return;
    size_t blocks = (n + 255) / 256;
    if (blocks > 4096)
        blocks = 4096;
    k_fill_u32<<<(unsigned)blocks, 256, 0, s>>>(p, v, n);
}

// Starting temperature of each run: the caller's value, or a draw from stream 1
// of the counter generator (section MARS: the descent starts from a randomly
// chosen temperature within a given range).
__global__ void k_init_T0(uint64_t seed, int R, double T_lo, double T_hi, const double *T0_in, double *T0_out)
{
    int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= R)
        return;
    T0_out[r] = T0_in ? T0_in[r] : draw_T0(seed, r, T_lo, T_hi);
}

void launch_init_T0(uint64_t seed, int R, double T_lo, double T_hi, const double *T0_in, double *T0_out,
                    hipStream_t s)
{
    k_init_T0<<<(R + 255) / 256, 256, 0, s>>>(seed, R, T_lo, T_hi, T0_in, T0_out);
}

// Inverse temperatures of the levels [first_level, first_level+level_count)
// of every run, level-major: table[k * ldt + r].  Entries past a run's last
// level hold -1 (the run is frozen there).  nlev[r] = levels in range.
__global__ void k_level_table(RunSchedule rs, int R, const double *T0, int kmax, int ldt, float *inv32,
                              double *inv64, int32_t *nlev)
{
    int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= R)
        return;
    LevelWalker w;
    w.start(rs, T0[r]);
    int n = 0;
    while (!w.done && n < kmax) {
        double T = w.T;
        if (inv32)
            inv32[(size_t)n * ldt + r] = (float)(1.0 / T);
        if (inv64)
            inv64[(size_t)n * ldt + r] = 1.0 / T;
        ++n;
        w.next(rs);
    }
    nlev[r] = n;
    for (int k = n; k < kmax; ++k) {
        if (inv32)
            inv32[(size_t)k * ldt + r] = -1.0f;
        if (inv64)
            inv64[(size_t)k * ldt + r] = -1.0;
    }
}

void launch_level_table(const mars_schedule &sc, int R, const double *T0, int kmax, int ldt, float *invT32,
                        double *invT64, int32_t *nlev, hipStream_t s)
{
    k_level_table<<<(R + 255) / 256, 256, 0, s>>>(make_run_schedule(sc), R, T0, kmax, ldt, invT32, invT64, nlev);
}

// Best of runs (section MARS: the best solution of the sample of descents;
// success probability = hits / runs): lowest energy, ties to the lowest run
// index, hit count, mean energy and run statistics.  One block.
constexpr int ARG_NT = 1024;

__global__ __launch_bounds__(ARG_NT) void k_argmin(const double *E, const double *T0, const int64_t *runstat, int R,
                                                   int N, double wsum, mars_result *res, int32_t *best_out,
                                                   double tick_s)
{
    __shared__ double sE[ARG_NT];
    __shared__ int sI[ARG_NT];
    __shared__ double sSum[ARG_NT];
    __shared__ long long sCnt[4][ARG_NT];
    int t = threadIdx.x;
    double be = DBL_MAX;
    int bi = 0x7fffffff;
    double sum = 0.0;
    long long sw = 0, lv = 0, cp = 0;
    for (int r = t; r < R; r += ARG_NT) {
        double e = E[r];
        if (e < be || (e == be && r < bi)) {
            be = e;
            bi = r;
        }
        sum += e;
        sw += runstat[(size_t)r * 4 + 0];
        lv += runstat[(size_t)r * 4 + 1];
        cp += runstat[(size_t)r * 4 + 2];
    }
    sE[t] = be;
    sI[t] = bi;
    sSum[t] = sum;
    sCnt[0][t] = sw;
    sCnt[1][t] = lv;
    sCnt[2][t] = cp;
    __syncthreads();
    for (int s = ARG_NT / 2; s > 0; s >>= 1) {
        if (t < s) {
            double e2 = sE[t + s];
            int i2 = sI[t + s];
            if (e2 < sE[t] || (e2 == sE[t] && i2 < sI[t])) {
                sE[t] = e2;
                sI[t] = i2;
            }
            sSum[t] += sSum[t + s];
            sCnt[0][t] += sCnt[0][t + s];
            sCnt[1][t] += sCnt[1][t + s];
            sCnt[2][t] += sCnt[2][t + s];
        }
        __syncthreads();
    }
    const double best = sE[0];
    long long hits = 0;
    for (int r = t; r < R; r += ARG_NT)
        hits += (E[r] == best) ? 1 : 0;
    sCnt[3][t] = hits;
    __syncthreads();
    for (int s = ARG_NT / 2; s > 0; s >>= 1) {
        if (t < s)
            sCnt[3][t] += sCnt[3][t + s];
        __syncthreads();
    }
    if (t == 0) {
        int bidx = sI[0];
        res->best_energy = best;
        res->best_cut = (wsum - best) * 0.25;
        res->mean_energy = sSum[0] / (double)R;
        res->best_T0 = T0[bidx];
        res->best_run = bidx;
        res->runs = R;
        res->hit_count = sCnt[3][0];
        res->sweeps_executed = sCnt[0][0];
        res->spin_updates = sCnt[0][0] * (long long)N;
        res->levels_executed = sCnt[1][0];
        res->cap_hits = sCnt[2][0];
        const uint64_t t0 = *result_stamp(res);
        res->seconds = (double)((uint64_t)wall_clock64() - t0) * tick_s;
        *best_out = bidx;
    }
}

void launch_argmin(const double *E, const double *T0, const int64_t *runstat, int R, int N, double wsum,
                   mars_result *res_dev, int32_t *best_dev, double tick_s, hipStream_t s)
{
    k_argmin<<<1, ARG_NT, 0, s>>>(E, T0, runstat, R, N, wsum, res_dev, best_dev, tick_s);
}

// the device's constant-rate clock at this point of the stream
__global__ void k_stamp(uint64_t *slot)
{
    if (threadIdx.x == 0)
        *slot = (uint64_t)wall_clock64();
}

void launch_stamp(uint64_t *slot, hipStream_t s) { k_stamp<<<1, 64, 0, s>>>(slot); }

__global__ void k_gather_best(const int8_t *spins, int ld, const int32_t *best, int N, int8_t *out)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < N)
        out[i] = spins[(size_t)(*best) * ld + i];
}

void launch_gather_best(const int8_t *spins, int ld, const int32_t *best_dev, int N, int8_t *out, hipStream_t s)
{
    k_gather_best<<<(N + 255) / 256, 256, 0, s>>>(spins, ld, best_dev, N, out);
}

}  // namespace mars
