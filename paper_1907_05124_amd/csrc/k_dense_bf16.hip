// BF16 form of the dense path: conversion of J, state initialisation in the
// run-major bf16 layout, the phase launcher, and rounding into the padded
// spin operand shared with the fp32 form (exact energies are unchanged).
#include "common_device.h"
#include "dense_phase_bf16.h"
#include "mars_internal.h"

namespace mars {

// Tile shape measured fastest on the SK N=2000 x 4096-run phase shape.
constexpr int HBM_ = 128, HBN_ = 128, HWM = 4, HWN = 4, HPF = 1;

__global__ void k_bf16_from_f32(const float *J, size_t n, unsigned short *Jb)
{
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (size_t)gridDim.x * blockDim.x)
        Jb[e] = float_to_bf16(J[e]);
}

mars_status ensure_bf16_couplings(Instance &I, hipStream_t s)
{
    if (I.Jbf)
        return MARS_OK;
    const size_t n = (size_t)I.Np * I.Np;
    hipError_t e = hipMalloc(&I.Jbf, n * sizeof(unsigned short));
    if (e != hipSuccess) {
        I.Jbf = nullptr;
        return hip_error(e, "hipMalloc bf16 couplings");
    }
    k_bf16_from_f32<<<2048, 256, 0, s>>>(I.J, n, I.Jbf);
    e = hipGetLastError();
    if (e != hipSuccess)
        return hip_error(e, "bf16 conversion");
    return MARS_OK;
}

int bf16_state_rows(int R) { return (R + 255) / 256 * 256; }

// M^T[r][i] = bf16(m0[i][r]) or the generator's draw (Algorithm 1's random start)
__global__ void k_bf16_init_state(uint64_t seed, int N, int R, int ldk, const float *m0, unsigned short *MT)
{
    const int r = blockIdx.y;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < N; i += gridDim.x * blockDim.x) {
        const float v = m0 ? m0[(size_t)i * R + r] : draw_m0(seed, r, i);
        MT[(size_t)r * ldk + i] = float_to_bf16(v);
    }
}

void launch_bf16_init_state(uint64_t seed, int N, int R, int ldk, const float *m0, unsigned short *MT, hipStream_t s)
{
    dim3 grid((N + 255) / 256, R);
    k_bf16_init_state<<<grid, 256, 0, s>>>(seed, N, R, ldk, m0, MT);
}

void launch_dense_phase_bf16(const Instance &I, const unsigned short *Mold, unsigned short *Mnew, int ldk, int R,
                             int p0, int p1, const float *invT, float gamma, uint32_t *dmax, hipStream_t s)
{
    const int nrt = (R + HBM_ - 1) / HBM_;
    const int nct = (p1 - p0 + HBN_ - 1) / HBN_;
    const int kpad = (I.N + HBK - 1) / HBK * HBK;
    k_dense_phase_bf16<HBM_, HBN_, HWM, HWN, HPF><<<nrt * nct, 64 * HWM * HWN, 0, s>>>(
        I.Jbf, I.Np, Mold, Mnew, ldk, R, p0, p1, nrt, nct, kpad, invT, I.has_h ? I.hhalf : nullptr, gamma, dmax);
}

// s = +1 if m >= 0 else -1 into the padded operand [ldr x Ke]; optional
// caller spins [R x N] and fp32 magnetisations [N x R]
__global__ void k_bf16_round(const unsigned short *MT, int ldk, int N, int R, int Ke, int ldr, int8_t *spad,
                             int8_t *spins, float *m_final)
{
    const int r = blockIdx.y;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < Ke; i += gridDim.x * blockDim.x) {
        int8_t v = 0;
        if (r < R && i < N) {
            const float m = bf16_to_float(MT[(size_t)r * ldk + i]);
            v = (m >= 0.0f) ? 1 : -1;
            if (spins)
                spins[(size_t)r * N + i] = v;
            if (m_final)
                m_final[(size_t)i * R + r] = m;
        }
        if (r < ldr)
            spad[(size_t)r * Ke + i] = v;
    }
}

void launch_bf16_round(const unsigned short *MT, int ldk, int N, int R, int Ke, int8_t *spad, int8_t *spins,
                       float *m_final, hipStream_t s)
{
    const int ldr = (R + 127) / 128 * 128;
    dim3 grid((Ke + 255) / 256, ldr);
    k_bf16_round<<<grid, 256, 0, s>>>(MT, ldk, N, R, Ke, ldr, spad, spins, m_final);
}

}  // namespace mars
