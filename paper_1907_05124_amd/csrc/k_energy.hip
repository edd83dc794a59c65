// Exact energies of dense instances on the int8 matrix cores.
//
// eq. (2): E = -sum_i s_i (sum_j J_ij s_j + h_i).  Every coupling and field
// value is an integer multiple of 2^emin, Jfix = J * 2^-emin.  Jfix is split
// into balanced base-256 digits, Jfix = sum_l 256^l D_l with D_l in
// [-128, 127]; each digit matrix times the +-1 spins is an exact int8 x int8
// product with int32 accumulation (|sum| <= 128 N < 2^31).  Then
//     E_r = -2^emin * sum_l 256^l * sum_i s_ir (D_l S)_ir  -  2^emin sum_i s_ir hfix_i,
// summed exactly in 64/128-bit integers and rounded once to double.
//
// Operands (both K-contiguous): A = D_l rows [Me x Ke] int8, B^T = spins
// [ldr x Ke] int8 (run-major, zero padded: a zero spin contributes nothing).
// Workgroup tile 128 spins x 128 runs, 4 waves of 64 x 64 (2 x 2 blocks of
// the 32x32x32 int8 MFMA), K in 128-byte slabs through double-buffered LDS.
#include "common_device.h"
#include "mars_internal.h"

namespace mars {

typedef int intx4 __attribute__((ext_vector_type(4)));
typedef int intx16 __attribute__((ext_vector_type(16)));

constexpr int EBM = 128, EBN = 128, EBK = 128, ENT = 256;
constexpr int ELDS = EBK + 16;  // padded LDS row (bytes)

// digits of the fixed-point couplings, written once at create time
__global__ void k_dense_limbs(const int64_t *Jfix, int N, int nlimb, int Me, int Ke, int8_t *D)
{
    size_t n = (size_t)Me * Ke;
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (size_t)gridDim.x * blockDim.x) {
        const size_t i = e / Ke, j = e % Ke;
        int64_t v = (i < (size_t)N && j < (size_t)N) ? Jfix[i * N + j] : 0;
        for (int l = 0; l < nlimb; ++l) {
            const int8_t d = (int8_t)(v & 0xff);  // low byte read as signed: in [-128, 127]
            D[(size_t)l * n + e] = d;
            v = (v - d) >> 8;                     // exact: v - d is a multiple of 256
        }
    }
}

// run-major user spins [R x N] -> zero-padded operand [ldr x Ke]
__global__ void k_pad_spins(const int8_t *s, int R, int N, int Ke, int8_t *out)
{
    const int r = blockIdx.y;
    for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < Ke; k += gridDim.x * blockDim.x)
        out[(size_t)r * Ke + k] = (r < R && k < N) ? s[(size_t)r * N + k] : 0;
}

__global__ __launch_bounds__(ENT) void k_dense_energy_i8(const int8_t *__restrict__ D, int nlimb, int Me, int Ke,
                                                          const int8_t *__restrict__ S, int R,
                                                          const int64_t *__restrict__ hfix, int N,
                                                          __int128 *__restrict__ partial)
{
    __shared__ __attribute__((aligned(16))) int8_t As[2][EBM][ELDS];
    __shared__ __attribute__((aligned(16))) int8_t Bs[2][EBN][ELDS];
    __shared__ long long red[2][EBN][2];  // [wm][column][lo/hi] partial energies of the two row halves

    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int wm = wave >> 1, wn = wave & 1;
    const int li = lane & 31, kh = lane >> 5;
    const int i0 = blockIdx.y * EBM;   // spin rows of the tile
    const int c0 = blockIdx.x * EBN;   // run columns of the tile
    const size_t plane = (size_t)Me * Ke;

    // loader: 128 rows x 128 bytes per operand = 1024 chunks of 16 B, 4 per thread
    const int lr = tid >> 3;          // 0..31
    const int lc = (tid & 7) * 16;    // byte column

    // signs of this lane's output elements: s_{r, i} for its 2 x 2 blocks x 16 rows
    uint32_t neg[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) {
            uint32_t m = 0;
            const int r = c0 + wn * 64 + b * 32 + li;
#pragma unroll
            for (int v = 0; v < 16; ++v) {
                const int i = i0 + wm * 64 + a * 32 + 8 * (v >> 2) + 4 * kh + (v & 3);
                const int8_t sv = (i < Ke) ? S[(size_t)r * Ke + i] : 0;
                m |= (sv < 0 ? 1u : 0u) << v;
            }
            neg[a][b] = m;
        }

    __int128 tot[2] = {0, 0};  // per column b of this lane, summed over its rows and all digits
    const int nk = Ke / EBK;
    for (int l = 0; l < nlimb; ++l) {
        const int8_t *A = D + (size_t)l * plane;
        intx16 acc[2][2];
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int b = 0; b < 2; ++b)
#pragma unroll
                for (int v = 0; v < 16; ++v)
                    acc[a][b][v] = 0;
        intx4 ga[4], gb[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            ga[q] = *reinterpret_cast<const intx4 *>(A + (size_t)(i0 + lr + 32 * q) * Ke + lc);
            gb[q] = *reinterpret_cast<const intx4 *>(S + (size_t)(c0 + lr + 32 * q) * Ke + lc);
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            *reinterpret_cast<intx4 *>(&As[0][lr + 32 * q][lc]) = ga[q];
            *reinterpret_cast<intx4 *>(&Bs[0][lr + 32 * q][lc]) = gb[q];
        }
        __syncthreads();
        for (int kt = 0; kt < nk; ++kt) {
            const int cur = kt & 1;
            if (kt + 1 < nk) {
                const int k0 = (kt + 1) * EBK;
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    ga[q] = *reinterpret_cast<const intx4 *>(A + (size_t)(i0 + lr + 32 * q) * Ke + k0 + lc);
                    gb[q] = *reinterpret_cast<const intx4 *>(S + (size_t)(c0 + lr + 32 * q) * Ke + k0 + lc);
                }
            }
#pragma unroll
            for (int ks = 0; ks < EBK / 32; ++ks) {
                intx4 fa[2], fb[2];
#pragma unroll
                for (int a = 0; a < 2; ++a)
                    fa[a] = *reinterpret_cast<const intx4 *>(&As[cur][wm * 64 + a * 32 + li][ks * 32 + kh * 16]);
#pragma unroll
                for (int b = 0; b < 2; ++b)
                    fb[b] = *reinterpret_cast<const intx4 *>(&Bs[cur][wn * 64 + b * 32 + li][ks * 32 + kh * 16]);
#pragma unroll
                for (int a = 0; a < 2; ++a)
#pragma unroll
                    for (int b = 0; b < 2; ++b)
                        acc[a][b] = __builtin_amdgcn_mfma_i32_32x32x32_i8(fa[a], fb[b], acc[a][b], 0, 0, 0);
            }
            if (kt + 1 < nk) {
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    *reinterpret_cast<intx4 *>(&As[cur ^ 1][lr + 32 * q][lc]) = ga[q];
                    *reinterpret_cast<intx4 *>(&Bs[cur ^ 1][lr + 32 * q][lc]) = gb[q];
                }
            }
            __syncthreads();
        }
        // fold this digit: sum_i s_ir (D_l S)_ir over the lane's rows, weighted 256^l
#pragma unroll
        for (int b = 0; b < 2; ++b) {
            long long qsum = 0;
#pragma unroll
            for (int a = 0; a < 2; ++a)
#pragma unroll
                for (int v = 0; v < 16; ++v) {
                    const long long x = acc[a][b][v];
                    qsum += ((neg[a][b] >> v) & 1u) ? -x : x;
                }
            tot[b] += (__int128)qsum << (8 * l);
        }
    }
    // field term sum_i s_ir hfix_i, counted once per row (lanes with wn == 0... every
    // lane holds distinct (row, column) pairs, so each pair adds its own term)
    if (hfix) {
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int a = 0; a < 2; ++a)
#pragma unroll
                for (int v = 0; v < 16; ++v) {
                    const int i = i0 + wm * 64 + a * 32 + 8 * (v >> 2) + 4 * kh + (v & 3);
                    if (i < N) {
                        const __int128 hv = hfix[i];
                        tot[b] += ((neg[a][b] >> v) & 1u) ? -hv : hv;
                    }
                }
    }
    // combine the two lane halves (rows 4*kh..) of each column, then the two
    // waves (wm) sharing the column, and write the tile's partial energy sum
#pragma unroll
    for (int b = 0; b < 2; ++b) {
        long long lo = (long long)(uint64_t)tot[b], hi = (long long)(tot[b] >> 64);
        const long long lo2 = __shfl_xor(lo, 32), hi2 = __shfl_xor(hi, 32);
        __int128 t = ((__int128)hi << 64) | (uint64_t)lo;
        t += ((__int128)hi2 << 64) | (uint64_t)lo2;
        if (kh == 0) {
            const int col = wn * 64 + b * 32 + li;
            red[wm][col][0] = (long long)(uint64_t)t;
            red[wm][col][1] = (long long)(t >> 64);
        }
    }
    __syncthreads();
    if (tid < EBN) {
        const int r = c0 + tid;
        __int128 t0 = ((__int128)red[0][tid][1] << 64) | (uint64_t)red[0][tid][0];
        __int128 t1 = ((__int128)red[1][tid][1] << 64) | (uint64_t)red[1][tid][0];
        if (r < R)
            partial[(size_t)blockIdx.y * R + r] = t0 + t1;
    }
}

void launch_dense_limbs(const Instance &I, hipStream_t s)
{
    k_dense_limbs<<<4096, 256, 0, s>>>(I.Jfix, I.N, I.nlimb, I.Me, I.Ke, I.Jlimb);
}

size_t dense_spin_operand_bytes(const Instance &I, int R)
{
    return (size_t)((R + EBN - 1) / EBN * EBN) * I.Ke;
}

void launch_pad_spins(const Instance &I, const int8_t *spins, int R, int8_t *Spad, hipStream_t s)
{
    const int ldr = (R + EBN - 1) / EBN * EBN;
    dim3 grid((I.Ke + 255) / 256, ldr);
    k_pad_spins<<<grid, 256, 0, s>>>(spins, R, I.N, I.Ke, Spad);
}

__global__ void k_energy_finish_i8(const __int128 *partial, int nblk, int R, int emin, double *E)
{
    int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= R)
        return;
    __int128 t = 0;
    for (int b = 0; b < nblk; ++b)
        t += partial[(size_t)b * R + r];
    E[r] = i128_to_double_scaled(-t, emin);
}

size_t dense_energy_partial_bytes(const Instance &I, int R)
{
    return (size_t)(I.Me / EBM) * (size_t)R * sizeof(__int128);
}

void launch_dense_energy_i8(const Instance &I, const int8_t *Spad, int R, double *E, void *partial, hipStream_t s)
{
    const int nrt = I.Me / EBM;
    dim3 grid((R + EBN - 1) / EBN, nrt);
    __int128 *part = reinterpret_cast<__int128 *>(partial);
    k_dense_energy_i8<<<grid, ENT, 0, s>>>(I.Jlimb, I.nlimb, I.Me, I.Ke, Spad, R, I.has_h ? I.hfix : nullptr, I.N,
                                           part);
    k_energy_finish_i8<<<(R + 255) / 256, 256, 0, s>>>(part, nrt, R, I.emin, E);
}

}  // namespace mars
