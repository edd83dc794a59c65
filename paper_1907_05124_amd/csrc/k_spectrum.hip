// Extreme eigenvalues of the coupling matrix J by the Lanczos iteration
// (fp64 vectors, no reorthogonalisation: the extreme Ritz values converge
// first and are not disturbed by the spurious copies that loss of
// orthogonality produces inside the spectrum).  Every step runs on the device
// with the recurrence coefficients kept in device memory, so the host waits
// once, at the end.
//
// Why the extremes: around the trivial fixed point m = 0 the update
// m <- tanh((J m + h/2) / T) is linear, m <- J m / T (h = 0), so the random
// start decays to 0 at every temperature above lambda_max(J), and the
// synchronous update turns unstable along the most negative eigenvector
// below |lambda_min(J)|.  The temperature range of an anneal is therefore
// measured in units of these two numbers.
#include <cmath>

#include "common_device.h"
#include "mars_internal.h"

namespace mars {

constexpr int SPT = 1024;  // threads of the one-workgroup reductions

// y = J x: dense rows (fp32 couplings, fp64 sums), one wave per row
__global__ __launch_bounds__(256) void k_spec_mv_dense(const float *__restrict__ J, int ld, int N,
                                                       const double *__restrict__ x, double *__restrict__ y)
{
    const int row = blockIdx.x * 4 + (int)(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (row >= N)
        return;
    const float *Jr = J + (size_t)row * ld;
    double acc = 0.0;
    for (int j = lane; j < N; j += 64)
        acc += (double)Jr[j] * x[j];
    for (int m = 32; m >= 1; m >>= 1)
        acc += __shfl_xor(acc, m);
    if (lane == 0)
        y[row] = acc;
}

// y = J x: sparse rows (CSR copy: (col << 8) | uint8(weight))
__global__ void k_spec_mv_csr(int N, const int32_t *__restrict__ rowptr, const uint32_t *__restrict__ colval,
                              const double *__restrict__ x, double *__restrict__ y)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N)
        return;
    double acc = 0.0;
    for (int k = rowptr[i]; k < rowptr[i + 1]; ++k) {
        const uint32_t cv = colval[k];
        acc += (double)(int8_t)(cv & 0xff) * x[cv >> 8];
    }
    y[i] = acc;
}

// y = J x: periodic lattice, bond bit q set means J = -1 towards neighbour q
// (+x, -x, +y, -y, +z, -z)
__global__ void k_spec_mv_lattice(int N, int dim, int L0, int L1, int L2, const uint8_t *__restrict__ bonds,
                                  const double *__restrict__ x, double *__restrict__ y)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N)
        return;
    const int xx = i % L0, yy = (i / L0) % L1, zz = i / (L0 * L1);
    const int nb[6] = {i - xx + (xx + 1) % L0,
                       i - xx + (xx + L0 - 1) % L0,
                       i + ((yy + 1) % L1 - yy) * L0,
                       i + ((yy + L1 - 1) % L1 - yy) * L0,
                       i + ((zz + 1) % L2 - zz) * L0 * L1,
                       i + ((zz + L2 - 1) % L2 - zz) * L0 * L1};
    const uint32_t b = bonds[i];
    double acc = 0.0;
    for (int q = 0; q < 2 * dim; ++q)
        acc += ((b >> q) & 1) ? -x[nb[q]] : x[nb[q]];
    y[i] = acc;
}

// one workgroup: out = sum_i a_i b_i in a fixed order (thread partial sums
// over a fixed stride, then a fixed tree)
__device__ double block_dot(const double *a, const double *b, int N)
{
    __shared__ double red[SPT];
    double acc = 0.0;
    for (int i = threadIdx.x; i < N; i += SPT)
        acc += a[i] * b[i];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int w = SPT / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w)
            red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    const double r = red[0];
    __syncthreads();
    return r;
}

// start vector: uniform draws in (-1, 1) from the counter generator, scaled to unit norm
__global__ __launch_bounds__(SPT) void k_spec_start(uint64_t seed, int N, double *v)
{
    for (int i = threadIdx.x; i < N; i += SPT)
        v[i] = (double)draw_m0(seed, 0, i);
    __syncthreads();
    const double nrm = sqrt(block_dot(v, v, N));
    for (int i = threadIdx.x; i < N; i += SPT)
        v[i] /= nrm;
}

// Lanczos step j after w = J v: alpha_j = w . v, w -= alpha_j v + beta_{j-1} v_prev,
// beta_j = |w|, v_next = w / beta_j (0 if the Krylov space closed)
__global__ __launch_bounds__(SPT) void k_spec_step(int N, int j, const double *v, const double *vprev, double *w,
                                                   double *vnext, double *alpha, double *beta)
{
    const double a = block_dot(w, v, N);
    const double bprev = j > 0 ? beta[j - 1] : 0.0;
    for (int i = threadIdx.x; i < N; i += SPT)
        w[i] -= a * v[i] + (j > 0 ? bprev * vprev[i] : 0.0);
    __syncthreads();
    const double b = sqrt(block_dot(w, w, N));
    for (int i = threadIdx.x; i < N; i += SPT)
        vnext[i] = b > 0.0 ? w[i] / b : 0.0;
    if (threadIdx.x == 0) {
        alpha[j] = a;
        beta[j] = b;
    }
}

hipError_t launch_spectrum_lanczos(const Instance &I, int steps, uint64_t seed, double *vecs, double *alpha,
                                   double *beta, hipStream_t s)
{
    const int N = I.N;
    double *v[3] = {vecs, vecs + N, vecs + 2 * (size_t)N};
    double *w = vecs + 3 * (size_t)N;
    k_spec_start<<<1, SPT, 0, s>>>(seed, N, v[0]);
    int cur = 0, prev = 2, next = 1;
    for (int j = 0; j < steps; ++j) {
        if (I.kind == KIND_DENSE)
            k_spec_mv_dense<<<(N + 3) / 4, 256, 0, s>>>(I.J, I.Np, N, v[cur], w);
        else if (I.kind == KIND_CSR)
            k_spec_mv_csr<<<(N + 255) / 256, 256, 0, s>>>(N, I.rowptr, I.colval, v[cur], w);
        else
            k_spec_mv_lattice<<<(N + 255) / 256, 256, 0, s>>>(N, I.dim, I.L[0], I.L[1], I.L[2], I.bondbits,
                                                               v[cur], w);
        k_spec_step<<<1, SPT, 0, s>>>(N, j, v[cur], v[prev], w, v[next], alpha, beta);
        const int t = prev;
        prev = cur;
        cur = next;
        next = t;
    }
    return hipGetLastError();
}

}  // namespace mars
