// Host runtime behind include/mars.h: input validation, device encodings of
// an instance, workspace management and the order of kernel launches of a
// solve.  No arithmetic of the method runs here; every step of a solve is a
// kernel on the caller's stream.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <vector>

#include "common_device.h"
#include "mars_internal.h"

namespace mars {

static thread_local std::string g_last_error;

mars_status set_error(mars_status s, const std::string &msg)
{
    g_last_error = msg;
    return s;
}

mars_status hip_error(hipError_t e, const char *what)
{
    std::string m = std::string(what) + ": " + hipGetErrorString(e);
    if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation)
        return set_error(MARS_E_OOM, m);
    return set_error(MARS_E_DEVICE, m);
}

// Test hook: with MARS_TEST_FAIL_ALLOC=1 in the environment (read at each
// allocation) every device allocation of the library's instances and
// workspaces fails as out of memory, so that tests can drive the error paths
// of creation and of solves.
static bool injected_alloc_failure()
{
    const char *f = std::getenv("MARS_TEST_FAIL_ALLOC");
    return f && f[0] == '1' && !f[1];
}

mars_status ensure(DevBuf &b, size_t bytes)
{
    if (bytes == 0)
        bytes = 16;
    if (b.bytes >= bytes)
        return MARS_OK;
    if (b.p) {
        hipError_t e = hipFree(b.p);
        b.p = nullptr;
        b.bytes = 0;
        if (e != hipSuccess)
            return hip_error(e, "hipFree");
    }
    if (injected_alloc_failure())
        return set_error(MARS_E_OOM, "workspace allocation refused (MARS_TEST_FAIL_ALLOC)");
    hipError_t e = hipMalloc(&b.p, bytes);
    if (e != hipSuccess) {
        b.p = nullptr;
        return hip_error(e, "hipMalloc workspace");
    }
    b.bytes = bytes;
    return MARS_OK;
}

static void free_buf(DevBuf &b)
{
    if (b.p)
        (void)hipFree(b.p);
    b.p = nullptr;
    b.bytes = 0;
}

template <typename T>
static mars_status dev_alloc(T **p, size_t count)
{
    *p = nullptr;
    if (count == 0)
        count = 1;
    if (injected_alloc_failure())
        return set_error(MARS_E_OOM, "device allocation refused (MARS_TEST_FAIL_ALLOC)");
    hipError_t e = hipMalloc(reinterpret_cast<void **>(p), count * sizeof(T));
    if (e != hipSuccess) {
        *p = nullptr;
        return hip_error(e, "hipMalloc");
    }
    return MARS_OK;
}

static void destroy_instance(Instance *I)
{
    if (!I)
        return;
    (void)hipSetDevice(I->device);
    if (I->own_stream)
        (void)hipStreamSynchronize(I->own_stream);
    if (I->grp_event) {
        (void)hipEventSynchronize(I->grp_event);
        (void)hipEventDestroy(I->grp_event);
    }
    if (I->done_event) {
        (void)hipEventSynchronize(I->done_event);
        (void)hipEventDestroy(I->done_event);
    }
    void *ptrs[] = {I->J,      I->Jbf,     I->Jfix,    I->Jlimb,   I->hhalf, I->hhalf64,
                    I->hfix,   I->rowptr,  I->colval,  I->perm,    I->sl_meta, I->colsell,
                    I->cls,    I->hperm,   I->hperm64, I->bondbits, I->bondsgn};
    for (void *p : ptrs)
        if (p)
            (void)hipFree(p);
    Workspace &w = I->ws;
    DevBuf *bufs[] = {&w.Ma,      &w.Mb,       &w.invT,   &w.invT64, &w.T0,       &w.nlev, &w.runstat,
                      &w.dmax,    &w.spins,    &w.spad,   &w.energies, &w.partial, &w.result, &w.runstate,
                      &w.flag,    &w.spec,     &w.phi,      &w.paper,  &w.gstate, &w.grp};
    for (DevBuf *b : bufs)
        free_buf(*b);
    if (I->own_stream)
        (void)hipStreamDestroy(I->own_stream);
    delete I;
}

// ---------------------------------------------------------------------------
// fixed point for exact energies
// ---------------------------------------------------------------------------

// A nonzero finite float is an integer mantissa m times 2^q (normal: m has
// its implicit bit, q = biased exponent - 150; subnormal: q = -149).
// Exponent of its lowest set bit: q + ctz(m).
static int low_bit_exponent(float v)
{
    uint32_t u;
    std::memcpy(&u, &v, 4);
    const uint32_t be = (u >> 23) & 0xffu, m = (u & 0x7fffffu) | (be ? 0x800000u : 0u);
    const int q = be ? (int)be - 150 : -149;
    return q + __builtin_ctz(m);
}

// The e with 2^(e-1) <= |v| < 2^e: q + (number of bits of m).
static int high_bit_exponent(float v)
{
    uint32_t u;
    std::memcpy(&u, &v, 4);
    const uint32_t be = (u >> 23) & 0xffu, m = (u & 0x7fffffu) | (be ? 0x800000u : 0u);
    const int q = be ? (int)be - 150 : -149;
    return q + (32 - __builtin_clz(m));
}

// Bit budget: every term is a multiple of 2^emin below 2^emax.  Row sums of
// N terms need emax - emin + log2(N) bits; the total another log2(N).
struct FixInfo {
    int emin = 0, emax = -1000;
    bool any = false;
    void add(float v)
    {
        if (v == 0.0f)
            return;
        emin = any ? std::min(emin, low_bit_exponent(v)) : low_bit_exponent(v);
        emax = any ? std::max(emax, high_bit_exponent(v)) : high_bit_exponent(v);
        any = true;
    }
};

static int ceil_log2(long long n)
{
    int b = 0;
    while ((1ll << b) < n)
        ++b;
    return b;
}

// ---------------------------------------------------------------------------
// instance creation
// ---------------------------------------------------------------------------

static mars_status start_instance(Instance *I)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess)
        return hip_error(e, "hipGetDevice");
    I->device = dev;
    hipDeviceProp_t prop;
    e = hipGetDeviceProperties(&prop, dev);
    if (e != hipSuccess)
        return hip_error(e, "hipGetDeviceProperties");
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
        return set_error(MARS_E_DEVICE, std::string("this library is built for gfx950, device is ") + prop.gcnArchName);
    e = hipStreamCreateWithFlags(&I->own_stream, hipStreamNonBlocking);
    if (e != hipSuccess)
        return hip_error(e, "hipStreamCreate");
    e = hipEventCreateWithFlags(&I->done_event, hipEventDisableTiming);
    if (e != hipSuccess)
        return hip_error(e, "hipEventCreate");
    int khz = 0;
    e = hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev);
    if (e != hipSuccess || khz <= 0)
        return e != hipSuccess ? hip_error(e, "hipDeviceGetAttribute(WallClockRate)")
                               : set_error(MARS_E_DEVICE, "device reports no constant-rate clock");
    I->tick_s = 1.0 / (1000.0 * (double)khz);
    return MARS_OK;
}

static mars_status check_h(const float *h, int N, FixInfo &fx)
{
    if (!h)
        return MARS_OK;
    for (int i = 0; i < N; ++i) {
        if (!std::isfinite(h[i]))
            return set_error(MARS_E_NONFINITE, "h contains a non-finite value");
        fx.add(h[i]);
    }
    return MARS_OK;
}

static mars_status upload_h(Instance *I, const float *h, int padN)
{
    const int N = I->N;
    I->has_h = false;
    if (!h)
        return MARS_OK;
    bool any = false;
    for (int i = 0; i < N; ++i)
        any |= h[i] != 0.0f;
    if (!any)
        return MARS_OK;
    I->has_h = true;
    std::vector<float> hh((size_t)padN, 0.0f);
    std::vector<double> hh64((size_t)N);
    std::vector<int64_t> hf((size_t)N);
    for (int i = 0; i < N; ++i) {
        hh[i] = h[i] * 0.5f;  // exact: halving a float (normal range) is exact
        hh64[i] = (double)h[i] * 0.5;
        hf[i] = (int64_t)std::ldexp((double)h[i], -I->emin);
    }
    mars_status st;
    if ((st = dev_alloc(&I->hhalf, (size_t)padN)) != MARS_OK)
        return st;
    if ((st = dev_alloc(&I->hhalf64, (size_t)N)) != MARS_OK)
        return st;
    if ((st = dev_alloc(&I->hfix, (size_t)N)) != MARS_OK)
        return st;
    MARS_HIP(hipMemcpyAsync(I->hhalf, hh.data(), sizeof(float) * padN, hipMemcpyHostToDevice, I->own_stream));
    MARS_HIP(hipMemcpyAsync(I->hhalf64, hh64.data(), sizeof(double) * N, hipMemcpyHostToDevice, I->own_stream));
    MARS_HIP(hipMemcpyAsync(I->hfix, hf.data(), sizeof(int64_t) * N, hipMemcpyHostToDevice, I->own_stream));
    // the host vectors die on return: wait for the copies
    MARS_HIP(hipStreamSynchronize(I->own_stream));
    return MARS_OK;
}

// Validation scan of dense couplings, rows split over host threads.  Pass 1
// checks every value is finite.  Pass 2 walks 64 x 64 tiles of the upper
// triangle (the transposed tile stays in cache): zero diagonal, bitwise
// symmetry, the fixed-point exponent range, and row sums kept per row and
// added in row order afterwards (independent of the thread count).  A
// fault is reported for the lowest row that has one, diagonal before
// symmetry, as a row-by-row scan would.
struct DenseScan {
    FixInfo fx;
    bool nonfinite = false;
    long long fault_row = -1;  // lowest row with a diagonal (2) or symmetry (3) fault
    int fault = 0;
    void note(long long row, int kind)
    {
        if (fault_row < 0 || row < fault_row || (row == fault_row && kind < fault)) {
            fault_row = row;
            fault = kind;
        }
    }
};

static void scan_dense_tile_row(const float *J, long long N, long long bi, std::vector<double> &rowsum, DenseScan &out)
{
    constexpr long long TB = 64;
    const long long i0 = bi * TB, i1 = std::min(N, i0 + TB);
    for (long long i = i0; i < i1; ++i)
        if (J[i * N + i] != 0.0f)
            out.note(i, 2);
    for (long long j0 = i0; j0 < N; j0 += TB) {
        const long long j1 = std::min(N, j0 + TB);
        for (long long i = i0; i < i1; ++i) {
            double rs = 0.0;
            for (long long j = std::max(j0, i + 1); j < j1; ++j) {
                const float a = J[i * N + j], b = J[j * N + i];
                uint32_t ua, ub;
                std::memcpy(&ua, &a, 4);
                std::memcpy(&ub, &b, 4);
                if (ua != ub)
                    out.note(i, 3);
                out.fx.add(a);
                rs += (double)a;
            }
            rowsum[(size_t)i] += rs;
        }
    }
}

static mars_status create_dense(const float *J, const float *h, int N, Instance *I)
{
    I->kind = KIND_DENSE;
    I->N = N;
    FixInfo fx;
    double wsum = 0.0;
    {
        const long long nb = ((long long)N + 63) / 64;
        int nt = (int)std::min<unsigned>(std::max(1u, std::thread::hardware_concurrency()), 16u);
        nt = (int)std::min<long long>(nt, std::max(1ll, nb / 4));
        std::vector<double> rowsum((size_t)N, 0.0);
        std::vector<DenseScan> part((size_t)nt);
        auto run = [&](auto &&fn) {
            std::vector<std::thread> pool;
            for (int t = 1; t < nt; ++t)
                pool.emplace_back(fn, t);
            fn(0);
            for (auto &th : pool)
                th.join();
        };
        const long long NN = (long long)N * N;
        run([&](int t) {
            const long long a = NN * t / nt, b = NN * (t + 1) / nt;
            for (long long k = a; k < b; ++k)
                if (!std::isfinite(J[k])) {
                    part[(size_t)t].nonfinite = true;
                    return;
                }
        });
        for (const DenseScan &d : part)
            if (d.nonfinite)
                return set_error(MARS_E_NONFINITE, "J contains a non-finite value");
        // interleaved tile rows balance the triangle's uneven row lengths; a
        // thread stops after the first tile row where it found a fault
        run([&](int t) {
            for (long long bi = t; bi < nb && part[(size_t)t].fault == 0; bi += nt)
                scan_dense_tile_row(J, N, bi, rowsum, part[(size_t)t]);
        });
        const DenseScan *first = nullptr;
        for (const DenseScan &d : part) {
            if (d.fault && (!first || d.fault_row < first->fault_row ||
                            (d.fault_row == first->fault_row && d.fault < first->fault)))
                first = &d;
            if (d.fx.any) {
                fx.emin = fx.any ? std::min(fx.emin, d.fx.emin) : d.fx.emin;
                fx.emax = fx.any ? std::max(fx.emax, d.fx.emax) : d.fx.emax;
                fx.any = true;
            }
        }
        if (first && first->fault == 2)
            return set_error(MARS_E_DIAGONAL, "J has a nonzero diagonal entry (the energy sums j != i)");
        if (first)
            return set_error(MARS_E_ASYMMETRIC, "J is not symmetric (bitwise)");
        for (int i = 0; i < N; ++i)
            wsum -= 2.0 * rowsum[(size_t)i];
    }
    mars_status st = check_h(h, N, fx);
    if (st != MARS_OK)
        return st;
    I->emin = fx.any ? fx.emin : 0;
    const int bits = fx.any ? fx.emax - I->emin : 0;  // |fixed value| < 2^bits
    if (bits > 62)
        return set_error(MARS_E_RANGE, "coupling/field values span more than 62 bits of binary range");
    const int lg = ceil_log2((long long)N + 1);
    if (bits + 2 * lg + 2 > 126)
        return set_error(MARS_E_RANGE, "exact energy would need more than 126 bits");
    I->wsum = wsum;
    // balanced base-256 digits: L digits cover |v| < 2^(8L-1)
    I->nlimb = std::max(1, (bits + 1 + 7) / 8);
    I->Me = I->Ke = ((N + 127) / 128) * 128;
    I->Np = ((N + 127) / 128) * 128 + 128;
    const size_t Np = (size_t)I->Np;
    if ((st = dev_alloc(&I->J, Np * Np)) != MARS_OK)
        return st;
    MARS_HIP(hipMemsetAsync(I->J, 0, sizeof(float) * Np * Np, I->own_stream));
    MARS_HIP(hipMemcpy2DAsync(I->J, sizeof(float) * Np, J, sizeof(float) * N, sizeof(float) * N, N,
                              hipMemcpyHostToDevice, I->own_stream));
    // the fixed-point copy is a temporary of the limb encoding: stream-ordered
    // allocation and release, so that creating an instance does not wait for
    // the device's other work (a plain free synchronises the device)
    {
        void *p = nullptr;
        hipError_t e = hipMallocAsync(&p, sizeof(*I->Jfix) * (size_t)N * N, I->own_stream);
        if (e != hipSuccess)
            return e == hipErrorOutOfMemory ? set_error(MARS_E_OOM, "device memory exhausted")
                                            : hip_error(e, "hipMallocAsync");
        I->Jfix = static_cast<decltype(I->Jfix)>(p);
    }
    launch_dense_fixpoint(*I, I->own_stream);
    MARS_HIP(hipGetLastError());
    if ((st = dev_alloc(&I->Jlimb, (size_t)I->nlimb * I->Me * I->Ke)) != MARS_OK)
        return st;
    launch_dense_limbs(*I, I->own_stream);
    MARS_HIP(hipGetLastError());
    MARS_HIP(hipFreeAsync(I->Jfix, I->own_stream));
    I->Jfix = nullptr;
    if ((st = upload_h(I, h, I->Np)) != MARS_OK)
        return st;
    MARS_HIP(hipStreamSynchronize(I->own_stream));
    return MARS_OK;
}

// Solver encodings of a symmetric sparse coupling matrix given as CSR: the
// greedy colouring (update phases), the sliced-ELL table and the field by
// slot (ncolours, nslot, unit, h_cls, perm, sl_meta, colsell, cls, hperm,
// hperm64 of the instance).  Inputs are valid (checked by the caller).
static mars_status build_sell(Instance *I, int N, const int32_t *rowptr, const int32_t *col, const int8_t *val,
                              const float *h)
{
    mars_status st;
    int maxdeg = 0;
    for (int i = 0; i < N; ++i)
        maxdeg = std::max(maxdeg, rowptr[i + 1] - rowptr[i]);
    // greedy colouring in index order: colour(v) = smallest colour not used by
    // neighbours u < v; each colour class is one update phase
    std::vector<int32_t> colour((size_t)N, 0);
    std::vector<char> used((size_t)maxdeg + 2, 0);
    int ncol = 1;
    for (int v = 0; v < N; ++v) {
        for (int k = rowptr[v]; k < rowptr[v + 1]; ++k)
            if (col[k] < v && colour[col[k]] <= maxdeg)
                used[colour[col[k]]] = 1;
        int c = 0;
        while (used[c])
            ++c;
        colour[v] = c;
        ncol = std::max(ncol, c + 1);
        for (int k = rowptr[v]; k < rowptr[v + 1]; ++k)
            if (col[k] < v && colour[col[k]] <= maxdeg)
                used[colour[col[k]]] = 0;
    }
    std::vector<int32_t> pptr((size_t)ncol + 1, 0), pvert((size_t)N);
    for (int v = 0; v < N; ++v)
        ++pptr[colour[v] + 1];
    for (int c = 0; c < ncol; ++c)
        pptr[c + 1] += pptr[c];
    {
        std::vector<int32_t> fill(pptr.begin(), pptr.end() - 1);
        for (int v = 0; v < N; ++v)
            pvert[fill[colour[v]]++] = v;
    }
    I->ncolours = ncol;
    // sliced-ELL copy for the solver: classes in colour order, each sorted by
    // degree (descending, ties by index) and padded to whole slices, so that
    // the SELL_H vertices of a slice have similar degrees and the threads of a
    // wave read consecutive entries
    std::vector<int32_t> perm, slot_of((size_t)N), cls((size_t)2 * ncol);
    for (int c = 0; c < ncol; ++c) {
        std::vector<int32_t> vs(pvert.begin() + pptr[c], pvert.begin() + pptr[c + 1]);
        std::stable_sort(vs.begin(), vs.end(), [&](int32_t x, int32_t y) {
            return rowptr[x + 1] - rowptr[x] > rowptr[y + 1] - rowptr[y];
        });
        cls[2 * c] = (int32_t)perm.size();
        cls[2 * c + 1] = (int32_t)vs.size();
        for (int32_t v : vs) {
            slot_of[v] = (int32_t)perm.size();
            perm.push_back(v);
        }
        while (perm.size() % SELL_H)
            perm.push_back(-1);
    }
    const int nslot = (int)perm.size();
    if (nslot >= (1 << 24))
        return set_error(MARS_E_UNSUPPORTED, "sparse instances are limited to fewer than 2^24 slots");
    const int nslice = nslot / SELL_H;
    std::vector<int32_t> meta((size_t)2 * nslice);
    size_t total = 0;
    for (int sl = 0; sl < nslice; ++sl) {
        int w = 0;
        for (int l = 0; l < SELL_H; ++l) {
            const int v = perm[(size_t)sl * SELL_H + l];
            if (v >= 0)
                w = std::max(w, rowptr[v + 1] - rowptr[v]);
        }
        w = (w + SELL_W - 1) / SELL_W * SELL_W;  // whole groups of SELL_W entries
        meta[2 * sl] = (int32_t)total;
        meta[2 * sl + 1] = w;
        total += (size_t)w * SELL_H;
    }
    if (total >= (size_t)1 << 31)
        return set_error(MARS_E_UNSUPPORTED, "sliced layout exceeds 2^31 entries");
    // +-1 weights keep only the sign, in bit 31 (the solver then shifts the
    // entry into a byte offset without masking); other weights the int8 byte
    bool unit = true;
    for (long long k = 0; k < (long long)rowptr[N]; ++k)
        unit &= (val[k] == 1 || val[k] == -1);
    // entry groups of padding after the last slice: a lane reads up to
    // SPARSE_READ_AHEAD of its groups past the last one it sums, and a lane's
    // groups are up to SPARSE_LPS_MAX apart
    std::vector<uint32_t> cs(total + (size_t)SPARSE_READ_AHEAD * SPARSE_LPS_MAX * SELL_W * SELL_H, unit ? (uint32_t)nslot : (uint32_t)nslot | (1u << 24));
    for (int sl = 0; sl < nslice; ++sl)
        for (int l = 0; l < SELL_H; ++l) {
            const int v = perm[(size_t)sl * SELL_H + l];
            if (v < 0)
                continue;
            for (int k = rowptr[v]; k < rowptr[v + 1]; ++k) {
                const int j = k - rowptr[v];
                const size_t at = (size_t)meta[2 * sl] + ((size_t)(j / SELL_W) * SELL_H + l) * SELL_W + j % SELL_W;
                cs[at] = (uint32_t)slot_of[col[k]] |
                         (unit ? (val[k] < 0 ? 0x80000000u : 0u) : ((uint32_t)(uint8_t)val[k] << 24));
            }
        }
    I->nslot = nslot;
    I->unit = unit;
    I->h_cls = cls;
    if ((st = dev_alloc(&I->perm, perm.size())) != MARS_OK)
        return st;
    if ((st = dev_alloc(&I->sl_meta, meta.size())) != MARS_OK)
        return st;
    if ((st = dev_alloc(&I->colsell, cs.size())) != MARS_OK)
        return st;
    if ((st = dev_alloc(&I->cls, cls.size())) != MARS_OK)
        return st;
    hipStream_t s = I->own_stream;
    MARS_HIP(hipMemcpyAsync(I->perm, perm.data(), sizeof(int32_t) * perm.size(), hipMemcpyHostToDevice, s));
    MARS_HIP(hipMemcpyAsync(I->sl_meta, meta.data(), sizeof(int32_t) * meta.size(), hipMemcpyHostToDevice, s));
    MARS_HIP(hipMemcpyAsync(I->colsell, cs.data(), sizeof(uint32_t) * cs.size(), hipMemcpyHostToDevice, s));
    MARS_HIP(hipMemcpyAsync(I->cls, cls.data(), sizeof(int32_t) * cls.size(), hipMemcpyHostToDevice, s));
    if (h) {
        bool any = false;
        for (int i = 0; i < N; ++i)
            any |= h[i] != 0.0f;
        if (any) {
            std::vector<float> hp((size_t)nslot, 0.0f);
            std::vector<double> hp64((size_t)nslot, 0.0);
            for (int sl = 0; sl < nslot; ++sl)
                if (perm[sl] >= 0) {
                    hp[sl] = h[perm[sl]] * 0.5f;
                    hp64[sl] = (double)h[perm[sl]] * 0.5;
                }
            if ((st = dev_alloc(&I->hperm, (size_t)nslot)) != MARS_OK)
                return st;
            if ((st = dev_alloc(&I->hperm64, (size_t)nslot)) != MARS_OK)
                return st;
            MARS_HIP(hipMemcpyAsync(I->hperm, hp.data(), sizeof(float) * nslot, hipMemcpyHostToDevice, s));
            MARS_HIP(hipMemcpyAsync(I->hperm64, hp64.data(), sizeof(double) * nslot, hipMemcpyHostToDevice, s));
            MARS_HIP(hipStreamSynchronize(s));
        }
    }
    MARS_HIP(hipStreamSynchronize(s));
    return MARS_OK;
}

static mars_status create_csr(int N, const int32_t *rowptr, const int32_t *col, const int8_t *val, const float *h,
                              Instance *I)
{
    I->kind = KIND_CSR;
    I->N = N;
    if (rowptr[0] != 0)
        return set_error(MARS_E_ARG, "rowptr[0] must be 0");
    for (int i = 0; i < N; ++i)
        if (rowptr[i + 1] < rowptr[i])
            return set_error(MARS_E_ARG, "rowptr must be non-decreasing");
    const long long nnz = rowptr[N];
    if (nnz > 0 && (!col || !val))
        return set_error(MARS_E_ARG, "col and val are required when nnz > 0");
    if (N >= (1 << 24))
        return set_error(MARS_E_UNSUPPORTED, "sparse instances are limited to N < 2^24");
    FixInfo fx;
    int maxdeg = 0;
    double wsum = 0.0;
    for (int i = 0; i < N; ++i) {
        maxdeg = std::max(maxdeg, rowptr[i + 1] - rowptr[i]);
        for (int k = rowptr[i]; k < rowptr[i + 1]; ++k) {
            int j = col[k];
            if (j < 0 || j >= N)
                return set_error(MARS_E_ARG, "column index out of range");
            if (k > rowptr[i] && col[k - 1] >= j)
                return set_error(MARS_E_ARG, "columns must be strictly increasing within a row");
            if (j == i)
                return set_error(MARS_E_DIAGONAL, "self loop in CSR");
            if (val[k] == 0)
                return set_error(MARS_E_ARG, "stored values must be nonzero");
            // the mirror entry (j, i) must exist with the same value
            const int32_t *b = col + rowptr[j], *e = col + rowptr[j + 1];
            const int32_t *f = std::lower_bound(b, e, i);
            if (f == e || *f != i || val[rowptr[j] + (f - b)] != val[k])
                return set_error(MARS_E_ASYMMETRIC, "CSR couplings are not symmetric");
            fx.add((float)val[k]);
            wsum -= (double)val[k];
        }
    }
    mars_status st = check_h(h, N, fx);
    if (st != MARS_OK)
        return st;
    I->emin = fx.any ? std::min(0, fx.emin) : 0;
    I->maxdeg = maxdeg;
    I->wsum = wsum;
    I->nnz = (int)nnz;
    {
        // energy accumulates in 64 bits: N * (maxdeg * 128 + max|h|) in units of 2^emin
        const int bits = (fx.any ? fx.emax : 0) - I->emin + ceil_log2((long long)maxdeg + 2) + 1;
        if (bits + ceil_log2((long long)N + 1) + 1 > 62)
            return set_error(MARS_E_RANGE, "exact energy would overflow 64-bit accumulation");
    }
    // CSR copy for exact energies (original labels)
    std::vector<uint32_t> cv((size_t)std::max<long long>(nnz, 1));
    for (long long k = 0; k < nnz; ++k)
        cv[k] = ((uint32_t)col[k] << 8) | (uint32_t)(uint8_t)val[k];
    if ((st = dev_alloc(&I->rowptr, (size_t)N + 1)) != MARS_OK)
        return st;
    if ((st = dev_alloc(&I->colval, cv.size())) != MARS_OK)
        return st;
    MARS_HIP(hipMemcpyAsync(I->rowptr, rowptr, sizeof(int32_t) * (N + 1), hipMemcpyHostToDevice, I->own_stream));
    MARS_HIP(hipMemcpyAsync(I->colval, cv.data(), sizeof(uint32_t) * cv.size(), hipMemcpyHostToDevice,
                            I->own_stream));
    if ((st = build_sell(I, N, rowptr, col, val, h)) != MARS_OK)
        return st;
    return upload_h(I, h, N);
}

static mars_status create_lattice(int dim, const int32_t *L, const int8_t *bond, const float *h, Instance *I)
{
    I->kind = KIND_LATTICE;
    I->dim = dim;
    long long N = 1;
    for (int a = 0; a < dim; ++a) {
        if (L[a] < 4 || (L[a] & 1))
            return set_error(MARS_E_ARG, "lattice sizes must be even and >= 4");
        I->L[a] = L[a];
        N *= L[a];
    }
    if (N >= (1ll << 30))
        return set_error(MARS_E_ARG, "lattice too large");
    if (I->L[0] > 2048)
        return set_error(MARS_E_UNSUPPORTED, "lattice rows longer than 2048 sites");
    I->N = (int)N;
    FixInfo fx;
    double wsum = 0.0;
    for (long long k = 0; k < dim * N; ++k) {
        if (bond[k] != 1 && bond[k] != -1)
            return set_error(MARS_E_ARG, "lattice bonds must be +1 or -1");
        fx.add((float)bond[k]);
        wsum -= 2.0 * bond[k];
    }
    mars_status st = check_h(h, (int)N, fx);
    if (st != MARS_OK)
        return st;
    I->emin = fx.any ? std::min(0, fx.emin) : 0;
    I->maxdeg = 2 * dim;
    I->wsum = wsum;
    {
        const int bits = (fx.any ? fx.emax : 0) - I->emin + 4;
        if (bits + ceil_log2(N + 1) + 1 > 62)
            return set_error(MARS_E_RANGE, "exact energy would overflow 64-bit accumulation");
    }
    // per site: bit 2a = coupling to +e_a is negative, bit 2a+1 = coupling to -e_a
    std::vector<uint8_t> bits((size_t)N, 0);
    const int L0 = I->L[0], L1 = I->L[1], L2 = dim == 3 ? I->L[2] : 1;
    for (long long v = 0; v < N; ++v) {
        int x = (int)(v % L0), y = (int)((v / L0) % L1), z = (int)(v / ((long long)L0 * L1));
        long long mx = v - x + (x + L0 - 1) % L0;
        long long my = v + (long long)((y + L1 - 1) % L1 - y) * L0;
        long long mz = v + (long long)((z + L2 - 1) % L2 - z) * L0 * L1;
        uint8_t b = 0;
        if (bond[0 * N + v] < 0) b |= 1;
        if (bond[0 * N + mx] < 0) b |= 2;
        if (bond[1 * N + v] < 0) b |= 4;
        if (bond[1 * N + my] < 0) b |= 8;
        if (dim == 3) {
            if (bond[2 * N + v] < 0) b |= 16;
            if (bond[2 * N + mz] < 0) b |= 32;
        }
        bits[v] = b;
    }
    // the same signs as fp16 sign-bit positions: axis a's pair at bits 15 - a
    // and 31 - a, so that shifting left by a and masking 0x80008000 yields the
    // pair; twice over, so that a site index plus one walk step stays inside
    std::vector<uint32_t> sgn((size_t)2 * N, 0);
    for (long long v = 0; v < N; ++v) {
        uint32_t w = 0;
        for (int ax = 0; ax < 3; ++ax) {
            if (bits[v] >> (2 * ax) & 1)
                w |= 1u << (15 - ax);
            if (bits[v] >> (2 * ax + 1) & 1)
                w |= 1u << (31 - ax);
        }
        sgn[v] = sgn[v + N] = w;
    }
    if ((st = dev_alloc(&I->bondbits, (size_t)N)) != MARS_OK)
        return st;
    if ((st = dev_alloc(&I->bondsgn, (size_t)2 * N)) != MARS_OK)
        return st;
    MARS_HIP(hipMemcpyAsync(I->bondbits, bits.data(), (size_t)N, hipMemcpyHostToDevice, I->own_stream));
    MARS_HIP(hipMemcpyAsync(I->bondsgn, sgn.data(), (size_t)2 * N * sizeof(uint32_t), hipMemcpyHostToDevice,
                            I->own_stream));
    MARS_HIP(hipStreamSynchronize(I->own_stream));
    // the bonds and field as given, for the sparse encodings of a solve
    // beyond LDS (built on first use)
    I->lat_bond.assign(bond, bond + (size_t)dim * N);
    if (h)
        I->lat_h.assign(h, h + N);
    return upload_h(I, h, (int)N);
}

// The sparse encodings of a lattice (its couplings as a symmetric CSR matrix:
// site v couples to v + e_a with bond[a N + v] and to v - e_a with
// bond[a N + (v - e_a)], periodic), for the solver beyond LDS.  Greedy
// colouring in index order gives the checkerboard (every site but 0 has an
// earlier neighbour, of the other parity), class 0 the even sites, as the
// lattice solver's phases.
static mars_status lattice_sell(Instance *I)
{
    if (I->lat_sell)
        return MARS_OK;
    const int dim = I->dim, N = I->N;
    if (N >= (1 << 24))
        return set_error(MARS_E_UNSUPPORTED, "lattices beyond LDS are limited to fewer than 2^24 sites");
    const int L0 = I->L[0], L1 = I->L[1], L2 = dim == 3 ? I->L[2] : 1;
    std::vector<int32_t> rowptr((size_t)N + 1), col((size_t)2 * dim * N);
    std::vector<int8_t> val((size_t)2 * dim * N);
    const int8_t *bond = I->lat_bond.data();
    for (int v = 0; v < N; ++v) {
        const int x = v % L0, y = (v / L0) % L1, z = v / (L0 * L1);
        const int step[3] = {1, L0, L0 * L1};
        const int coord[3] = {x, y, z}, len[3] = {L0, L1, L2};
        std::pair<int32_t, int8_t> nb[6];
        int n = 0;
        for (int a = 0; a < dim; ++a) {
            const int up = v + ((coord[a] + 1) % len[a] - coord[a]) * step[a];
            const int dn = v + ((coord[a] + len[a] - 1) % len[a] - coord[a]) * step[a];
            nb[n++] = {up, bond[(size_t)a * N + v]};
            nb[n++] = {dn, bond[(size_t)a * N + dn]};
        }
        std::sort(nb, nb + n);
        rowptr[v] = 2 * dim * v;
        for (int k = 0; k < n; ++k) {
            col[(size_t)2 * dim * v + k] = nb[k].first;
            val[(size_t)2 * dim * v + k] = nb[k].second;
        }
    }
    rowptr[N] = 2 * dim * N;
    mars_status st = build_sell(I, N, rowptr.data(), col.data(), val.data(), I->lat_h.empty() ? nullptr : I->lat_h.data());
    if (st != MARS_OK)
        return st;
    if (I->ncolours != 2)
        return set_error(MARS_E_DEVICE, "lattice encodings: the colouring is not the checkerboard");
    I->lat_sell = true;
    return MARS_OK;
}

// ---------------------------------------------------------------------------
// solve
// ---------------------------------------------------------------------------

static mars_status check_schedule(const mars_schedule *s, int kind)
{
    if (!s)
        return set_error(MARS_E_ARG, "schedule is NULL");
    if (s->kind != MARS_GEOMETRIC && s->kind != MARS_LINEAR)
        return set_error(MARS_E_ARG, "schedule.kind must be MARS_GEOMETRIC or MARS_LINEAR");
    if (!std::isfinite(s->T_lo) || !std::isfinite(s->T_hi) || s->T_hi < s->T_lo || s->T_lo < 0.0)
        return set_error(MARS_E_ARG, "need finite 0 <= T_lo <= T_hi");
    if (s->kind == MARS_GEOMETRIC) {
        if (!(s->T_lo > 0.0) || !(s->T_end > 0.0) || !std::isfinite(s->T_end))
            return set_error(MARS_E_ARG, "geometric schedule needs T_lo > 0 and finite T_end > 0");
        if (s->steps < 0)
            return set_error(MARS_E_ARG, "steps must be >= 0");
    } else {
        if (!(s->c_step > 0.0) || !std::isfinite(s->c_step))
            return set_error(MARS_E_ARG, "linear schedule needs c_step > 0");
    }
    if (s->max_sweeps < 1)
        return set_error(MARS_E_ARG, "max_sweeps must be >= 1");
    if (!(s->d_min >= 0.0))
        return set_error(MARS_E_ARG, "d_min must be >= 0");
    if (s->update != MARS_PHASED && s->update != MARS_JACOBI && s->update != MARS_SEQUENTIAL)
        return set_error(MARS_E_ARG, "update must be MARS_PHASED, MARS_JACOBI or MARS_SEQUENTIAL");
    if (s->update == MARS_SEQUENTIAL && (kind != KIND_DENSE || s->precision != MARS_FP32))
        return set_error(MARS_E_UNSUPPORTED, "MARS_SEQUENTIAL is implemented for dense instances in MARS_FP32");
    if (kind == KIND_DENSE && s->update == MARS_PHASED && s->phases < 1)
        return set_error(MARS_E_ARG, "phases must be >= 1");
    if (!(s->damping > 0.0 && s->damping <= 1.0))
        return set_error(MARS_E_ARG, "damping must be in (0, 1]");
    if (s->first_level < 0)
        return set_error(MARS_E_ARG, "first_level must be >= 0");
    if (s->precision < MARS_FP32 || s->precision > MARS_FP16)
        return set_error(MARS_E_ARG, "unknown precision");
    return MARS_OK;
}

// Upper bound on the levels any run visits (table rows).
static mars_status max_levels(const mars_schedule &sc, double Tmax, int *out)
{
    RunSchedule rs = make_run_schedule(sc);
    if (sc.kind == MARS_GEOMETRIC) {
        int stop = sc.steps;
        if (sc.level_count >= 0 && rs.first + sc.level_count < stop)
            stop = rs.first + sc.level_count;
        *out = std::max(0, stop - rs.first);
        return MARS_OK;
    }
    LevelWalker w;
    w.start(rs, Tmax);
    int n = 0;
    while (!w.done) {
        ++n;
        if (n > 10000000)
            return set_error(MARS_E_ARG, "linear schedule has more than 1e7 levels");
        w.next(rs);
    }
    *out = n;
    return MARS_OK;
}

// Dense solve, first stage: buffers, starting temperatures, the level table
// and the initial state (Algorithm 1's random start), enqueued on s.
mars_status dense_setup(Instance *I, int R, const mars_schedule &sc, uint64_t seed, const float *m0,
                        const double *T0in, DenseRun &d, hipStream_t s)
{
    if (sc.precision != MARS_FP32 && sc.precision != MARS_BF16)
        return set_error(MARS_E_UNSUPPORTED, "dense instances support MARS_FP32 and MARS_BF16");
    d.bf16 = sc.precision == MARS_BF16;
    Workspace &w = I->ws;
    const int N = I->N;
    mars_status st;
    if (d.bf16 && (st = ensure_bf16_couplings(*I, s)) != MARS_OK)
        return st;
    // state: fp32 [Np x ldm] spin-major, or bf16 [ldr x Np] run-major
    d.R = R;
    d.ldm = ((R + 127) / 128) * 128;
    d.ldr = bf16_state_rows(R);
    const size_t mbytes =
        d.bf16 ? sizeof(unsigned short) * (size_t)d.ldr * I->Np : sizeof(float) * (size_t)I->Np * d.ldm;
    if ((st = ensure(w.Ma, mbytes)) || (st = ensure(w.Mb, mbytes)) || (st = ensure(w.T0, sizeof(double) * R)) ||
        (st = ensure(w.nlev, sizeof(int32_t) * R)) || (st = ensure(w.runstat, sizeof(int64_t) * 4 * R)) ||
        (st = ensure(w.dmax, sizeof(uint32_t) * d.ldr)) ||
        (st = ensure(w.runstate, (sizeof(int32_t) * 4 + sizeof(double)) * d.ldr)) ||
        (st = ensure(w.flag, 64)))
        return st;
    launch_fill_u32((uint32_t *)w.Ma.p, 0u, mbytes / 4, s);
    launch_fill_u32((uint32_t *)w.Mb.p, 0u, mbytes / 4, s);
    d.T0 = (double *)w.T0.p;
    launch_init_T0(seed, R, sc.T_lo, sc.T_hi, T0in, d.T0, s);
    double Tmax = sc.T_hi;
    if (T0in && sc.kind == MARS_LINEAR) {
        std::vector<double> h((size_t)R);
        MARS_HIP(hipMemcpyAsync(h.data(), T0in, sizeof(double) * R, hipMemcpyDeviceToHost, s));
        MARS_HIP(hipStreamSynchronize(s));
        Tmax = *std::max_element(h.begin(), h.end());
        if (!std::isfinite(Tmax))
            return set_error(MARS_E_ARG, "T0 contains a non-finite value");
    }
    if ((st = max_levels(sc, Tmax, &d.kmax)) != MARS_OK)
        return st;
    if ((st = ensure(w.invT, sizeof(float) * (size_t)std::max(d.kmax, 1) * d.ldr)) != MARS_OK)
        return st;
    // one table row per level; ldr >= ldm, so the same stride serves both forms
    d.ldt = d.ldr;
    d.table = (float *)w.invT.p;
    d.nlev = (int32_t *)w.nlev.p;
    // the fp32 form evaluates its update in fp64 and keeps an fp64 copy of the table
    if (!d.bf16 && sc.update != MARS_SEQUENTIAL) {
        if ((st = ensure(w.invT64, sizeof(double) * (size_t)std::max(d.kmax, 1) * d.ldr)) != MARS_OK)
            return st;
        d.table64 = (double *)w.invT64.p;
    }
    launch_level_table(sc, R, d.T0, d.kmax, d.ldt, d.table, d.table64, d.nlev, s);
    if (d.bf16)
        launch_bf16_init_state(seed, N, R, I->Np, m0, (unsigned short *)w.Ma.p, s);
    else
        launch_dense_init_state(seed, N, R, d.ldm, m0, (float *)w.Ma.p, s);
    if (sc.update == MARS_SEQUENTIAL) {
        d.B = (N + SEQ_NB - 1) / SEQ_NB;
        d.pb.assign((size_t)d.B + 1, 0);
        for (int b = 0; b <= d.B; ++b)
            d.pb[b] = std::min(b * SEQ_NB, N);
    } else {
        d.B = sc.update == MARS_JACOBI ? 1 : std::min(sc.phases, N);
        d.pb.assign((size_t)d.B + 1, 0);
        for (int b = 0; b <= d.B; ++b)
            d.pb[b] = (int)((long long)b * N / d.B);
    }
    d.seq = sc.update == MARS_SEQUENTIAL;
    d.gamma = (float)sc.damping;
    d.Ma = w.Ma.p;
    d.Mb = w.Mb.p;
    return MARS_OK;
}

// Dense solve, last stage: round the final state (cur), exact energies,
// best of runs.
mars_status dense_finish(Instance *I, const DenseRun &d, const void *cur, float *m_final, int8_t *spins, double *E,
                         int8_t *best_spins, mars_result *res_dev, int32_t *best_dev, hipStream_t s)
{
    Workspace &w = I->ws;
    const int N = I->N, R = d.R;
    mars_status st;
    if ((st = ensure(w.spad, dense_spin_operand_bytes(*I, R))) != MARS_OK)
        return st;
    int8_t *spad = (int8_t *)w.spad.p;
    if (d.bf16)
        launch_bf16_round((const unsigned short *)cur, I->Np, N, R, I->Ke, spad, spins, m_final, s);
    else
        launch_dense_round((const float *)cur, d.ldm, N, R, I->Ke, spad, spins, m_final, s);
    launch_dense_energy_i8(*I, spad, R, E, I->ws.partial.p, s);
    launch_argmin(E, d.T0, (const int64_t *)w.runstat.p, R, N, I->wsum, res_dev, best_dev, I->tick_s, s);
    if (best_spins)
        launch_gather_best(spad, I->Ke, best_dev, N, best_spins, s);
    MARS_HIP(hipGetLastError());
    return MARS_OK;
}

static mars_status solve_dense(Instance *I, int R, const mars_schedule &sc, uint64_t seed, const float *m0,
                               const double *T0in, float *m_final, int8_t *spins, double *E, int8_t *best_spins,
                               int32_t *spl, int spl_cap, mars_result *res_dev, int32_t *best_dev, hipStream_t s)
{
    DenseRun d;
    mars_status st = dense_setup(I, R, sc, seed, m0, T0in, d, s);
    if (st != MARS_OK)
        return st;
    Workspace &w = I->ws;
    const int B = d.B, kmax = d.kmax, ldt = d.ldt, ldr = d.ldr, ldm = d.ldm;
    const std::vector<int> &pb = d.pb;
    const bool bf16 = d.bf16;
    const float gamma = d.gamma;
    float *table = d.table;
    int32_t *nlev = d.nlev;
    void *cur = d.Ma, *nxt = d.Mb;
    // bf16 tile variant: the autotuner's choice for this shape (timed on the
    // first phase at the first level, which the sweep then recomputes)
    int variant = 0;
    if (bf16 && kmax > 0)
        variant = bf16_phase_variant(*I, (const unsigned short *)cur, (unsigned short *)nxt, I->Np, R, pb[0], pb[1],
                                     table, gamma, s);
    float *phi = nullptr;
    if (d.seq) {
        if ((st = ensure(w.phi, sizeof(float) * (size_t)I->Np * ldm)) != MARS_OK)
            return st;
        phi = (float *)w.phi.p;
    }
    auto sweep = [&](const float *invT, const double *invT64, uint32_t *dmax) {
        for (int b = 0; b < B; ++b) {
            if (pb[b + 1] <= pb[b])
                continue;
            if (phi)
                launch_dense_seq_block(*I, (const float *)cur, (float *)nxt, phi, ldm, R, pb[b], pb[b + 1], invT,
                                       gamma, dmax, s);
            else if (bf16)
                launch_dense_phase_bf16(*I, (const unsigned short *)cur, (unsigned short *)nxt, I->Np, R, pb[b],
                                        pb[b + 1], invT, gamma, dmax, variant, s);
            else
                launch_dense_phase_f32(*I, (const float *)cur, (float *)nxt, ldm, R, pb[b], pb[b + 1], invT, invT64,
                                       gamma, dmax, s);
        }
        std::swap(cur, nxt);
    };
    int64_t *runstat = (int64_t *)w.runstat.p;
    if (sc.max_sweeps == 1) {
        for (int k = 0; k < kmax; ++k)
            sweep(table + (size_t)k * ldt, d.table64 ? d.table64 + (size_t)k * ldt : nullptr, nullptr);
        launch_dense_runstat(R, nlev, runstat, s);
        if (spl)
            launch_dense_spl_ones(R, nlev, spl, spl_cap, s);
    } else {
        // several sweeps per level: per-run level state advanced on the device
        // [ldr] floats, [ldr x 2] ints, then [ldr] doubles
        float *invT_cur = (float *)w.runstate.p;
        int32_t *state = (int32_t *)(invT_cur + ldr);
        double *invT64_cur = d.table64 ? (double *)(state + 2 * (size_t)ldr) : nullptr;
        uint32_t *dmax = (uint32_t *)w.dmax.p;
        launch_dense_advance_init(R, table, d.table64, nlev, invT_cur, invT64_cur, state, runstat, dmax, s);
        if (!d.seq && B <= kPaperMaxPhases) {
            // the whole anneal as one cooperative launch: nothing waits on the host
            const int ntr = (R + 127) / 128;
            if ((st = ensure(w.paper, sizeof(int32_t) * 4 * (size_t)ntr + 16)) != MARS_OK)
                return st;
            launch_fill_u32((uint32_t *)w.paper.p, 0u, 4 * (size_t)ntr + 4, s);
            DensePaperArgs a{};
            a.R = R;
            a.N = I->N;
            a.Np = I->Np;
            a.B = B;
            a.kmax = kmax;
            a.ldt = ldt;
            a.max_sweeps = sc.max_sweeps;
            a.spl_cap = spl_cap;
            a.ntr = ntr;
            a.d_min = sc.d_min;
            a.gamma = gamma;
            for (int b = 0; b <= B; ++b)
                a.pb[b] = pb[b];
            a.table = table;
            a.table64 = d.table64;
            a.nlev = nlev;
            a.invT_cur = invT_cur;
            a.invT64_cur = invT64_cur;
            a.state = state;
            a.runstat = runstat;
            a.dmax = dmax;
            a.spl = spl;
            int32_t *pw = (int32_t *)w.paper.p;
            a.cnt = pw;
            a.frozen = pw + 2 * (size_t)ntr;
            a.skip = pw + 3 * (size_t)ntr;
            a.active = (uint32_t *)(pw + 4 * (size_t)ntr);
            a.hhalf = I->has_h ? I->hhalf : nullptr;
            a.J = I->J;
            a.ldj = I->Np;
            a.ldm = ldm;
            a.Ma = (float *)d.Ma;
            a.Mb = (float *)d.Mb;
            a.Jb = I->Jbf;
            a.ldr = ldr;
            a.Ba = (unsigned short *)d.Ma;
            a.Bb = (unsigned short *)d.Mb;
            MARS_HIP(launch_dense_paper(a, bf16, s));
            cur = d.Ma;
        } else {
            uint32_t *active = (uint32_t *)w.flag.p;
            const long long cap = (long long)kmax * sc.max_sweeps + 1;
            long long done_sweeps = 0;
            const int chunk = 8;
            while (done_sweeps < cap) {
                for (int c = 0; c < chunk; ++c) {
                    sweep(invT_cur, invT64_cur, dmax);
                    launch_fill_u32(active, 0u, 1, s);
                    launch_dense_advance(R, table, d.table64, ldt, nlev, sc.max_sweeps, sc.d_min, invT_cur,
                                         invT64_cur, state, runstat, dmax, active, spl, spl_cap, s);
                    ++done_sweeps;
                }
                uint32_t h_active = 0;
                MARS_HIP(hipMemcpyAsync(&h_active, active, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
                MARS_HIP(hipStreamSynchronize(s));
                if (h_active == 0)
                    break;
            }
        }
    }
    return dense_finish(I, d, cur, m_final, spins, E, best_spins, res_dev, best_dev, s);
}

// A lattice/sparse solve in three parts, so that several solves can share
// the anneal's launch: the starting temperatures and the solve description
// (graph_pre), the anneal (launch_graph_solve, or a shared launch), then
// exact energies, best run and best spins (graph_post).
static mars_status graph_pre(Instance *I, int R, const mars_schedule &sc, uint64_t seed, const void *m0,
                             const double *T0in, void *m_final, int8_t *spins, double *E, int32_t *spl, int spl_cap,
                             GraphSolve *g, hipStream_t s)
{
    Workspace &w = I->ws;
    mars_status st;
    if ((st = ensure(w.T0, sizeof(double) * R)) || (st = ensure(w.runstat, sizeof(int64_t) * 4 * R)))
        return st;
    double *T0 = (double *)w.T0.p;
    launch_init_T0(seed, R, sc.T_lo, sc.T_hi, T0in, T0, s);
    g->sc = &sc;
    g->seed = seed;
    g->R = R;
    g->m0 = m0;
    g->T0 = T0;
    g->m_final = m_final;
    g->spins = spins;
    g->energies = E;
    g->runstat = (int64_t *)w.runstat.p;
    g->spl = spl;
    g->spl_cap = spl_cap;
    if (I->kind == KIND_LATTICE && graph_uses_global(*I, sc) && (st = lattice_sell(I)) != MARS_OK)
        return st;
    const size_t gbytes = graph_global_bytes(*I, sc, R);
    if (gbytes) {
        if ((st = ensure(w.gstate, gbytes)) != MARS_OK)
            return st;
        g->gscratch = w.gstate.p;
    }
    return MARS_OK;
}

static mars_status graph_post(Instance *I, const GraphSolve &g, int8_t *best_spins, mars_result *res_dev,
                              int32_t *best_dev, hipStream_t s)
{
    launch_graph_energy(*I, g.spins, g.R, g.energies, s);
    launch_argmin(g.energies, g.T0, g.runstat, g.R, I->N, I->wsum, res_dev, best_dev, I->tick_s, s);
    if (best_spins)
        launch_gather_best(g.spins, I->N, best_dev, I->N, best_spins, s);
    MARS_HIP(hipGetLastError());
    return MARS_OK;
}

static mars_status solve_graph(Instance *I, int R, const mars_schedule &sc, uint64_t seed, const void *m0,
                               const double *T0in, void *m_final, int8_t *spins, double *E, int8_t *best_spins,
                               int32_t *spl, int spl_cap, mars_result *res_dev, int32_t *best_dev, hipStream_t s)
{
    GraphSolve g;
    mars_status st = graph_pre(I, R, sc, seed, m0, T0in, m_final, spins, E, spl, spl_cap, &g, s);
    if (st != MARS_OK)
        return st;
    if ((st = launch_graph_solve(*I, g, s)) != MARS_OK)
        return st;
    return graph_post(I, g, best_spins, res_dev, best_dev, s);
}

// Stream ordering of the shared workspace: wait for the instance's previous
// work, then (after enqueueing) mark the new end of its work.
static mars_status order_begin(Instance *I, hipStream_t s)
{
    if (I->done_recorded)
        MARS_HIP(hipStreamWaitEvent(s, I->done_event, 0));
    return MARS_OK;
}

static mars_status order_end(Instance *I, hipStream_t s)
{
    MARS_HIP(hipEventRecord(I->done_event, s));
    I->done_recorded = true;
    return MARS_OK;
}

static mars_status solve_impl(Instance *I, int R, const mars_schedule *sched, uint64_t seed, const void *m0,
                              const double *T0, void *m_final, int8_t *spins, double *E, int8_t *best_spins,
                              int32_t *spl, int spl_cap, mars_result *res, hipStream_t s)
{
    if (R < 1)
        return set_error(MARS_E_ARG, "runs must be >= 1");
    if (R >= (1 << 30))
        return set_error(MARS_E_ARG, "runs must be < 2^30");
    if (spl && spl_cap < 1)
        return set_error(MARS_E_ARG, "sweeps_per_level needs level_cap >= 1");
    if (!spl)
        spl_cap = 0;
    mars_status st = check_schedule(sched, I->kind);
    if (st != MARS_OK)
        return st;
    MARS_HIP(hipSetDevice(I->device));
    if ((st = order_begin(I, s)) != MARS_OK)
        return st;
    Workspace &w = I->ws;
    const size_t spin_bytes = (size_t)R * I->N;
    if ((st = ensure(w.result, sizeof(mars_result) + 64)) != MARS_OK)
        return st;
    if (!spins && I->kind != KIND_DENSE) {
        // lattice/sparse solves always write every run's spins (energy and best-run input)
        if ((st = ensure(w.spins, spin_bytes)) != MARS_OK)
            return st;
        spins = (int8_t *)w.spins.p;
    }
    if (!E) {
        if ((st = ensure(w.energies, sizeof(double) * R)) != MARS_OK)
            return st;
        E = (double *)w.energies.p;
    }
    if (I->kind == KIND_DENSE && (st = ensure(w.partial, dense_energy_partial_bytes(*I, R))) != MARS_OK)
        return st;
    mars_result *res_dev = (mars_result *)w.result.p;
    int32_t *best_dev = result_best(res_dev);
    launch_stamp(result_stamp(res_dev), s);
    if (spl)
        launch_fill_u32(reinterpret_cast<uint32_t *>(spl), 0u, (size_t)R * spl_cap, s);
    if (I->kind == KIND_DENSE)
        st = solve_dense(I, R, *sched, seed, (const float *)m0, T0, (float *)m_final, spins, E, best_spins, spl,
                         spl_cap, res_dev, best_dev, s);
    else
        st = solve_graph(I, R, *sched, seed, m0, T0, m_final, spins, E, best_spins, spl, spl_cap, res_dev, best_dev,
                         s);
    if (st != MARS_OK)
        return st;
    if ((st = order_end(I, s)) != MARS_OK)
        return st;
    if (res) {
        mars_result tmp;
        MARS_HIP(hipMemcpyAsync(&tmp, res_dev, sizeof(mars_result), hipMemcpyDeviceToHost, s));
        MARS_HIP(hipStreamSynchronize(s));
        *res = tmp;
    }
    return MARS_OK;
}

// ---------------------------------------------------------------------------
// batched BF16 solver: members advance together, one launch per phase
// ---------------------------------------------------------------------------

struct BatchMember {
    Instance *I = nullptr;
    DenseRun d;
    int k = 0;      // next level (mirrors the device counter)
    int lslot = -1;  // index of the member's device level counter
    int64_t tag = 0;
    int8_t *best = nullptr;
    mars_result *res_pinned = nullptr;
    double *E = nullptr;
    mars_result *res_dev = nullptr;
    int32_t *best_dev = nullptr;
};

struct Batch {
    int device = 0;
    hipStream_t s = nullptr;
    std::mutex mu;
    std::vector<BatchMember> members;
    int *level = nullptr;  // [kMaxBatchMembers] device level counters
    uint32_t used = 0;     // level counters in use (bit mask)
    // graph of a whole step (sweeps x sweep), valid while the membership
    // and the sweep count are unchanged
    bool graphs = true;
    hipGraphExec_t exec = nullptr;
    int exec_sweeps = 0;
    // the whole step as one persistent cooperative launch (members with at
    // most four phases; otherwise the graph or eager path).  Off by default:
    // its grid barriers measured slower than replaying the per-phase launches
    bool persist = false;
};

static void drop_graph(Batch &b)
{
    if (b.exec)
        (void)hipGraphExecDestroy(b.exec);
    b.exec = nullptr;
    b.exec_sweeps = 0;
}

static void release_member(Batch &b, BatchMember &m)
{
    if (m.lslot >= 0)
        b.used &= ~(1u << m.lslot);
    std::lock_guard<std::mutex> lk(m.I->mu);
    m.I->in_batch = false;
}

// last level done: per-run statistics, rounding, exact energies, best run,
// copies to the caller's buffers
static mars_status finish_member(Batch &b, BatchMember &m)
{
    // the state after the last level is in Ma when kmax is even, else in Mb
    const void *cur = (m.d.kmax & 1) ? m.d.Mb : m.d.Ma;
    launch_dense_runstat(m.d.R, m.d.nlev, (int64_t *)m.I->ws.runstat.p, b.s);
    mars_status st = dense_finish(m.I, m.d, cur, nullptr, nullptr, m.E, m.best, m.res_dev, m.best_dev, b.s);
    if (st == MARS_OK && m.res_pinned) {
        hipError_t e = hipMemcpyAsync(m.res_pinned, m.res_dev, sizeof(mars_result), hipMemcpyDeviceToHost, b.s);
        if (e != hipSuccess)
            st = hip_error(e, "hipMemcpyAsync result");
    }
    if (st == MARS_OK)
        st = order_end(m.I, b.s);
    release_member(b, m);
    return st;
}

static mars_status batch_add(Batch &b, Instance *I, int R, const mars_schedule *sc, uint64_t seed, int64_t tag,
                             int8_t *best, mars_result *res_pinned)
{
    if (R < 1 || R >= (1 << 30))
        return set_error(MARS_E_ARG, "runs must be in [1, 2^30)");
    mars_status st = check_schedule(sc, I->kind);
    if (st != MARS_OK)
        return st;
    if (I->kind != KIND_DENSE || sc->precision != MARS_BF16 || sc->max_sweeps != 1)
        return set_error(MARS_E_UNSUPPORTED, "a batch holds dense instances solved in MARS_BF16 with max_sweeps 1");
    if (I->device != b.device)
        return set_error(MARS_E_UNSUPPORTED, "the instance lives on another device than the batch");
    if ((int)b.members.size() >= kMaxBatchMembers)
        return set_error(MARS_E_UNSUPPORTED, "the batch is full");
    {
        std::lock_guard<std::mutex> lk(I->mu);
        if (I->in_batch)
            return set_error(MARS_E_ARG, "the instance already belongs to a batch");
        I->in_batch = true;
    }
    BatchMember m;
    m.I = I;
    m.tag = tag;
    m.best = best;
    m.res_pinned = res_pinned;
    Workspace &w = I->ws;
    auto fail = [&](mars_status e) {
        release_member(b, m);
        return e;
    };
    if ((st = order_begin(I, b.s)) != MARS_OK)
        return fail(st);
    if ((st = ensure(w.result, sizeof(mars_result) + 64)) != MARS_OK ||
        (st = ensure(w.energies, sizeof(double) * R)) != MARS_OK ||
        (st = ensure(w.partial, dense_energy_partial_bytes(*I, R))) != MARS_OK)
        return fail(st);
    m.E = (double *)w.energies.p;
    m.res_dev = (mars_result *)w.result.p;
    m.best_dev = result_best(m.res_dev);
    launch_stamp(result_stamp(m.res_dev), b.s);
    if ((st = dense_setup(I, R, *sc, seed, nullptr, nullptr, m.d, b.s)) != MARS_OK)
        return fail(st);
    for (int q = 0; q < kMaxBatchMembers; ++q)
        if (!(b.used & (1u << q))) {
            m.lslot = q;
            break;
        }
    b.used |= 1u << m.lslot;
    launch_fill_u32(reinterpret_cast<uint32_t *>(b.level + m.lslot), 0u, 1, b.s);
    MARS_HIP(hipGetLastError());
    b.members.push_back(m);
    drop_graph(b);
    return MARS_OK;
}

static void describe(const Batch &b, BatchMemberDesc *dm)
{
    for (size_t i = 0; i < b.members.size(); ++i) {
        const BatchMember &m = b.members[i];
        dm[i].I = m.I;
        dm[i].Ma = (unsigned short *)m.d.Ma;
        dm[i].Mb = (unsigned short *)m.d.Mb;
        dm[i].table = m.d.table;
        dm[i].pb = m.d.pb.data();
        dm[i].R = m.d.R;
        dm[i].ldt = m.d.ldt;
        dm[i].kmax = m.d.kmax;
        dm[i].B = m.d.B;
        dm[i].lslot = m.lslot;
        dm[i].gamma = m.d.gamma;
    }
}

// Members past their last level leave, as long as the tag array has room
// (the others leave at a later call; their launches exit at once meanwhile).
static mars_status retire(Batch &b, int64_t *tags, int cap, int *n_fin)
{
    mars_status st = MARS_OK;
    for (size_t i = 0; i < b.members.size() && *n_fin < cap;) {
        BatchMember &m = b.members[i];
        if (m.k < m.d.kmax) {
            ++i;
            continue;
        }
        mars_status e = finish_member(b, m);
        if (e != MARS_OK && st == MARS_OK)
            st = e;
        tags[(*n_fin)++] = m.tag;
        b.members.erase(b.members.begin() + (long)i);
        drop_graph(b);
    }
    return st;
}

static mars_status batch_step(Batch &b, int sweeps, int64_t *tags, int cap, int *n_fin)
{
    *n_fin = 0;
    mars_status st = retire(b, tags, cap, n_fin);
    bool active = false;
    for (const BatchMember &m : b.members)
        active |= m.k < m.d.kmax;
    if (st != MARS_OK || sweeps == 0 || !active)
        return st;
    BatchMemberDesc dm[kMaxBatchMembers];
    describe(b, dm);
    const int n = (int)b.members.size();
    if (b.persist) {
        const hipError_t e = launch_batch_persistent(dm, n, b.level, sweeps, b.s);
        if (e == hipSuccess) {
            for (BatchMember &m : b.members)
                m.k = std::min(m.k + sweeps, m.d.kmax);
            return retire(b, tags, cap, n_fin);
        }
        if (e != hipErrorNotSupported)
            return hip_error(e, "persistent batch step");
        (void)hipGetLastError();  // too many phases: the step below
    }
    if (b.graphs && b.s) {
        // the whole step as one graph launch, captured once per membership
        if (!b.exec || b.exec_sweeps != sweeps) {
            drop_graph(b);
            hipGraph_t g = nullptr;
            MARS_HIP(hipStreamBeginCapture(b.s, hipStreamCaptureModeThreadLocal));
            hipError_t e = hipSuccess;
            for (int sw = 0; sw < sweeps && e == hipSuccess; ++sw)
                e = launch_batch_sweep(dm, n, b.level, b.s);
            const hipError_t e2 = hipStreamEndCapture(b.s, &g);
            if (e == hipSuccess)
                e = e2;
            if (e == hipSuccess)
                e = hipGraphInstantiate(&b.exec, g, nullptr, nullptr, 0);
            if (g)
                (void)hipGraphDestroy(g);
            if (e != hipSuccess) {
                b.exec = nullptr;
                return hip_error(e, "capturing the batch step");
            }
            b.exec_sweeps = sweeps;
        }
        MARS_HIP(hipGraphLaunch(b.exec, b.s));
        for (BatchMember &m : b.members)
            m.k = std::min(m.k + sweeps, m.d.kmax);
        return retire(b, tags, cap, n_fin);
    }
    // eager: one sweep at a time, members leave as soon as they finish
    for (int sw = 0; sw < sweeps && st == MARS_OK && !b.members.empty(); ++sw) {
        describe(b, dm);
        const int nm = (int)b.members.size();
        bool any = false;
        for (const BatchMember &m : b.members)
            any |= m.k < m.d.kmax;
        if (!any)
            break;
        hipError_t e = launch_batch_sweep(dm, nm, b.level, b.s);
        if (e != hipSuccess)
            return hip_error(e, "batch sweep launch");
        for (BatchMember &m : b.members)
            m.k = std::min(m.k + 1, m.d.kmax);
        st = retire(b, tags, cap, n_fin);
    }
    return st;
}

}  // namespace mars

// ---------------------------------------------------------------------------
// C interface
// ---------------------------------------------------------------------------

using namespace mars;

static mars_status finish_create(Instance *I, mars_status st, mars_instance **out)
{
    if (st != MARS_OK) {
        destroy_instance(I);
        return st;
    }
    *out = reinterpret_cast<mars_instance *>(I);
    return MARS_OK;
}

extern "C" {

mars_status mars_create(const float *J, const float *h, int32_t N, mars_instance **out)
{
    if (!out)
        return set_error(MARS_E_ARG, "out is NULL");
    *out = nullptr;
    if (!J || N < 1)
        return set_error(MARS_E_ARG, "need J != NULL and N >= 1");
    if (N > 200000)
        return set_error(MARS_E_UNSUPPORTED, "dense N above 200000");
    Instance *I = new (std::nothrow) Instance();
    if (!I)
        return set_error(MARS_E_OOM, "host allocation");
    mars_status st = start_instance(I);
    if (st == MARS_OK)
        st = create_dense(J, h, N, I);
    return finish_create(I, st, out);
}

mars_status mars_create_csr(int32_t N, const int32_t *rowptr, const int32_t *col, const int8_t *val, const float *h,
                            mars_instance **out)
{
    if (!out)
        return set_error(MARS_E_ARG, "out is NULL");
    *out = nullptr;
    if (N < 1 || !rowptr)
        return set_error(MARS_E_ARG, "need N >= 1 and rowptr != NULL");
    Instance *I = new (std::nothrow) Instance();
    if (!I)
        return set_error(MARS_E_OOM, "host allocation");
    mars_status st = start_instance(I);
    if (st == MARS_OK)
        st = create_csr(N, rowptr, col, val, h, I);
    return finish_create(I, st, out);
}

mars_status mars_create_lattice(int32_t dim, const int32_t *L, const int8_t *bond, const float *h,
                                mars_instance **out)
{
    if (!out)
        return set_error(MARS_E_ARG, "out is NULL");
    *out = nullptr;
    if ((dim != 2 && dim != 3) || !L || !bond)
        return set_error(MARS_E_ARG, "need dim in {2, 3}, L and bond");
    Instance *I = new (std::nothrow) Instance();
    if (!I)
        return set_error(MARS_E_OOM, "host allocation");
    mars_status st = start_instance(I);
    if (st == MARS_OK)
        st = create_lattice(dim, L, bond, h, I);
    return finish_create(I, st, out);
}

void mars_destroy(mars_instance *inst)
{
    if (inst)
        destroy_instance(reinterpret_cast<Instance *>(inst));
}

mars_status mars_describe(const mars_instance *inst, const mars_schedule *sched, int32_t *N, int32_t *phases)
{
    if (!inst)
        return set_error(MARS_E_ARG, "instance is NULL");
    const Instance *I = reinterpret_cast<const Instance *>(inst);
    if (N)
        *N = I->N;
    if (phases) {
        int p;
        if (sched && sched->update == MARS_JACOBI)
            p = 1;
        else if (sched && sched->update == MARS_SEQUENTIAL)
            p = I->N;
        else if (I->kind == KIND_DENSE)
            p = sched ? std::max(1, std::min(sched->phases, I->N)) : 1;
        else if (I->kind == KIND_LATTICE)
            p = 2;
        else
            p = I->ncolours;
        *phases = p;
    }
    return MARS_OK;
}

mars_status mars_solve_ex(mars_instance *inst, int32_t runs, const mars_schedule *sched, uint64_t seed,
                          const void *m0, const double *T0, double *T0_used, void *m_final, int8_t *spins,
                          double *energies, int8_t *best_spins, int32_t *sweeps_per_level, int32_t level_cap,
                          mars_result *res, void *stream)
{
    if (!inst)
        return set_error(MARS_E_ARG, "instance is NULL");
    Instance *I = reinterpret_cast<Instance *>(inst);
    std::lock_guard<std::mutex> lk(I->mu);
    if (I->in_batch)
        return set_error(MARS_E_ARG, "the instance belongs to a batch until its solve finishes");
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    mars_status st = solve_impl(I, runs, sched, seed, m0, T0, m_final, spins, energies, best_spins,
                                sweeps_per_level, level_cap, T0_used ? nullptr : res, s);
    if (st != MARS_OK || !T0_used)
        return st;
    MARS_HIP(hipMemcpyAsync(T0_used, I->ws.T0.p, sizeof(double) * runs, hipMemcpyDeviceToDevice, s));
    if (res) {
        mars_result tmp;
        MARS_HIP(hipMemcpyAsync(&tmp, I->ws.result.p, sizeof(mars_result), hipMemcpyDeviceToHost, s));
        MARS_HIP(hipStreamSynchronize(s));
        *res = tmp;
    }
    return MARS_OK;
}

mars_status mars_solve_async(mars_instance *inst, int32_t runs, const mars_schedule *sched, uint64_t seed,
                             const void *m0, const double *T0, void *m_final, int8_t *spins, double *energies,
                             int8_t *best_spins, mars_result *res_pinned, void *stream)
{
    if (!inst)
        return set_error(MARS_E_ARG, "instance is NULL");
    Instance *I = reinterpret_cast<Instance *>(inst);
    std::lock_guard<std::mutex> lk(I->mu);
    if (I->in_batch)
        return set_error(MARS_E_ARG, "the instance belongs to a batch until its solve finishes");
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    mars_status st =
        solve_impl(I, runs, sched, seed, m0, T0, m_final, spins, energies, best_spins, nullptr, 0, nullptr, s);
    if (st != MARS_OK || !res_pinned)
        return st;
    MARS_HIP(hipMemcpyAsync(res_pinned, I->ws.result.p, sizeof(mars_result), hipMemcpyDeviceToHost, s));
    return order_end(I, s);
}

mars_status mars_solve_group_async(int32_t count, mars_instance *const *insts, const int32_t *runs,
                                   const mars_schedule *scheds, const uint64_t *seeds, int8_t *const *best_spins,
                                   double *const *energies, mars_result *res_pinned, void *stream)
{
    if (count < 1 || count > GRAPH_GROUP_MAX)
        return set_error(MARS_E_ARG, "a group holds 1 to 64 solves");
    if (!insts || !runs || !scheds || !seeds)
        return set_error(MARS_E_ARG, "instances, runs, schedules and seeds must be given");
    std::vector<Instance *> L(count);
    for (int i = 0; i < count; ++i) {
        L[i] = reinterpret_cast<Instance *>(insts[i]);
        if (!L[i])
            return set_error(MARS_E_ARG, "instance is NULL");
        for (int j = 0; j < i; ++j)
            if (L[j] == L[i])
                return set_error(MARS_E_ARG, "an instance appears twice in a group (solves share its workspace)");
    }
    // lock every member (in address order, so that concurrent groups cannot
    // deadlock)
    std::vector<Instance *> order(L);
    std::sort(order.begin(), order.end());
    std::vector<std::unique_lock<std::mutex>> locks;
    for (Instance *I : order)
        locks.emplace_back(I->mu);
    for (int i = 0; i < count; ++i) {
        Instance *I = L[i];
        if (I->in_batch)
            return set_error(MARS_E_ARG, "the instance belongs to a batch until its solve finishes");
        if (I->kind == KIND_DENSE)
            return set_error(MARS_E_UNSUPPORTED, "groups hold lattice and sparse instances");
        if (I->device != L[0]->device)
            return set_error(MARS_E_ARG, "the instances of a group are on one device");
        if (runs[i] < 1 || runs[i] >= (1 << 30))
            return set_error(MARS_E_ARG, "runs must be >= 1 and < 2^30");
        mars_status st = check_schedule(&scheds[i], I->kind);
        if (st != MARS_OK)
            return st;
    }
    MARS_HIP(hipSetDevice(L[0]->device));
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    // members whose stream work has begun: on an error their instances still
    // record the end of what was enqueued, so later solves wait for it
    int begun = 0;
    auto enqueue = [&]() -> mars_status {
        std::vector<GraphSolve> G(count);
        std::vector<SparsePlan> P(count);
        mars_status st;
        for (int i = 0; i < count; ++i) {
            Instance *I = L[i];
            Workspace &w = I->ws;
            const int R = runs[i];
            if ((st = order_begin(I, s)) != MARS_OK)
                return st;
            begun = i + 1;
            if ((st = ensure(w.result, sizeof(mars_result) + 64)) != MARS_OK ||
                (st = ensure(w.spins, (size_t)R * I->N)) != MARS_OK)
                return st;
            double *E = energies ? energies[i] : nullptr;
            if (!E) {
                if ((st = ensure(w.energies, sizeof(double) * R)) != MARS_OK)
                    return st;
                E = (double *)w.energies.p;
            }
            launch_stamp(result_stamp((mars_result *)w.result.p), s);
            if ((st = graph_pre(I, R, scheds[i], seeds[i], nullptr, nullptr, nullptr, (int8_t *)w.spins.p, E, nullptr,
                                0, &G[i], s)) != MARS_OK)
                return st;
            // a sparse solve on the LDS-resident solver is planned; any other is
            // enqueued here
            if ((st = plan_graph_solve(*I, G[i], s, &P[i])) != MARS_OK)
                return st;
        }
        // one launch per kernel among the planned solves
        std::vector<bool> launched(count, false);
        for (int i = 0; i < count; ++i) {
            if (!P[i].fn || launched[i])
                continue;
            std::vector<SparsePlan> same{P[i]};
            launched[i] = true;
            for (int j = i + 1; j < count && P[i].gfn; ++j)
                if (!launched[j] && P[j].fn && P[j].gfn == P[i].gfn) {
                    same.push_back(P[j]);
                    launched[j] = true;
                }
            GraphGroup *hd = nullptr, *dd = nullptr;
            Instance *lead = L[i];
            if (same.size() > 1) {
                // the leader's descriptor: its previous copy must have run before
                // the host copy is rewritten
                if (lead->grp_pending)
                    MARS_HIP(hipEventSynchronize(lead->grp_event));
                if (!lead->grp_event)
                    MARS_HIP(hipEventCreateWithFlags(&lead->grp_event, hipEventDisableTiming));
                lead->grp_host.resize(sizeof(GraphGroup));
                if ((st = ensure(lead->ws.grp, sizeof(GraphGroup))) != MARS_OK)
                    return st;
                hd = reinterpret_cast<GraphGroup *>(lead->grp_host.data());
                dd = reinterpret_cast<GraphGroup *>(lead->ws.grp.p);
            }
            hipError_t e = launch_sparse_plans(same.data(), (int)same.size(), hd, dd, s);
            if (e != hipSuccess)
                return hip_error(e, "shared sparse solve launch");
            if (hd) {
                MARS_HIP(hipEventRecord(lead->grp_event, s));
                lead->grp_pending = true;
            }
        }
        for (int i = 0; i < count; ++i) {
            Instance *I = L[i];
            mars_result *res_dev = (mars_result *)I->ws.result.p;
            if ((st = graph_post(I, G[i], best_spins ? best_spins[i] : nullptr, res_dev, result_best(res_dev), s)) !=
                MARS_OK)
                return st;
            if (res_pinned)
                MARS_HIP(hipMemcpyAsync(&res_pinned[i], res_dev, sizeof(mars_result), hipMemcpyDeviceToHost, s));
            if ((st = order_end(I, s)) != MARS_OK)
                return st;
        }
        return MARS_OK;
    };
    const mars_status st = enqueue();
    if (st != MARS_OK) {
        for (int i = 0; i < begun; ++i)
            (void)order_end(L[i], s);
        return st;
    }
    return MARS_OK;
}

mars_status mars_solve(mars_instance *inst, int32_t runs, const mars_schedule *sched, uint64_t seed,
                       int8_t *best_spins, double *energies, mars_result *res)
{
    if (!inst)
        return set_error(MARS_E_ARG, "instance is NULL");
    Instance *I = reinterpret_cast<Instance *>(inst);
    std::lock_guard<std::mutex> lk(I->mu);
    if (I->in_batch)
        return set_error(MARS_E_ARG, "the instance belongs to a batch until its solve finishes");
    if (runs < 1)
        return set_error(MARS_E_ARG, "runs must be >= 1");
    mars_status st = check_schedule(sched, I->kind);
    if (st != MARS_OK)
        return st;
    MARS_HIP(hipSetDevice(I->device));
    hipStream_t s = I->own_stream;
    int8_t *dbest = nullptr;
    double *dE = nullptr;
    if (best_spins)
        MARS_HIP(hipMalloc(&dbest, (size_t)I->N));
    if (energies) {
        hipError_t e = hipMalloc(&dE, sizeof(double) * runs);
        if (e != hipSuccess) {
            if (dbest)
                (void)hipFree(dbest);
            return hip_error(e, "hipMalloc energies");
        }
    }
    mars_result tmp;
    st = solve_impl(I, runs, sched, seed, nullptr, nullptr, nullptr, nullptr, dE, dbest, nullptr, 0, &tmp, s);
    if (st == MARS_OK) {
        hipError_t e = hipSuccess;
        if (best_spins && e == hipSuccess)
            e = hipMemcpy(best_spins, dbest, (size_t)I->N, hipMemcpyDeviceToHost);
        if (energies && e == hipSuccess)
            e = hipMemcpy(energies, dE, sizeof(double) * runs, hipMemcpyDeviceToHost);
        if (e != hipSuccess)
            st = hip_error(e, "copy results");
        else if (res)
            *res = tmp;
    }
    if (dbest)
        (void)hipFree(dbest);
    if (dE)
        (void)hipFree(dE);
    return st;
}

mars_status mars_energy(mars_instance *inst, const int8_t *spins, int32_t R, double *energies, void *stream)
{
    if (!inst || !spins || !energies || R < 1)
        return set_error(MARS_E_ARG, "need instance, spins, energies and R >= 1");
    Instance *I = reinterpret_cast<Instance *>(inst);
    std::lock_guard<std::mutex> lk(I->mu);
    if (I->in_batch)
        return set_error(MARS_E_ARG, "the instance belongs to a batch until its solve finishes");
    MARS_HIP(hipSetDevice(I->device));
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    {
        mars_status st0 = order_begin(I, s);
        if (st0 != MARS_OK)
            return st0;
    }
    if (I->kind == KIND_DENSE) {
        mars_status st;
        if ((st = ensure(I->ws.partial, dense_energy_partial_bytes(*I, R))) != MARS_OK ||
            (st = ensure(I->ws.spad, dense_spin_operand_bytes(*I, R))) != MARS_OK)
            return st;
        launch_pad_spins(*I, spins, R, (int8_t *)I->ws.spad.p, s);
        launch_dense_energy_i8(*I, (const int8_t *)I->ws.spad.p, R, energies, I->ws.partial.p, s);
    } else {
        launch_graph_energy(*I, spins, R, energies, s);
    }
    MARS_HIP(hipGetLastError());
    return order_end(I, s);
}

// ---------------------------------------------------------------------------
// exact energies with no allocation: a fixed scratch array per device
// ---------------------------------------------------------------------------

// Scratch of mars_energy_noalloc (dense instances: the zero-padded run-major
// spin operand, then the per-tile 128-bit partial sums).  Each device the
// library runs on holds its own copy until the process ends.  In host code
// this name is not a device address: only the pointer returned by
// hipGetSymbolAddress for the current device is passed to kernels.
constexpr size_t kNoAllocScratchBytes = (size_t)32 << 20;
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

constexpr int kMaxScratchDevices = 64;
static std::mutex g_scratch_mu;
static void *g_scratch_ptr[kMaxScratchDevices];

// Device address of `scratch` on device dev (which must be current), looked up
// once per device.
static mars_status scratch_on_device(int dev, void **out)
{
    if (dev < 0 || dev >= kMaxScratchDevices)
        return set_error(MARS_E_DEVICE, "device index beyond the scratch table");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess)
            return hip_error(e, "hipGetSymbolAddress(scratch)");
        if (!p)
            return set_error(MARS_E_DEVICE, "hipGetSymbolAddress(scratch) returned no address");
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return MARS_OK;
}

mars_status mars_energy_noalloc(mars_instance *inst, const int8_t *spins, int32_t R, double *energies, void *stream)
{
    if (!inst || !spins || !energies || R < 1)
        return set_error(MARS_E_ARG, "need instance, spins, energies and R >= 1");
    Instance *I = reinterpret_cast<Instance *>(inst);
    std::lock_guard<std::mutex> lk(I->mu);
    if (I->in_batch)
        return set_error(MARS_E_ARG, "the instance belongs to a batch until its solve finishes");
    size_t spad_bytes = 0, part_bytes = 0;
    if (I->kind == KIND_DENSE) {
        spad_bytes = (dense_spin_operand_bytes(*I, R) + 255) & ~(size_t)255;
        part_bytes = dense_energy_partial_bytes(*I, R);
        if (spad_bytes + part_bytes > kNoAllocScratchBytes)
            return set_error(MARS_E_UNSUPPORTED,
                             "mars_energy_noalloc: " + std::to_string(R) + " spin vectors of N = " +
                                 std::to_string(I->N) + " need " + std::to_string(spad_bytes + part_bytes) +
                                 " bytes of scratch, more than its " + std::to_string(kNoAllocScratchBytes));
    }
    MARS_HIP(hipSetDevice(I->device));
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    mars_status st = order_begin(I, s);
    if (st != MARS_OK)
        return st;
    if (I->kind == KIND_DENSE) {
        void *base = nullptr;
        if ((st = scratch_on_device(I->device, &base)) != MARS_OK)
            return st;
        int8_t *spad = reinterpret_cast<int8_t *>(base);
        void *partial = reinterpret_cast<unsigned char *>(base) + spad_bytes;
        // every byte of both regions is written before it is read (padding
        // included), so nothing needs clearing between calls
        launch_pad_spins(*I, spins, R, spad, s);
        launch_dense_energy_i8(*I, spad, R, energies, partial, s);
    } else {
        launch_graph_energy(*I, spins, R, energies, s);
    }
    MARS_HIP(hipGetLastError());
    return order_end(I, s);
}

// Smallest and largest eigenvalues of the symmetric tridiagonal matrix with
// diagonal a[0..m) and off-diagonal b[0..m-1), by bisection on Sturm counts
// (count(x) = number of eigenvalues below x, from the signs of the pivots of
// T - x I).
static void tridiag_extremes(const std::vector<double> &a, const std::vector<double> &b, int m, double *lo_out,
                             double *hi_out)
{
    double lo = a[0], hi = a[0];
    for (int i = 0; i < m; ++i) {
        const double r = (i > 0 ? std::fabs(b[i - 1]) : 0.0) + (i + 1 < m ? std::fabs(b[i]) : 0.0);
        lo = std::min(lo, a[i] - r);
        hi = std::max(hi, a[i] + r);
    }
    const double pad = 1e-12 * std::max(1.0, std::max(std::fabs(lo), std::fabs(hi)));
    lo -= pad;
    hi += pad;
    auto count = [&](double x) {
        int c = 0;
        double d = 1.0;
        for (int i = 0; i < m; ++i) {
            d = a[i] - x - (i > 0 ? b[i - 1] * b[i - 1] / d : 0.0);
            if (d == 0.0)
                d = -1e-300;
            c += d < 0.0;
        }
        return c;
    };
    auto bisect = [&](int k) {  // the (k+1)-th smallest eigenvalue
        double l = lo, h = hi;
        for (int it = 0; it < 200 && h - l > 1e-15 * std::max(std::fabs(l), std::fabs(h)); ++it) {
            const double mid = 0.5 * (l + h);
            if (count(mid) > k)
                h = mid;
            else
                l = mid;
        }
        return 0.5 * (l + h);
    };
    *lo_out = bisect(0);
    *hi_out = bisect(m - 1);
}

mars_status mars_spectrum(mars_instance *inst, int32_t steps, uint64_t seed, double *lambda_min, double *lambda_max,
                          void *stream)
{
    if (!inst || !lambda_min || !lambda_max || steps < 1)
        return set_error(MARS_E_ARG, "need instance, outputs and steps >= 1");
    Instance *I = reinterpret_cast<Instance *>(inst);
    std::lock_guard<std::mutex> lk(I->mu);
    if (I->in_batch)
        return set_error(MARS_E_ARG, "the instance belongs to a batch until its solve finishes");
    MARS_HIP(hipSetDevice(I->device));
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    const int N = I->N;
    const int k = std::min(steps, N);
    mars_status st = order_begin(I, s);
    if (st != MARS_OK)
        return st;
    if ((st = ensure(I->ws.spec, sizeof(double) * (4 * (size_t)N + 2 * (size_t)k))) != MARS_OK)
        return st;
    double *vecs = (double *)I->ws.spec.p;
    double *alpha = vecs + 4 * (size_t)N, *beta = alpha + k;
    MARS_HIP(launch_spectrum_lanczos(*I, k, seed, vecs, alpha, beta, s));
    std::vector<double> a((size_t)k), b((size_t)k);
    MARS_HIP(hipMemcpyAsync(a.data(), alpha, sizeof(double) * k, hipMemcpyDeviceToHost, s));
    MARS_HIP(hipMemcpyAsync(b.data(), beta, sizeof(double) * k, hipMemcpyDeviceToHost, s));
    if ((st = order_end(I, s)) != MARS_OK)
        return st;
    MARS_HIP(hipStreamSynchronize(s));
    // the Krylov space closes at the first vanishing beta (an invariant subspace)
    double scale = 0.0;
    for (int j = 0; j < k; ++j)
        scale = std::max(scale, std::fabs(a[j]) + std::fabs(b[j]));
    int m = k;
    for (int j = 0; j + 1 < k; ++j)
        if (!(b[j] > 1e-13 * scale)) {
            m = j + 1;
            break;
        }
    for (int j = 0; j < m; ++j)
        if (!std::isfinite(a[j]) || !std::isfinite(b[j]))
            return set_error(MARS_E_DEVICE, "Lanczos coefficients are not finite");
    tridiag_extremes(a, b, m, lambda_min, lambda_max);
    return MARS_OK;
}

mars_status mars_auto_temperatures(mars_instance *inst, int32_t steps, uint64_t seed, mars_schedule *sched,
                                   void *stream)
{
    if (!sched)
        return set_error(MARS_E_ARG, "schedule is NULL");
    double lo = 0.0, hi = 0.0;
    mars_status st = mars_spectrum(inst, steps, seed, &lo, &hi, stream);
    if (st != MARS_OK)
        return st;
    // the scale: lambda_max, where the random start stops decaying; if J has
    // no positive eigenvalue, the spectral radius
    const double scale = hi > 0.0 ? hi : std::max(std::fabs(lo), std::fabs(hi));
    if (!(scale > 0.0) || !std::isfinite(scale))
        return set_error(MARS_E_ARG, "J has no nonzero eigenvalue: no temperature scale");
    sched->T_lo = 0.5 * scale;
    sched->T_hi = 1.5 * scale;
    sched->T_end = 0.005 * scale;
    return MARS_OK;
}

mars_status mars_batch_create(void *stream, mars_batch **out)
{
    if (!out)
        return set_error(MARS_E_ARG, "out is NULL");
    *out = nullptr;
    Batch *b = new (std::nothrow) Batch;
    if (!b)
        return set_error(MARS_E_OOM, "batch");
    hipError_t e = hipGetDevice(&b->device);
    if (e != hipSuccess) {
        delete b;
        return hip_error(e, "hipGetDevice");
    }
    b->s = reinterpret_cast<hipStream_t>(stream);
    e = hipMalloc(&b->level, sizeof(int) * kMaxBatchMembers);
    if (e != hipSuccess) {
        delete b;
        return hip_error(e, "hipMalloc batch level counters");
    }
    if (const char *f = std::getenv("MARS_BATCH_GRAPH"))
        b->graphs = std::atoi(f) != 0;
    if (const char *f = std::getenv("MARS_BATCH_PERSIST"))
        b->persist = std::atoi(f) != 0;
    *out = reinterpret_cast<mars_batch *>(b);
    return MARS_OK;
}

mars_status mars_batch_add(mars_batch *batch, mars_instance *inst, int32_t runs, const mars_schedule *sched,
                           uint64_t seed, int64_t tag, int8_t *best_spins, mars_result *res_pinned)
{
    if (!batch || !inst || !sched)
        return set_error(MARS_E_ARG, "need batch, instance and schedule");
    Batch *b = reinterpret_cast<Batch *>(batch);
    std::lock_guard<std::mutex> lk(b->mu);
    MARS_HIP(hipSetDevice(b->device));
    return batch_add(*b, reinterpret_cast<Instance *>(inst), runs, sched, seed, tag, best_spins, res_pinned);
}

mars_status mars_batch_step(mars_batch *batch, int32_t sweeps, int64_t *finished_tags, int32_t cap,
                            int32_t *n_finished, int32_t *n_active)
{
    if (!batch || !n_finished || !n_active || sweeps < 0 || cap < 0 || (cap > 0 && !finished_tags))
        return set_error(MARS_E_ARG, "need batch, counters, sweeps >= 0 and room for the tags");
    Batch *b = reinterpret_cast<Batch *>(batch);
    std::lock_guard<std::mutex> lk(b->mu);
    MARS_HIP(hipSetDevice(b->device));
    int nf = 0;
    mars_status st = batch_step(*b, sweeps, finished_tags, cap, &nf);
    *n_finished = nf;
    *n_active = (int32_t)b->members.size();
    return st;
}

void mars_batch_destroy(mars_batch *batch)
{
    if (!batch)
        return;
    Batch *b = reinterpret_cast<Batch *>(batch);
    {
        std::lock_guard<std::mutex> lk(b->mu);
        (void)hipSetDevice(b->device);
        (void)hipStreamSynchronize(b->s);
        for (BatchMember &m : b->members) {
            (void)order_end(m.I, b->s);
            release_member(*b, m);
        }
        b->members.clear();
        drop_graph(*b);
        (void)hipFree(b->level);
    }
    delete b;
}

const char *mars_status_str(mars_status s)
{
    switch (s) {
    case MARS_OK: return "ok";
    case MARS_E_ARG: return "invalid argument";
    case MARS_E_ASYMMETRIC: return "couplings not symmetric";
    case MARS_E_DIAGONAL: return "nonzero diagonal coupling";
    case MARS_E_NONFINITE: return "non-finite input";
    case MARS_E_RANGE: return "exact energy out of range";
    case MARS_E_OOM: return "out of device memory";
    case MARS_E_DEVICE: return "device error";
    case MARS_E_UNSUPPORTED: return "unsupported";
    }
    return "unknown status";
}

const char *mars_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"
