// Internal declarations of the MARS HIP library (not part of the public ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/mars.h"
#include "common_device.h"

namespace mars {

enum Kind { KIND_DENSE = 0, KIND_CSR = 1, KIND_LATTICE = 2 };

constexpr int SELL_H = 8;  // slots per slice of the sparse solver's layout
constexpr int SELL_W = 4;  // slice widths are padded to a multiple of this
constexpr int SPARSE_LPS_MAX = 4;  // most lanes the sparse solver splits one slot's row over
constexpr int SPARSE_READ_AHEAD = 2;  // entry groups of a long row a lane reads ahead
constexpr size_t RUN_AREA_MAX = 96;  // LDS bytes reserved per run for its level state
// LDS level table of an LDS-resident solver's block (geometric schedules):
// 1/T in fp64 for every run and level it visits, then the same in fp32,
// after the runs' level records (8-byte aligned)
inline size_t level_table_bytes(int rpw, int ttab)
{
    return ttab > 0 ? 8 + (size_t)rpw * ttab * 12 : 0;
}
// the table of n levels is kept where it fits the LDS budget without
// lowering the number of the launch's workgroups resident on a CU (160 KB of
// LDS and 32 waves per CU, blocks spread over 256 CUs); 0: walk the levels
inline int level_table_fit(int n, int rpw, size_t base_lds, int threads, long long blocks)
{
    if (n <= 0)
        return 0;
    const size_t with = base_lds + level_table_bytes(rpw, n);
    if (with > 160 * 1024 - 1024)
        return 0;
    auto resident = [&](size_t bytes) {
        long long r = (long long)((160 * 1024) / bytes);
        r = std::min(r, (long long)(32 / ((threads + 63) / 64)));
        return std::min(r, (blocks + 255) / 256);
    };
    return resident(with) >= resident(base_lds) ? n : 0;
}

// Device buffer owned by an instance; grows on demand, freed on destroy.
struct DevBuf {
    void *p = nullptr;
    size_t bytes = 0;
};

struct Workspace {
    DevBuf Ma, Mb;          // dense state ping-pong buffers [Np x ldm]
    DevBuf invT;            // per-level per-run inverse temperatures
    DevBuf invT64;          // the same in fp64 (dense fp32 form)
    DevBuf T0;              // [R] double
    DevBuf nlev;            // [R] int32 levels in range per run
    DevBuf runstat;         // [R x 4] int64: sweeps, levels, cap hits, spare
    DevBuf dmax;            // [R] uint32 (bit pattern of a non-negative float)
    DevBuf spins;           // [R x N] int8 (lattice/sparse)
    DevBuf spad;            // dense: [ldr x Ke] int8 zero-padded run-major spins
    DevBuf energies;        // [R] double
    DevBuf partial;         // dense energy partial sums
    DevBuf result;          // device mars_result + best index
    DevBuf runstate;        // paper mode per-run level state
    DevBuf flag;            // small counters
    DevBuf spec;            // Lanczos vectors and coefficients
    DevBuf phi;             // fields of a sequential block
    DevBuf paper;           // block counters of the one-launch paper schedule
    DevBuf gstate;          // sparse instances beyond LDS: state and per-run records in device memory
    DevBuf grp;             // descriptor of a shared sparse launch (GraphGroup)
};

struct Instance {
    int kind = KIND_DENSE;
    int N = 0;
    int device = 0;
    // fixed point used for exact energies: every coupling and field value is
    // an integer multiple of 2^emin
    int emin = 0;
    double wsum = 0.0;      // sum_{i != j} -J_ij (for the cut value)
    bool has_h = false;
    // dense
    int Np = 0;             // padded dimension of J and of the state rows
    float *J = nullptr;     // [Np x Np] zero padded
    unsigned short *Jbf = nullptr;  // [Np x Np] bf16 copy (created on the first bf16 solve)
    int64_t *Jfix = nullptr;  // [N x N] fixed-point couplings (create-time only)
    int8_t *Jlimb = nullptr;  // [nlimb x Me x Ke] balanced base-256 digits of Jfix
    int nlimb = 0;
    int Me = 0, Ke = 0;       // padded digit-matrix rows / columns (multiples of 128)
    float *hhalf = nullptr;   // [Np] h/2 (fp32), zero padded
    double *hhalf64 = nullptr;  // [N] h/2 (fp64)
    int64_t *hfix = nullptr;  // [N] fixed-point field
    // csr
    int nnz = 0;
    int32_t *rowptr = nullptr;
    uint32_t *colval = nullptr;   // (col << 8) | uint8(val)
    int ncolours = 0;
    int maxdeg = 0;
    // sliced-ELL copy used by the solver: vertices relabelled into slots,
    // colour class by colour class, each class sorted by degree (descending)
    // and padded to a multiple of SELL_H slots; slice s (SELL_H consecutive
    // slots) holds width w_s = its largest degree rounded up to a multiple
    // of SELL_W and entries
    // colsell[off_s + ((j / SELL_W) * SELL_H + slot % SELL_H) * SELL_W + j % SELL_W],
    // j < w_s (a slot's group of SELL_W entries is 16 contiguous bytes, and
    // the SELL_H slots of a slice read 128 contiguous bytes per group), each
    // (neighbour slot) | (uint8(weight) << 24), or, when every weight is
    // +-1 (unit), (neighbour slot) | (weight < 0) << 31; a missing entry
    // names the all-zero row nslot with weight +1; SPARSE_READ_AHEAD x
    // SPARSE_LPS_MAX groups of such entries follow the last slice
    int nslot = 0;
    bool unit = false;            // every |weight| == 1
    int32_t *perm = nullptr;      // [nslot] slot -> vertex, -1 for padding
    int32_t *sl_meta = nullptr;   // [2 x nslot / SELL_H] (off_s, w_s)
    uint32_t *colsell = nullptr;
    int32_t *cls = nullptr;       // [2 x ncolours] (first slot, vertex count)
    std::vector<int32_t> h_cls;
    float *hperm = nullptr;       // [nslot] h/2 by slot (fp32), 0 on padding
    double *hperm64 = nullptr;    // [nslot] h/2 by slot (fp64)
    // lattice
    int dim = 0;
    int L[3] = {1, 1, 1};
    uint8_t *bondbits = nullptr;  // [N]: bit 2a set if J(v, v+e_a) < 0, bit 2a+1 if J(v, v-e_a) < 0
    // [2N] (the second half repeats the first): per site the bond signs as
    // fp16 sign bits, bit 15 - a for J(v, v+e_a) < 0, bit 31 - a for J(v, v-e_a) < 0
    uint32_t *bondsgn = nullptr;
    // runtime
    hipStream_t own_stream = nullptr;
    // the instance's workspace is reused by every solve: a solve on another
    // stream first waits for the previous one (recorded in done_event)
    hipEvent_t done_event = nullptr;
    bool done_recorded = false;
    bool in_batch = false;  // owned by a batch until its member finishes
    double tick_s = 0.0;    // seconds per tick of the device's constant-rate clock
    // lattice: the bonds and field as given (host), from which the sparse
    // encodings are built when a solve needs the solver beyond LDS
    std::vector<int8_t> lat_bond;
    std::vector<float> lat_h;
    bool lat_sell = false;
    // descriptor of a shared sparse launch this instance led: host copy (kept
    // until its copy to the device has run, grp_event) and device copy
    std::vector<unsigned char> grp_host;
    hipEvent_t grp_event = nullptr;
    bool grp_pending = false;
    Workspace ws;
    std::mutex mu;
};

// ---- error reporting -------------------------------------------------------
mars_status set_error(mars_status s, const std::string &msg);
mars_status hip_error(hipError_t e, const char *what);
mars_status ensure(DevBuf &b, size_t bytes);

#define MARS_HIP(call)                                   \
    do {                                                 \
        hipError_t e_ = (call);                          \
        if (e_ != hipSuccess) return hip_error(e_, #call); \
    } while (0)

// ---- launchers (each defined next to its kernels) -------------------------
// common
void launch_fill_u32(uint32_t *p, uint32_t v, size_t n, hipStream_t s);
void launch_init_T0(uint64_t seed, int R, double T_lo, double T_hi, const double *T0_in, double *T0_out,
                    hipStream_t s);
void launch_level_table(const mars_schedule &sc, int R, const double *T0, int kmax, int ldt, float *invT32,
                        double *invT64, int32_t *nlev, hipStream_t s);
// The device result area of a solve: mars_result, then the device clock at
// the start of the solve (uint64, written by launch_stamp), then the best run
// index (int32 at +16).
__host__ __device__ inline uint64_t *result_stamp(mars_result *res_dev) { return reinterpret_cast<uint64_t *>(res_dev + 1); }
inline int32_t *result_best(mars_result *res_dev)
{
    return reinterpret_cast<int32_t *>(reinterpret_cast<char *>(res_dev + 1) + 16);
}
void launch_stamp(uint64_t *slot, hipStream_t s);
// best of runs into res_dev; res_dev->seconds = device clock now minus
// *result_stamp(res_dev), times tick_s
void launch_argmin(const double *E, const double *T0, const int64_t *runstat, int R, int N, double wsum,
                   mars_result *res_dev, int32_t *best_dev, double tick_s, hipStream_t s);
void launch_gather_best(const int8_t *spins, int ld, const int32_t *best_dev, int N, int8_t *out, hipStream_t s);
void launch_graph_energy(const Instance &I, const int8_t *spins, int R, double *E, hipStream_t s);
// dense exact energy on the int8 matrix cores (k_energy.hip)
void launch_dense_limbs(const Instance &I, hipStream_t s);
size_t dense_spin_operand_bytes(const Instance &I, int R);
void launch_pad_spins(const Instance &I, const int8_t *spins, int R, int8_t *Spad, hipStream_t s);
size_t dense_energy_partial_bytes(const Instance &I, int R);
void launch_dense_energy_i8(const Instance &I, const int8_t *Spad, int R, double *E, void *partial, hipStream_t s);

// dense
void launch_dense_init_state(uint64_t seed, int N, int R, int ldm, const float *m0, float *M, hipStream_t s);
// sequential update: blocks of SEQ_NB spins, each a field product into phi
// ([Np x ldm]) followed by an in-block pass in index order
constexpr int SEQ_NB = 64;
void launch_dense_seq_block(const Instance &I, const float *Mold, float *Mnew, float *phi, int ldm, int R, int p0,
                            int p1, const float *invT, float gamma, uint32_t *dmax, hipStream_t s);
// invT64 (or null): fp64 1/T of the runs, then the update is evaluated in fp64
void launch_dense_phase_f32(const Instance &I, const float *Mold, float *Mnew, int ldm, int R, int p0, int p1,
                            const float *invT, const double *invT64, float gamma, uint32_t *dmax, hipStream_t s);
void launch_dense_round(const float *M, int ldm, int N, int R, int Ke, int8_t *spad, int8_t *spins, float *m_final,
                        hipStream_t s);
void launch_dense_runstat(int R, const int32_t *nlev, int64_t *runstat, hipStream_t s);
void launch_dense_fixpoint(const Instance &I, hipStream_t s);
// table64 / invT64_cur: the fp64 copies (both null when the form has none)
void launch_dense_advance_init(int R, const float *table, const double *table64, const int32_t *nlev,
                               float *invT_cur, double *invT64_cur, int32_t *state, int64_t *runstat, uint32_t *dmax,
                               hipStream_t s);
void launch_dense_advance(int R, const float *table, const double *table64, int ldt, const int32_t *nlev,
                          int max_sweeps, double d_min, float *invT_cur, double *invT64_cur, int32_t *state,
                          int64_t *runstat, uint32_t *dmax, uint32_t *active, int32_t *spl, int cap, hipStream_t s);
// one sweep per level: spl[r * cap + k] = (k < nlev[r])
void launch_dense_spl_ones(int R, const int32_t *nlev, int32_t *spl, int cap, hipStream_t s);

// The paper's scheduler (several sweeps per level) on dense instances as one
// cooperative launch (k_dense_paper.hip): phases, the level advance of every
// run and grid barriers between them, until no run anneals; the final state
// ends in buffer A (Ma / Ba).  Phase bounds travel in the arguments.
constexpr int kPaperMaxPhases = 64;
struct DensePaperArgs {
    int R, N, Np, B, kmax, ldt, max_sweeps, spl_cap, ntr;  // ntr: 128-run blocks
    double d_min;
    float gamma;
    int pb[kPaperMaxPhases + 1];
    const float *table;
    const double *table64;  // fp32 form: fp64 copy of the table (or null)
    const int32_t *nlev;
    float *invT_cur;
    double *invT64_cur;
    int32_t *state;
    int64_t *runstat;
    uint32_t *dmax;
    int32_t *spl;
    int32_t *cnt;      // [2 x ntr] active runs per 128-run block, by sweep parity
    int32_t *frozen;   // [ntr] advances in a row with no active run in the block
    int32_t *skip;     // [ntr] the block is left out of the products
    uint32_t *active;  // [2] runs still annealing, by sweep parity
    const float *hhalf;
    // fp32 form: state [Np x ldm]
    const float *J;
    int ldj, ldm;
    float *Ma, *Mb;
    // bf16 form: state [ldr x Np]
    const unsigned short *Jb;
    int ldr;
    unsigned short *Ba, *Bb;
};
hipError_t launch_dense_paper(const DensePaperArgs &a, bool bf16, hipStream_t s);

// dense, bf16 form (k_dense_bf16.hip)
mars_status ensure_bf16_couplings(Instance &I, hipStream_t s);
int bf16_state_rows(int R);
void launch_bf16_init_state(uint64_t seed, int N, int R, int ldk, const float *m0, unsigned short *MT, hipStream_t s);
void launch_dense_phase_bf16(const Instance &I, const unsigned short *Mold, unsigned short *Mnew, int ldk, int R,
                             int p0, int p1, const float *invT, float gamma, uint32_t *dmax, int variant,
                             hipStream_t s);
int bf16_phase_variant(const Instance &I, const unsigned short *Mold, unsigned short *Mnew, int ldk, int R, int p0,
                       int p1, const float *invT, float gamma, hipStream_t s);
// Lanczos iteration on J (steps <= N): vecs holds 4 N doubles; the
// recurrence coefficients alpha[steps], beta[steps] stay on the device.
hipError_t launch_spectrum_lanczos(const Instance &I, int steps, uint64_t seed, double *vecs, double *alpha,
                                   double *beta, hipStream_t s);
// one member of the batched solver's launches
struct BatchMemberDesc {
    const Instance *I;
    unsigned short *Ma, *Mb;  // state buffers (level k reads Ma if k is even)
    const float *table;       // 1/T: row k at table + k * ldt
    const int *pb;            // B + 1 phase bounds
    int R, ldt, kmax, B, lslot;  // lslot: the member's level counter
    float gamma;
};
constexpr int kMaxBatchMembers = 16;
// One sweep of the members: one launch per phase index over the tiles of
// every member that has that phase, then the level advance (level[lslot] += 1
// below kmax).  Kernel launches only, so it can be captured in a graph.
hipError_t launch_batch_sweep(const BatchMemberDesc *m, int n, int *level, hipStream_t s);
// `sweeps` sweeps of the members as one persistent cooperative launch (grid
// barriers between phases, the level counters advanced on the device),
// bitwise the same as that many launch_batch_sweep calls;
// hipErrorNotSupported when a member has more phases than the launch's
// descriptors hold.
hipError_t launch_batch_persistent(const BatchMemberDesc *m, int n, int *level, int sweeps, hipStream_t s);
void launch_bf16_round(const unsigned short *MT, int ldk, int N, int R, int Ke, int8_t *spad, int8_t *spins,
                       float *m_final, hipStream_t s);

// dense solve stages (runtime.hip), shared by single solves and the batch
struct DenseRun {
    int R = 0, ldm = 0, ldr = 0, ldt = 0, kmax = 0, B = 0;
    std::vector<int> pb;  // phase bounds [B + 1]
    bool bf16 = false;
    bool seq = false;  // sequential update: blocks of SEQ_NB spins
    float gamma = 1.0f;
    double *T0 = nullptr;
    float *table = nullptr;  // [kmax x ldt] 1/T per level and run, -1 past a run's levels
    double *table64 = nullptr;  // the same in fp64 (fp32 form; null for bf16 and sequential)
    int32_t *nlev = nullptr;
    void *Ma = nullptr, *Mb = nullptr;  // state ping-pong buffers (Ma holds the initial state)
};
mars_status dense_setup(Instance *I, int R, const mars_schedule &sc, uint64_t seed, const float *m0,
                        const double *T0in, DenseRun &d, hipStream_t s);
mars_status dense_finish(Instance *I, const DenseRun &d, const void *cur, float *m_final, int8_t *spins, double *E,
                         int8_t *best_spins, mars_result *res_dev, int32_t *best_dev, hipStream_t s);

// graph (lattice and csr): the whole anneal of a block of runs in LDS
struct GraphSolve {
    const mars_schedule *sc;
    uint64_t seed;
    int R;
    const void *m0;
    const double *T0;      // starting temperatures, filled before the launch
    void *m_final;
    int8_t *spins;
    double *energies;
    int64_t *runstat;      // [R x 4]
    int32_t *spl = nullptr;  // [R x spl_cap] sweeps per visited level (zero filled), or null
    int spl_cap = 0;
    void *gscratch = nullptr;  // graph_global_bytes() of device memory, or null
};
mars_status launch_graph_solve(const Instance &I, const GraphSolve &g, hipStream_t s);
struct SparsePlan;
// as launch_graph_solve, but a sparse solve on the LDS-resident solver is
// planned (*plan, plan->fn set) instead of enqueued, for a shared launch;
// other solves are enqueued (plan->fn null)
mars_status plan_graph_solve(const Instance &I, const GraphSolve &g, hipStream_t s, SparsePlan *plan);
// whether a lattice/sparse solve runs with its state in device memory (one
// run's state does not fit in LDS, or MARS_GRAPH_GLOBAL=1); a lattice then
// runs on the sparse solver over its sparse encodings (built on first use)
bool graph_uses_global(const Instance &I, const mars_schedule &sc);
// bytes of device memory that solve needs (0: the LDS-resident solvers take
// it); for a lattice the sparse encodings must exist
size_t graph_global_bytes(const Instance &I, const mars_schedule &sc, int R);

// kernel arguments of the lattice / sparse solvers
struct GraphArgs {
    int N;
    // csr
    const int32_t *rowptr;
    const uint32_t *colval;
    int nphase;
    // sliced ELL (see Instance)
    int nslot;
    const int32_t *perm;
    const int32_t *sl_meta;
    const uint32_t *colsell;
    const int32_t *cls;
    int long_rows;  // sparse: average degree >= 16, entry groups are read ahead
    int ttab;       // geometric schedules: levels in the block's LDS level table (0: none)
    int fixed_sweeps;  // > 0: every live run anneals exactly this many sweeps (geometric, one per level)
    // lattice
    int dim, L0, L1, L2;
    const uint8_t *bondbits;
    const uint32_t *bondsgn;
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
    int32_t *spl;  // [R x spl_cap] sweeps per visited level, or null
    int spl_cap;
};

hipError_t launch_lattice_solve(const GraphArgs &a, int esz, int rpw, bool jac, bool trackd, hipStream_t s);

// Several sparse solves in one launch of the LDS-resident solver: instance k
// owns blocks first[k] .. first[k + 1] - 1 (block index within it = block -
// first[k]) with its own arguments and runs per workgroup (2^lg[k]).
constexpr int GRAPH_GROUP_MAX = 64;
struct GraphGroup {
    int count;
    int first[GRAPH_GROUP_MAX + 1];
    int lg[GRAPH_GROUP_MAX];
    GraphArgs args[GRAPH_GROUP_MAX];
};
// How one sparse solve launches the LDS-resident solver: the kernel
// (instantiation), its arguments, and the launch shape.  Solves whose group
// instantiations agree can share one launch (the block shape is the largest of theirs: the
// kernel derives its slots in flight from it; the LDS size the largest).
struct SparsePlan {
    const void *fn = nullptr;   // the kernel of the solve alone
    const void *gfn = nullptr;  // its group instantiation, or null (then it launches alone)
    GraphArgs args;
    int lg = 0, blocks = 0, threads = 0;
    size_t lds = 0;
};
hipError_t plan_sparse_solve(const GraphArgs &a, int esz, int rpw, int Tq, int vec, int lps, bool jac, bool trackd,
                             bool unit, SparsePlan *plan);
hipError_t launch_sparse_plans(const SparsePlan *plans, int n, GraphGroup *host_desc, GraphGroup *dev_desc,
                               hipStream_t s);

// the sparse solver with its state in device memory (k_sparse_global.hip)
struct SparseGlobalArgs {
    GraphArgs a;
    void *m, *m2;       // [nslot + 1 rows x ldr] magnetisations (m2: synchronous update only)
    int ldr;            // row length: runs rounded up to the run group
    int ngc;            // run groups per chunk of a phase's items
    void *rs;           // [ldr] per-run level state
    void *tscale;       // [ldr] per-run factor of the update (run_tscale)
    int32_t *rdone;     // [ldr] run finished
    uint32_t *flag;     // [ldr] a change of the sweep reached d_min
    uint32_t *live;     // [2] alternating words: some run still anneals
    int jac, unit;
};
hipError_t launch_sparse_global(const SparseGlobalArgs &a, int esz, hipStream_t s);
hipError_t launch_sparse_solve(const GraphArgs &a, int esz, int rpw, int Tq, int vec, int lps, bool jac,
                               bool trackd, bool unit, hipStream_t s);

}  // namespace mars
