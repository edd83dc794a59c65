/*
 * MARS CPU oracle -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, FP64 implementation of Mean-field Annealing from a Random
 * State (MARS; Yavorsky, Markovich, Polyakov, Rubtsov, arXiv:1907.05124),
 * written from the paper to check the GPU library against.  Only the test
 * suite, the smoke check and the benchmark's CPU-baseline leg may load it.
 * It shares no code with the GPU library.
 *
 * Conventions (readings of the paper where it is silent, ambiguous or
 * garbled; each states the passage it follows):
 *
 *  - Energy (section "Ising Spin Glass Model", eq. (2), ordered-pair double
 *    sum over j != i), written with the minimisation sign used by the library
 *    interface:  E(s) = - sum_i sum_{j != i} J_ij s_i s_j - sum_i h_i s_i.
 *    The paper's own Hamiltonian is the same expression with J -> -J, h -> -h.
 *  - Local field and update (section "Mean-field Annealing from Random
 *    State", Algorithm 1 and the prose before it): Phi_i = sum_j J_ij m_j +
 *    h_i/2 and m_i <- tanh(Phi_i / T).  With J = -J_paper this is the
 *    paper's s_i <- -tanh(Phi_i^paper / T); the paper drops h, and h/2 is the
 *    mean-field derivative of E at the paper's temperature scale.
 *  - Update order: the spins are split into phases that are updated one after
 *    the other inside a sweep; inside a phase every spin sees the magnetisation
 *    as it was when the phase began.  Dense: B contiguous row blocks
 *    [floor(bN/B), floor((b+1)N/B)).  Lattice: checkerboard by parity of the
 *    coordinate sum.  Sparse: greedy colouring in index order.  "jacobi" is a
 *    single phase holding every spin (the synchronous reading of Algorithm 1).
 *  - Convergence: a level ends when the largest change of a sweep,
 *    d = max_i |m_i^new - m_i^old|, drops below d_min, or after max_sweeps
 *    sweeps (Algorithm 1's "repeat ... until" read as "until d < d_min").
 *  - Temperatures: linear (paper): T <- T0, then repeatedly T <- T - c_step,
 *    relaxing at each T > 0 (the decrement comes before relaxing, as in
 *    Algorithm 1).  Geometric: K levels T_k = T0 exp((k/(K-1)) ln(T_end/T0)).
 *  - Initial state and starting temperature (Algorithm 1, "rand(-1,1)"; the
 *    paper draws the starting temperature at random in a range): a
 *    counter-based generator, the SplitMix64 output function of
 *    Steele, Lea & Flood (OOPSLA 2014) applied to seed + (c+1)*0x9E3779B97F4A7C15
 *    with counter c = (stream << 62) | (run << 32) | spin.  Stream 0 gives
 *    m0 = (2k + 1 - 2^24) 2^-24 and stream 1 gives
 *    T0 = T_lo + (T_hi - T_lo) (k 2^-24), k = the top 24 bits of the output.
 *  - Rounding: s_i = +1 if m_i >= 0 else -1.
 *  - Best run: smallest exact energy, ties to the lowest run index; the hit
 *    count is the number of runs whose energy equals the best (section
 *    "Ground state of Sherrington-Kirkpatrick spin-glass", success
 *    probability P = hits / runs).
 *  - Exact energy: every term +-J_ij, +-h_i is a double; their sum is formed
 *    exactly in a long fixed-point accumulator and rounded once to double
 *    (round to nearest, ties to even).
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_DENSE 0
#define ORC_CSR 1
#define ORC_LATTICE 2

#define ORC_GEOMETRIC 0
#define ORC_LINEAR 1

#define ORC_PHASED 0
#define ORC_JACOBI 1

typedef struct {
    int kind; /* ORC_DENSE | ORC_CSR | ORC_LATTICE */
    int N;
    const float *J; /* dense: N*N row-major */
    const int32_t *rowptr; /* csr */
    const int32_t *col;
    const int8_t *val;
    int dim; /* lattice */
    int L[3];
    const int8_t *bond; /* lattice: dim*N, bond[a*N+i] couples i and i+e_a */
    const float *h; /* N or NULL */
} orc_instance;

typedef struct {
    int kind; /* ORC_GEOMETRIC | ORC_LINEAR */
    double T_lo, T_hi, T_end, c_step;
    int steps; /* geometric: number of levels */
    int max_sweeps;
    double d_min;
    int update; /* ORC_PHASED | ORC_JACOBI */
    int phases; /* dense: number of row blocks */
    double damping;
    int first_level; /* relax levels [first_level, first_level + level_count) */
    int level_count; /* < 0: to the end of the schedule */
} orc_schedule;

/* ------------------------------------------------------------------------ */
/* counter-based generator                                                   */
/* ------------------------------------------------------------------------ */

uint64_t orc_splitmix64(uint64_t seed, uint64_t counter)
{
    uint64_t z = seed + (counter + 1u) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

double orc_initial_m(uint64_t seed, int64_t run, int64_t spin)
{
    uint64_t c = ((uint64_t)run << 32) | (uint64_t)spin;
    uint64_t k = orc_splitmix64(seed, c) >> 40; /* top 24 bits */
    return ldexp((double)(2 * (int64_t)k + 1 - (1 << 24)), -24);
}

double orc_initial_T(uint64_t seed, int64_t run, double T_lo, double T_hi)
{
    uint64_t c = (1ull << 62) | ((uint64_t)run << 32);
    uint64_t k = orc_splitmix64(seed, c) >> 40;
    double u = ldexp((double)k, -24);
    double w = T_hi - T_lo;
    double t = w * u;
    return T_lo + t;
}

/* ------------------------------------------------------------------------ */
/* exact sums: a fixed-point accumulator over the whole double range         */
/* ------------------------------------------------------------------------ */

/* bit b of the accumulator has weight 2^(b - ACC_BIAS); digits hold 32 bits
 * each in an int64 (so up to 2^30 additions fit before carries are needed). */
#define ACC_BIAS 1140
#define ACC_DIGITS 80

typedef struct {
    int64_t d[ACC_DIGITS];
    int64_t pending;
} orc_acc;

static void acc_clear(orc_acc *a) { memset(a, 0, sizeof(*a)); }

static void acc_normalise(orc_acc *a)
{
    int64_t carry = 0;
    for (int q = 0; q < ACC_DIGITS; ++q) {
        int64_t v = a->d[q] + carry;
        /* floor division by 2^32 (gcc shifts signed values arithmetically);
         * the products below stay within int64 (|c| < 2^31) and, unlike a
         * left shift of a negative value, are defined C */
        int64_t c = v >> 32;
        a->d[q] = v - c * ((int64_t)1 << 32);
        carry = c;
    }
    /* the top digit keeps the sign: fold the final carry back in */
    a->d[ACC_DIGITS - 1] += carry * ((int64_t)1 << 32);
    a->pending = 0;
}

static void acc_add(orc_acc *a, double x)
{
    if (x == 0.0)
        return;
    int e;
    double f = frexp(x, &e); /* x = f * 2^e, 0.5 <= |f| < 1 */
    int64_t m = (int64_t)ldexp(f, 53); /* exact: |m| < 2^53 */
    int p = e - 53 + ACC_BIAS; /* bit position of m's lowest bit */
    int neg = m < 0;
    uint64_t u = (uint64_t)(neg ? -m : m);
    int q = p >> 5, r = p & 31;
    /* u << r spans at most 85 bits: three 32-bit digits */
    unsigned __int128 w = (unsigned __int128)u << r;
    for (int k = 0; k < 3; ++k) {
        int64_t piece = (int64_t)(uint32_t)(w >> (32 * k));
        a->d[q + k] += neg ? -piece : piece;
    }
    if (++a->pending >= (1 << 29))
        acc_normalise(a);
}

/* round the accumulated value to the nearest double (ties to even) */
static double acc_round(orc_acc *a)
{
    acc_normalise(a);
    int neg = a->d[ACC_DIGITS - 1] < 0;
    uint32_t mag[ACC_DIGITS];
    /* two's complement magnitude over ACC_DIGITS*32 bits */
    uint64_t borrow = 1;
    for (int q = 0; q < ACC_DIGITS; ++q) {
        uint32_t v = (uint32_t)(a->d[q] & 0xffffffff);
        if (neg) {
            uint64_t t = (uint64_t)(uint32_t)~v + borrow;
            mag[q] = (uint32_t)t;
            borrow = t >> 32;
        } else {
            mag[q] = v;
        }
    }
    int top = -1;
    for (int q = ACC_DIGITS - 1; q >= 0 && top < 0; --q)
        if (mag[q])
            for (int b = 31; b >= 0; --b)
                if (mag[q] >> b & 1) {
                    top = 32 * q + b;
                    break;
                }
    if (top < 0)
        return 0.0;
#define BIT(n) ((n) >= 0 ? (int)((mag[(n) >> 5] >> ((n) & 31)) & 1u) : 0)
    /* 53 significant bits from position top down to top-52 */
    uint64_t sig = 0;
    for (int b = top; b > top - 53; --b)
        sig = (sig << 1) | (uint64_t)BIT(b);
    int low = top - 53; /* the first discarded bit */
    int round_bit = BIT(low);
    int sticky = 0;
    for (int b = low - 1; b >= 0 && !sticky; --b)
        sticky = BIT(b);
#undef BIT
    if (round_bit && (sticky || (sig & 1)))
        sig += 1; /* may carry to 2^53: still exact as a double */
    double v = ldexp((double)sig, top - 52 - ACC_BIAS);
    return neg ? -v : v;
}

/* exact sum of n doubles, rounded once (exposed for tests) */
double orc_exact_sum(const double *x, int64_t n)
{
    orc_acc a;
    acc_clear(&a);
    for (int64_t k = 0; k < n; ++k)
        acc_add(&a, x[k]);
    return acc_round(&a);
}

/* ------------------------------------------------------------------------ */
/* instance access                                                          */
/* ------------------------------------------------------------------------ */

static int lat_neighbour(const orc_instance *in, int i, int axis, int step)
{
    int c[3] = {0, 0, 0}, rem = i;
    for (int a = 0; a < in->dim; ++a) {
        c[a] = rem % in->L[a];
        rem /= in->L[a];
    }
    c[axis] = (c[axis] + step + in->L[axis]) % in->L[axis];
    int idx = 0;
    for (int a = in->dim - 1; a >= 0; --a)
        idx = idx * in->L[a] + c[a];
    return idx;
}

/* sum_j J_ij x_j (j != i) in FP64, j in increasing order */
static double field_of(const orc_instance *in, int i, const double *x)
{
    double s = 0.0;
    if (in->kind == ORC_DENSE) {
        const float *row = in->J + (size_t)i * in->N;
        for (int j = 0; j < in->N; ++j)
            if (j != i)
                s += (double)row[j] * x[j];
    } else if (in->kind == ORC_CSR) {
        for (int k = in->rowptr[i]; k < in->rowptr[i + 1]; ++k)
            s += (double)in->val[k] * x[in->col[k]];
    } else {
        /* lattice: collect the 2*dim couplings, then add in increasing j */
        int nb[6];
        double w[6];
        int n = 0;
        for (int a = 0; a < in->dim; ++a) {
            int jp = lat_neighbour(in, i, a, +1);
            int jm = lat_neighbour(in, i, a, -1);
            nb[n] = jp;
            w[n++] = (double)in->bond[(size_t)a * in->N + i];
            nb[n] = jm;
            w[n++] = (double)in->bond[(size_t)a * in->N + jm];
        }
        for (int u = 1; u < n; ++u) /* insertion sort by neighbour index */
            for (int v = u; v > 0 && nb[v - 1] > nb[v]; --v) {
                int ti = nb[v];
                nb[v] = nb[v - 1];
                nb[v - 1] = ti;
                double tw = w[v];
                w[v] = w[v - 1];
                w[v - 1] = tw;
            }
        for (int u = 0; u < n; ++u)
            s += w[u] * x[nb[u]];
    }
    return s;
}

/* exact energy of spins s (values +-1) */
double orc_energy(const orc_instance *in, const int8_t *s)
{
    orc_acc a;
    acc_clear(&a);
    int N = in->N;
    for (int i = 0; i < N; ++i) {
        double si = (double)s[i];
        if (in->kind == ORC_DENSE) {
            const float *row = in->J + (size_t)i * N;
            for (int j = 0; j < N; ++j)
                if (j != i && row[j] != 0.0f)
                    acc_add(&a, -(double)row[j] * si * (double)s[j]);
        } else if (in->kind == ORC_CSR) {
            for (int k = in->rowptr[i]; k < in->rowptr[i + 1]; ++k)
                acc_add(&a, -(double)in->val[k] * si * (double)s[in->col[k]]);
        } else {
            for (int ax = 0; ax < in->dim; ++ax) {
                int jp = lat_neighbour(in, i, ax, +1);
                int jm = lat_neighbour(in, i, ax, -1);
                acc_add(&a, -(double)in->bond[(size_t)ax * N + i] * si * (double)s[jp]);
                acc_add(&a, -(double)in->bond[(size_t)ax * N + jm] * si * (double)s[jm]);
            }
        }
        if (in->h)
            acc_add(&a, -(double)in->h[i] * si);
    }
    return acc_round(&a);
}

/* ------------------------------------------------------------------------ */
/* phases                                                                   */
/* ------------------------------------------------------------------------ */

/* phase index of every spin; returns the number of phases */
int orc_phases(const orc_instance *in, const orc_schedule *sc, int32_t *phase_of)
{
    int N = in->N;
    if (sc->update == ORC_JACOBI) {
        for (int i = 0; i < N; ++i)
            phase_of[i] = 0;
        return 1;
    }
    if (in->kind == ORC_DENSE) {
        int B = sc->phases < 1 ? 1 : sc->phases;
        if (B > N)
            B = N;
        for (int b = 0; b < B; ++b) {
            int lo = (int)((int64_t)b * N / B), hi = (int)((int64_t)(b + 1) * N / B);
            for (int i = lo; i < hi; ++i)
                phase_of[i] = b;
        }
        return B;
    }
    if (in->kind == ORC_LATTICE) {
        for (int i = 0; i < N; ++i) {
            int rem = i, sum = 0;
            for (int a = 0; a < in->dim; ++a) {
                sum += rem % in->L[a];
                rem /= in->L[a];
            }
            phase_of[i] = sum & 1;
        }
        return 2;
    }
    /* sparse: greedy colouring in index order, looking at neighbours u < v */
    int ncol = 0;
    char *used = (char *)calloc((size_t)N + 1, 1);
    for (int v = 0; v < N; ++v) {
        for (int k = in->rowptr[v]; k < in->rowptr[v + 1]; ++k) {
            int u = in->col[k];
            if (u < v)
                used[phase_of[u]] = 1;
        }
        int c = 0;
        while (used[c])
            ++c;
        phase_of[v] = c;
        if (c + 1 > ncol)
            ncol = c + 1;
        for (int k = in->rowptr[v]; k < in->rowptr[v + 1]; ++k) {
            int u = in->col[k];
            if (u < v)
                used[phase_of[u]] = 0;
        }
    }
    free(used);
    return ncol < 1 ? 1 : ncol;
}

/* ------------------------------------------------------------------------ */
/* temperatures                                                             */
/* ------------------------------------------------------------------------ */

/* the run's temperature levels; returns how many (at most cap are written) */
int orc_levels(const orc_schedule *sc, double T0, double *T, int cap)
{
    int n = 0;
    if (sc->kind == ORC_GEOMETRIC) {
        int K = sc->steps;
        for (int k = 0; k < K; ++k) {
            double t = (K == 1) ? T0 : T0 * exp(((double)k / (double)(K - 1)) * log(sc->T_end / T0));
            if (n < cap)
                T[n] = t;
            ++n;
        }
    } else {
        double t = T0;
        for (;;) {
            t = t - sc->c_step;
            if (!(t > 0.0))
                break;
            if (n < cap)
                T[n] = t;
            ++n;
        }
    }
    return n;
}

/* ------------------------------------------------------------------------ */
/* one run                                                                  */
/* ------------------------------------------------------------------------ */

typedef struct {
    int64_t sweeps;
    int64_t levels;
    int64_t cap_hits;
    double last_T;
    double last_d;
} orc_run_stats;

/* Per-level records of one run, all optional (cap entries each; level kk of
 * the visited range at index kk, entries past the run's levels untouched).
 *   replay  sweeps to run at each level instead of the stopping rule (an
 *           entry <= 0 keeps the rule at that level): the sweep counts
 *           another implementation reports, so that its trajectory can be
 *           followed where its d-versus-d_min decisions differ from this
 *           one's (Algorithm 1's repeat ... until, decided in another
 *           precision).
 *   sweeps  sweeps run at each level.
 *   own     the sweep at which this oracle's own rule (d < d_min, or the
 *           max_sweeps cap) ends the level; under replay, count + 1 when the
 *           rule would not have ended it within the replayed count.
 *   d_own   the largest change d of sweep min(own, sweeps run). */
typedef struct {
    const int32_t *replay;
    int32_t *sweeps;
    int32_t *own;
    double *d_own;
    int cap;
} orc_level_io;

/* relax one run in place; m has N entries */
static void run_one(const orc_instance *in, const orc_schedule *sc, const int32_t *phase_of, int nph,
                    double T0, double *m, double *phi, orc_run_stats *st, const orc_level_io *io)
{
    int N = in->N;
    int cap = 0;
    int nlev = orc_levels(sc, T0, NULL, 0);
    double *lev = (double *)malloc(sizeof(double) * (size_t)(nlev > 0 ? nlev : 1));
    orc_levels(sc, T0, lev, nlev);
    int k0 = sc->first_level < 0 ? 0 : sc->first_level;
    int k1 = sc->level_count < 0 ? nlev : k0 + sc->level_count;
    if (k1 > nlev)
        k1 = nlev;
    double g = sc->damping;
    memset(st, 0, sizeof(*st));
    st->last_T = NAN;
    st->last_d = NAN;
    for (int k = k0; k < k1; ++k) {
        double T = lev[k];
        int sweeps = 0;
        double d;
        const int kk = k - k0;
        const int rec = io && kk < io->cap;
        /* the replayed count, or 0 to follow the stopping rule */
        const int want = (rec && io->replay) ? io->replay[kk] : 0;
        int own = 0;
        double d_own = NAN;
        do {
            d = 0.0;
            for (int p = 0; p < nph; ++p) {
                for (int i = 0; i < N; ++i)
                    if (phase_of[i] == p)
                        phi[i] = field_of(in, i, m) + (in->h ? 0.5 * (double)in->h[i] : 0.0);
                for (int i = 0; i < N; ++i)
                    if (phase_of[i] == p) {
                        double t = tanh(phi[i] / T);
                        double nw = (g == 1.0) ? t : (1.0 - g) * m[i] + g * t;
                        double dd = fabs(nw - m[i]);
                        if (dd > d)
                            d = dd;
                        m[i] = nw;
                    }
            }
            ++sweeps;
            if (!own && ((d < sc->d_min) || sweeps >= sc->max_sweeps)) {
                own = sweeps; /* where this oracle's own rule ends the level */
                d_own = d;
            }
        } while (want > 0 ? sweeps < want : (!(d < sc->d_min) && sweeps < sc->max_sweeps));
        if (!own) {
            own = sweeps + 1; /* the rule would have run on past the replayed count */
            d_own = d;
        }
        if (sc->max_sweeps > 1 && !(d < sc->d_min))
            ++cap; /* a level cut short by the sweep cap */
        if (rec) {
            if (io->sweeps)
                io->sweeps[kk] = sweeps;
            if (io->own)
                io->own[kk] = own;
            if (io->d_own)
                io->d_own[kk] = d_own;
        }
        st->sweeps += sweeps;
        st->levels += 1;
        st->last_T = T;
        st->last_d = d;
    }
    st->cap_hits = cap;
    free(lev);
}

/* ------------------------------------------------------------------------ */
/* solve over a range of runs (threads over runs)                           */
/* ------------------------------------------------------------------------ */

typedef struct {
    /* inputs */
    const orc_instance *in;
    const orc_schedule *sc;
    uint64_t seed;
    int run_begin, run_count;
    const double *m0; /* N x run_count (runs contiguous) or NULL */
    const double *T0; /* run_count or NULL */
    /* outputs (any may be NULL) */
    double *m_final; /* N x run_count */
    int8_t *spins; /* run_count x N */
    double *energy; /* run_count */
    double *T0_out; /* run_count */
    int64_t *sweeps; /* run_count */
    int64_t *levels; /* run_count */
    int64_t *cap_hits; /* run_count */
    double *last_T; /* run_count */
    orc_level_io lio; /* per-level records, cap entries per run (pointers to run 0's) */
    /* shared */
    const int32_t *phase_of;
    int nph;
    int next;
    pthread_mutex_t lock;
} orc_job;

static void *worker(void *arg)
{
    orc_job *jb = (orc_job *)arg;
    const orc_instance *in = jb->in;
    int N = in->N;
    double *m = (double *)malloc(sizeof(double) * (size_t)N);
    double *phi = (double *)malloc(sizeof(double) * (size_t)N);
    int8_t *s = (int8_t *)malloc((size_t)N);
    for (;;) {
        pthread_mutex_lock(&jb->lock);
        int q = jb->next++;
        pthread_mutex_unlock(&jb->lock);
        if (q >= jb->run_count)
            break;
        int64_t run = (int64_t)jb->run_begin + q;
        for (int i = 0; i < N; ++i)
            m[i] = jb->m0 ? jb->m0[(size_t)i * jb->run_count + q] : orc_initial_m(jb->seed, run, i);
        double T0 = jb->T0 ? jb->T0[q] : orc_initial_T(jb->seed, run, jb->sc->T_lo, jb->sc->T_hi);
        orc_run_stats st;
        orc_level_io io = jb->lio;
        const size_t o = (size_t)q * (size_t)(io.cap > 0 ? io.cap : 0);
        io.replay = io.replay ? io.replay + o : NULL;
        io.sweeps = io.sweeps ? io.sweeps + o : NULL;
        io.own = io.own ? io.own + o : NULL;
        io.d_own = io.d_own ? io.d_own + o : NULL;
        run_one(in, jb->sc, jb->phase_of, jb->nph, T0, m, phi, &st, io.cap > 0 ? &io : NULL);
        for (int i = 0; i < N; ++i)
            s[i] = (m[i] >= 0.0) ? 1 : -1;
        if (jb->m_final)
            for (int i = 0; i < N; ++i)
                jb->m_final[(size_t)i * jb->run_count + q] = m[i];
        if (jb->spins)
            memcpy(jb->spins + (size_t)q * N, s, (size_t)N);
        if (jb->energy)
            jb->energy[q] = orc_energy(in, s);
        if (jb->T0_out)
            jb->T0_out[q] = T0;
        if (jb->sweeps)
            jb->sweeps[q] = st.sweeps;
        if (jb->levels)
            jb->levels[q] = st.levels;
        if (jb->cap_hits)
            jb->cap_hits[q] = st.cap_hits;
        if (jb->last_T)
            jb->last_T[q] = st.last_T;
    }
    free(m);
    free(phi);
    free(s);
    return NULL;
}

/* orc_solve with per-level records (see orc_level_io; arrays [run_count x
 * cap], any pointer NULL; cap = 0 keeps none) */
int orc_solve_levels(const orc_instance *in, const orc_schedule *sc, uint64_t seed, int run_begin, int run_count,
                     const double *m0, const double *T0, double *m_final, int8_t *spins, double *energy,
                     double *T0_out, int64_t *sweeps, int64_t *levels, int64_t *cap_hits, double *last_T,
                     int nthreads, const int32_t *replay, int32_t *sweeps_per_level, int32_t *own_per_level,
                     double *d_per_level, int cap);

int orc_solve(const orc_instance *in, const orc_schedule *sc, uint64_t seed, int run_begin, int run_count,
              const double *m0, const double *T0, double *m_final, int8_t *spins, double *energy, double *T0_out,
              int64_t *sweeps, int64_t *levels, int64_t *cap_hits, double *last_T, int nthreads)
{
    return orc_solve_levels(in, sc, seed, run_begin, run_count, m0, T0, m_final, spins, energy, T0_out, sweeps,
                            levels, cap_hits, last_T, nthreads, NULL, NULL, NULL, NULL, 0);
}

int orc_solve_levels(const orc_instance *in, const orc_schedule *sc, uint64_t seed, int run_begin, int run_count,
                     const double *m0, const double *T0, double *m_final, int8_t *spins, double *energy,
                     double *T0_out, int64_t *sweeps, int64_t *levels, int64_t *cap_hits, double *last_T,
                     int nthreads, const int32_t *replay, int32_t *sweeps_per_level, int32_t *own_per_level,
                     double *d_per_level, int cap)
{
    if (!in || !sc || in->N < 1 || run_count < 0)
        return 1;
    int32_t *phase_of = (int32_t *)malloc(sizeof(int32_t) * (size_t)in->N);
    orc_job jb;
    memset(&jb, 0, sizeof(jb));
    jb.in = in;
    jb.sc = sc;
    jb.seed = seed;
    jb.run_begin = run_begin;
    jb.run_count = run_count;
    jb.m0 = m0;
    jb.T0 = T0;
    jb.m_final = m_final;
    jb.spins = spins;
    jb.energy = energy;
    jb.T0_out = T0_out;
    jb.sweeps = sweeps;
    jb.levels = levels;
    jb.cap_hits = cap_hits;
    jb.last_T = last_T;
    jb.lio.replay = replay;
    jb.lio.sweeps = sweeps_per_level;
    jb.lio.own = own_per_level;
    jb.lio.d_own = d_per_level;
    jb.lio.cap = cap < 0 ? 0 : cap;
    jb.nph = orc_phases(in, sc, phase_of);
    jb.phase_of = phase_of;
    pthread_mutex_init(&jb.lock, NULL);
    if (nthreads < 1)
        nthreads = 1;
    if (nthreads > 256)
        nthreads = 256;
    pthread_t th[256];
    for (int t = 1; t < nthreads; ++t)
        pthread_create(&th[t], NULL, worker, &jb);
    worker(&jb);
    for (int t = 1; t < nthreads; ++t)
        pthread_join(th[t], NULL);
    pthread_mutex_destroy(&jb.lock);
    free(phase_of);
    return 0;
}

/* best run over energies: smallest energy, ties to the lowest index;
 * returns the index and writes the hit count (runs equal to the best) */
int orc_best(const double *energy, int runs, int64_t *hits)
{
    int best = -1;
    for (int r = 0; r < runs; ++r)
        if (best < 0 || energy[r] < energy[best])
            best = r;
    int64_t h = 0;
    for (int r = 0; r < runs; ++r)
        if (best >= 0 && energy[r] == energy[best])
            ++h;
    if (hits)
        *hits = h;
    return best;
}
