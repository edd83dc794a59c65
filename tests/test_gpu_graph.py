"""GPU parity of the LDS-resident solver for lattices and sparse graphs
against the CPU oracle, through the C interface.

Tolerances: fp32 magnetisations within 1e-5 of the oracle; the fp64 form
within 1e-9 (it differs from the oracle only in the tanh implementation and
the order of the neighbour sum); energies of equal spin vectors bit-exact."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1907_05124_amd import inputs as I
from tests.gpu_common import announce, c16_parity, check_replay, require_gpu

pytestmark = pytest.mark.gpu


def _mars():
    require_gpu()
    from paper_1907_05124_amd import mars as M

    return M


def _rel_sched(inst, **kw):
    s = I.field_scale(inst)
    base = dict(T_lo=0.25 * s, T_hi=1.5 * s, T_end=0.01 * s, steps=300)
    base.update(kw)
    return I.Schedule(**base)


CASES = {
    "ea2d_16": lambda: I.lattice_instance((16, 16), 1),
    "ea2d_6x4": lambda: I.lattice_instance((6, 4), 2),
    "ea3d_8": lambda: I.lattice_instance((8, 8, 8), 3),
    "ea3d_4x6x8": lambda: I.lattice_instance((4, 6, 8), 4),
    # 16^3: each thread walks two planes (interior and wrapping ones);
    # 20x20x8: the walk step is odd, so the x parity alternates along it
    "ea3d_16": lambda: I.lattice_instance((16, 16, 16), 9),
    "ea3d_20x20x8": lambda: I.lattice_instance((20, 20, 8), 10),
    "lat3d_field": lambda: _with_field(I.lattice_instance((16, 16, 16), 14), 0.6),
    "er_pm1": lambda: I.er_instance(800, 5, p=0.06, weights="pm1"),
    "er_unit": lambda: I.er_instance(300, 6, p=0.05, weights="unit"),
    "er_field": lambda: _with_field(I.er_instance(200, 7, p=0.05, weights="pm1"), 0.4),
    "lat_field": lambda: _with_field(I.lattice_instance((8, 4), 8), 0.6),
    # average degree >= 16 (entry groups read ahead) with isolated vertices
    # (slices without entries)
    "er_dense_isolated": lambda: _with_isolated(I.er_instance(300, 11, p=0.12, weights="pm1"), 21),
    # int8 weights other than +-1 (the general entry encoding), short and long rows
    "er_int8": lambda: _with_int8_weights(I.er_instance(500, 15, p=0.01, weights="pm1")),
    "er_int8_dense": lambda: _with_int8_weights(I.er_instance(300, 16, p=0.1, weights="pm1")),
}


def _with_int8_weights(inst):
    """The instance with nonzero weights in -3..3: the sign of the original
    weight times 1 + ((31 min(i, j) + 17 max(i, j)) mod 3), equal for both
    directions of an edge."""
    rows = np.repeat(np.arange(inst.N), np.diff(inst.rowptr))
    lo, hi = np.minimum(rows, inst.col), np.maximum(rows, inst.col)
    mag = 1 + (31 * lo.astype(np.int64) + 17 * hi.astype(np.int64)) % 3
    return I.CsrInstance(N=inst.N, rowptr=inst.rowptr, col=inst.col,
                         val=(np.sign(inst.val) * mag).astype(np.int8))


def _with_isolated(inst, k):
    """The instance with k isolated vertices appended (no couplings)."""
    rowptr = np.concatenate([inst.rowptr, np.full(k, inst.rowptr[-1], dtype=np.int32)])
    return I.CsrInstance(N=inst.N + k, rowptr=rowptr.astype(np.int32), col=inst.col, val=inst.val)


def _with_field(inst, scale):
    inst.h = (np.random.default_rng(3).standard_normal(inst.N) * scale).astype(np.float32)
    return inst


@pytest.mark.parametrize("case", sorted(CASES))
@pytest.mark.parametrize("precision,tol", [("fp32", 1e-5), ("fp64", 1e-9)])
def test_one_level_parity(case, precision, tol):
    M = _mars()
    inst = CASES[case]()
    sch = _rel_sched(inst, precision=precision, level_count=1)
    R = 200
    announce("graph one level", case, precision, R)
    with M.Instance.from_inputs(inst) as g:
        out = g.solve_ex(R, sch, 17, want_m=True)
    ref = O.solve(inst, R, sch, 17, run_count=R)
    err = np.max(np.abs(out["m"].cpu().numpy().astype(np.float64) - ref["m"]))
    assert err <= tol, err


@pytest.mark.parametrize("case", ["ea3d_16", "ea3d_20x20x8", "ea2d_16", "er_pm1", "er_field", "lat_field"])
@pytest.mark.parametrize("update", ["phased", "jacobi"])
def test_damped_parity(case, update):
    """Damped update m <- (1 - g) m + g tanh(...) with g = 0.5 (the damped
    kernels are separate instantiations): after one fp32 level every element
    within 1e-5 of the oracle; after five, every run the oracle finds well
    conditioned (as in test_anneal_parity, at most 5 % excluded)."""
    M = _mars()
    inst = CASES[case]()
    R = 200
    announce("graph damped", case, update, R)
    for levels in (1, 5):
        sch = _rel_sched(inst, precision="fp32", update=update, damping=0.5, level_count=levels)
        with M.Instance.from_inputs(inst) as g:
            out = g.solve_ex(R, sch, 29, want_m=True)
        ref = O.solve(inst, R, sch, 29, run_count=R)
        m = out["m"].cpu().numpy()
        if levels == 1:
            err = np.max(np.abs(m.astype(np.float64) - ref["m"]))
            assert err <= 1e-5, err
        else:
            c16_parity(m, inst, R, sch, 29, ref, "fp32", max_excluded=0.05,
                       label="%s damped %s level 5" % (case, update))


RUN_BLOCK_CASES = ["er_pm1", "er_unit", "er_field", "er_dense_isolated", "er_int8", "er_int8_dense", "ea3d_8",
                   "ea3d_16", "ea2d_6x4", "lat_field"]


@pytest.mark.parametrize("case", RUN_BLOCK_CASES)
@pytest.mark.parametrize("R,vec,lps", [(1031, "", ""), (2053, "1", ""), (2053, "2", ""), (4100, "", ""),
                                       (4100, "2", ""), (16400, "", ""), (1031, "", "4"), (4100, "", "2"),
                                       (4100, "", "4"), (16400, "", "1")])
def test_one_level_run_blocks(case, R, vec, lps, monkeypatch):
    """Several runs per workgroup (R >= 1024) and per thread, with a ragged
    last block: one fp32 level within 1e-5 of the oracle.  The sparse path
    runs four runs per lane group by default on blocks of at least four runs;
    MARS_SPARSE_VEC forces 1 or 2; MARS_SPARSE_LPS forces 1, 2 or 4 lanes per
    slot (the row split over lanes, with four runs per group)."""
    M = _mars()
    for name, val in (("MARS_SPARSE_VEC", vec), ("MARS_SPARSE_LPS", lps)):
        if val:
            monkeypatch.setenv(name, val)
        else:
            monkeypatch.delenv(name, raising=False)
    inst = CASES[case]()
    sch = _rel_sched(inst, precision="fp32", level_count=1)
    announce("graph run blocks", case, R, vec, lps)
    with M.Instance.from_inputs(inst) as g:
        out = g.solve_ex(R, sch, 29, want_m=True)
    ref = O.solve(inst, R, sch, 29, run_count=R)
    err = np.max(np.abs(out["m"].cpu().numpy().astype(np.float64) - ref["m"]))
    assert err <= 1e-5, err


@pytest.mark.parametrize("case", ["er_field", "er_unit", "lat_field", "ea3d_8"])
@pytest.mark.parametrize("R", [200, 1031, 4100])
@pytest.mark.parametrize("precision,levels,tol", [("fp32", 1, 1e-5), ("fp64", 4, 1e-9)])
def test_jacobi_parity(case, R, precision, levels, tol):
    """Synchronous updates (both state copies, swapped after each sweep)."""
    M = _mars()
    inst = CASES[case]()
    sch = _rel_sched(inst, precision=precision, update="jacobi", level_count=levels)
    announce("graph jacobi", case, R, precision, levels)
    with M.Instance.from_inputs(inst) as g:
        out = g.solve_ex(R, sch, 37, want_m=True)
    ref = O.solve(inst, R, sch, 37, run_count=R)
    err = np.max(np.abs(out["m"].cpu().numpy().astype(np.float64) - ref["m"]))
    assert err <= tol, err


@pytest.mark.parametrize("case", ["er_field", "ea3d_8", "lat_field"])
@pytest.mark.parametrize("precision", ["fp64", "fp32", "fp16"])
@pytest.mark.parametrize("empty", ["steps", "count"])
def test_zero_levels(case, precision, empty):
    """A schedule with no level (steps = 0, or level_count = 0) leaves every
    run at its draw: m equals the stored m0, spins its signs, energies exact,
    no sweeps (Algorithm 1 with an empty temperature loop)."""
    M = _mars()
    inst = CASES[case]()
    R = 300
    kw = dict(steps=0) if empty == "steps" else dict(level_count=0)
    sch = _rel_sched(inst, precision=precision, **kw)
    announce("graph zero levels", case, precision, empty)
    with M.Instance.from_inputs(inst) as g:
        out = g.solve_ex(R, sch, 5, want_m=True, want_spins=True)
    ref = O.solve(inst, R, sch.replace(precision="fp64"), 5, run_count=R)
    m0 = O.initial_m(5, R, inst.N)
    if precision == "fp16":
        m0 = m0.astype(np.float16).astype(np.float64)
    assert np.array_equal(out["m"].cpu().numpy().astype(np.float64), m0)
    S = out["spins"].cpu().numpy()
    assert np.array_equal(S, np.where(m0 >= 0, 1, -1).T.astype(np.int8))
    assert np.array_equal(S, ref["spins"])
    assert np.array_equal(out["energies"].cpu().numpy(), ref["energy"])
    assert out["result"]["sweeps_executed"] == 0 and out["result"]["levels_executed"] == 0


def _dense_couplings(inst):
    if isinstance(inst, I.LatticeInstance):
        return I.lattice_dense(inst).J.astype(np.float64)
    return I.csr_dense(inst).J.astype(np.float64)


@pytest.mark.parametrize("case", ["er_pm1", "er_field", "er_int8_dense", "ea3d_8", "lat_field", "ea3d_16",
                                  "ea3d_20x20x8", "lat3d_field"])
@pytest.mark.parametrize("R", [200, 1031, 2048, 4100])
def test_one_level_fp16_storage(case, R):
    """fp16 magnetisation storage, fp32 fields, one level from fp16-exact
    initial states (the same for the oracle).  A spin's new value differs from
    the oracle's by its fp16 rounding (<= 2^-12 for |m| < 1) plus fp32
    arithmetic, and by what it inherits from the phases before its own: a
    neighbour off by e_j moves Phi_i by |J_ij| e_j and m_i by at most
    (1 - m_i^2) / T times that (first order, with 10 % slack); the bound is
    accumulated phase by phase.

    On the 3D lattices, run pairs (R >= 1031) walk z columns with an even
    step: 8^3 and 16^3 at R = 1031 four or eight planes apart, 16^3 at
    R = 2048 and 20x20x8 at R = 1031 two planes apart (the +z word of one
    site is carried as the -z word of the next; 20x20 planes do not split
    into whole waves, so z differs between the lanes of a wave)."""
    M = _mars()
    torch = require_gpu()
    inst = CASES[case]()
    sch = _rel_sched(inst, precision="fp16", level_count=1)
    m0 = O.initial_m(31, R, inst.N).astype(np.float16).astype(np.float32)
    announce("graph fp16 one level", case, R)
    with M.Instance.from_inputs(inst) as g:
        out = g.solve_ex(R, sch, 31, m0=torch.from_numpy(m0).cuda(), want_m=True)
    ref = O.solve(inst, R, sch.replace(precision="fp64"), 31, run_count=R, m0=m0.astype(np.float64))
    ph, _ = O.phases(inst, sch)
    Ja = np.abs(_dense_couplings(inst))
    gain = (1.0 - ref["m"] ** 2) / ref["T0"][None, :]
    tol = np.zeros_like(ref["m"])
    for c in np.unique(ph):
        own, earlier = ph == c, ph < c
        tol[own] = 2.0**-12 + 1e-5 + 1.1 * gain[own] * (Ja[np.ix_(own, earlier)] @ tol[earlier])
    err = np.abs(out["m"].cpu().numpy().astype(np.float64) - ref["m"])
    assert np.all(err <= tol), float(np.max(err / tol))


def _decided_spins_agree(S, m, ref, bar):
    """Spins equal the oracle's wherever the oracle's |m| exceeds the bar on
    runs that meet it (elsewhere the sign is a rounding decision)."""
    close = np.max(np.abs(np.asarray(m, dtype=np.float64) - ref["m"]), axis=0) <= bar
    decided = np.abs(ref["m"]) > bar
    assert not np.any((S.T != ref["spins"].T) & decided & close[None, :])


@pytest.mark.parametrize("case", ["ea2d_16", "ea3d_8", "er_pm1", "lat_field", "er_field"])
@pytest.mark.parametrize("precision,levels", [("fp64", 10), ("fp64", 300), ("fp32", 300)])
def test_anneal_parity(case, precision, levels):
    """Geometric anneal checked at levels 10 and 300 (fp64) and at the end
    (fp32): every run the oracle finds well conditioned (final m moves by
    <= 1e-6 under a 1e-9 change of m0; fp32: and by <= 2.5e-6 when T0 moves
    by one fp32 ulp) agrees within 1e-9 (fp64) / 1e-5 (fp32) in every
    element, at most 5 % of the runs excluded; decided spins agree and
    energies of equal spin vectors are equal.  (Mid-anneal, the fp32 form's
    rounding at every sweep moves some runs by more than 1e-5 in ways a
    single change of the oracle's inputs does not predict; the fp32 form is
    held to the bar after one level and at the end.)"""
    M = _mars()
    inst = CASES[case]()
    sch = _rel_sched(inst, precision=precision, level_count=levels)
    R = 96
    announce("graph anneal", case, precision, levels, R)
    with M.Instance.from_inputs(inst) as g:
        out = g.solve_ex(R, sch, 23, want_m=True, want_spins=True)
    ref = O.solve(inst, R, sch, 23, run_count=R)
    S = out["spins"].cpu().numpy()
    E = out["energies"].cpu().numpy()
    m = out["m"].cpu().numpy()
    bar = 1e-5 if precision == "fp32" else 1e-9
    c16_parity(m, inst, R, sch, 23, ref, precision, max_excluded=0.05,
               label="%s %s level %d" % (case, precision, levels))
    _decided_spins_agree(S, m, ref, bar)
    same = np.all(S == ref["spins"], axis=1)
    assert np.array_equal(E[same], ref["energy"][same])


def test_config1_lattice_fp64_full():
    """2D +-J L=16, 1024 runs, T0 ~ U[0.5, 3], 300 geometric levels to 0.02,
    fp64: every well-conditioned run within 1e-9 of the oracle (at most 2 %
    excluded), decided spins equal, energies of equal spins equal."""
    M = _mars()
    w = I.workload("ea2d_L16", seed=1)
    announce("config1 fp64", w.runs)
    with M.Instance.from_inputs(w.instance) as g:
        out = g.solve_ex(w.runs, w.schedule, 1, want_m=True, want_spins=True)
    ref = O.solve(w.instance, w.runs, w.schedule, 1, run_count=w.runs)
    S = out["spins"].cpu().numpy()
    m = out["m"].cpu().numpy()
    c16_parity(m, w.instance, w.runs, w.schedule, 1, ref, "fp64", max_excluded=0.02, label="config 1 fp64")
    _decided_spins_agree(S, m, ref, 1e-9)
    E = out["energies"].cpu().numpy()
    same = np.all(S == ref["spins"], axis=1)
    assert np.array_equal(E[same], ref["energy"][same])
    assert out["result"]["best_energy"] == E.min()


@pytest.mark.parametrize("precision", ["fp64", "fp32", "fp16"])
def test_brute_force_ground_state_4x4(precision):
    """4x4 +-J lattice: the best of 1024 runs is the brute-force ground state."""
    M = _mars()
    w = I.workload("ea2d_L4", seed=3)
    Jd = I.lattice_dense(w.instance).J.astype(np.float64)
    idx = np.arange(2**16)
    S = (1 - 2 * ((idx[:, None] >> np.arange(16)[None, :]) & 1)).astype(np.float64)
    gs = np.min(-np.einsum("ki,ij,kj->k", S, Jd, S))
    announce("brute force 4x4", precision)
    with M.Instance.from_inputs(w.instance) as g:
        out = g.solve_ex(w.runs, w.schedule.replace(precision=precision), 2, want_spins=True)
    E = out["energies"].cpu().numpy()
    assert np.all(E >= gs) and E.min() == gs
    spins = out["spins"].cpu().numpy().astype(np.float64)
    direct = -np.einsum("ri,ij,rj->r", spins, Jd, spins)
    assert np.array_equal(direct, E)


def test_energy_exact_graphs():
    M = _mars()
    torch = require_gpu()
    for name in ("ea2d_16", "ea3d_4x6x8", "er_pm1", "er_field", "lat_field"):
        inst = CASES[name]()
        S = I.random_spins(inst.N, 33, 5)
        announce("graph energy", name)
        with M.Instance.from_inputs(inst) as g:
            E = g.energy(torch.from_numpy(S).cuda()).cpu().numpy()
        assert np.array_equal(E, O.energy(inst, S)), name


def test_jacobi_sublattice_symmetry_gpu():
    """Synchronous update on a bipartite lattice: from D m0 the state is (-1)^k D m(k), bitwise."""
    M = _mars()
    torch = require_gpu()
    L = (8, 6)
    inst = I.lattice_instance(L, 9)
    N, R = 48, 16
    D = np.array([(-1.0) ** ((i % L[0]) + (i // L[0])) for i in range(N)])
    m0 = O.initial_m(3, R, N)
    T0 = torch.full((R,), 1.3, dtype=torch.float64, device="cuda")
    announce("jacobi symmetry")
    with M.Instance.from_inputs(inst) as g:
        for k in (1, 4, 7):
            sch = I.Schedule(T_lo=1.3, T_hi=1.3, T_end=0.2, steps=20, update="jacobi", level_count=k,
                             precision="fp64")
            a = g.solve_ex(R, sch, 0, m0=torch.from_numpy(m0).cuda(), T0=T0, want_m=True)
            b = g.solve_ex(R, sch, 0, m0=torch.from_numpy(D[:, None] * m0).cuda(), T0=T0, want_m=True)
            assert np.array_equal(b["m"].cpu().numpy(), ((-1.0) ** k) * D[:, None] * a["m"].cpu().numpy())


PAPER_CASES = {
    "er400": (lambda: I.er_instance(400, 10, p=0.03, weights="pm1"), 2.0, 0.2),
    "er_field": (lambda: CASES["er_field"](), 2.0, 0.2),
    "ea2d_16": (lambda: CASES["ea2d_16"](), 1.5, 0.1),
    "ea3d_8": (lambda: CASES["ea3d_8"](), 1.5, 0.1),
}


@pytest.mark.parametrize("case", sorted(PAPER_CASES))
@pytest.mark.parametrize("precision", ["fp32", "fp64"])
@pytest.mark.parametrize("R", [64, 2048])
def test_paper_schedule_replay(case, precision, R):
    """The paper's scheduler (linear decrement, sweeps until d < d_min = 1e-4)
    by replay: the oracle runs the GPU's per-level sweep counts on 32 runs
    spread over the range and agrees within 1e-5 (fp32) / 1e-9 (fp64) on
    every well-conditioned run; a stop decision that differs has its oracle d
    within 1e-5 of d_min.  R = 2048 puts several runs in each workgroup, and
    up to four in each thread of the sparse solver, so that runs of one
    workgroup finish their levels at different sweeps."""
    M = _mars()
    make, hi, step = PAPER_CASES[case]
    inst = make()
    s = I.field_scale(inst)
    sch = I.Schedule(kind="linear", T_lo=0.0, T_hi=hi * s, c_step=step * s, max_sweeps=1000, d_min=1e-4,
                     precision=precision)
    cap = 64
    announce("graph paper schedule replay", case, precision, R)
    with M.Instance.from_inputs(inst) as g:
        out = g.solve_ex(R, sch, 41, want_m=True, levels_cap=cap)
    spl = out["sweeps_per_level"].cpu().numpy()
    res = out["result"]
    assert res["sweeps_executed"] == int(spl.sum())
    sample = list(range(0, R, max(1, R // 32)))[:32]
    check_replay(out["m"].cpu().numpy(), spl, inst, R, sch, 41, precision, sample,
                 label="%s %s R=%d" % (case, precision, R))


@pytest.mark.parametrize("name", ["er800", "er20000", "ea3d_L32"])
def test_full_size_sampled(name):
    """Paper-shaped sizes in the benchmark's launch configuration (all runs on
    the GPU), fp32 form: 32 sampled runs' final magnetisations within 1e-5 of
    the oracle's in every element of every well-conditioned run (at most 5 %
    excluded), decided spins equal and energies of equal spins equal."""
    M = _mars()
    w = I.workload(name, seed=1)
    R = w.runs
    sch = w.schedule.replace(precision="fp32")
    announce("graph full size", name, R)
    with M.Instance.from_inputs(w.instance) as g:
        out = g.solve_ex(R, sch, 1, want_m=True, want_spins=True)
    m = out["m"].cpu().numpy()
    S = out["spins"].cpu().numpy()
    E = out["energies"].cpu().numpy()
    excl = 0.0
    for r0 in (0, R // 3, R // 2 + 5, R - 8):
        ref = O.solve(w.instance, R, sch, 1, run_begin=r0, run_count=8)
        excl += c16_parity(m[:, r0:r0 + 8], w.instance, R, sch, 1, ref, "fp32", run_begin=r0, max_excluded=1.0,
                           label="%s fp32 runs %d..%d" % (name, r0, r0 + 7))
        _decided_spins_agree(S[r0:r0 + 8], m[:, r0:r0 + 8], ref, 1e-5)
        for q in range(8):
            if np.array_equal(S[r0 + q], ref["spins"][q]):
                assert E[r0 + q] == ref["energy"][q]
    assert excl / 4 <= 0.05
    assert out["result"]["best_energy"] == E.min()


@pytest.mark.parametrize("name", ["er20000", "ea3d_L32"])
def test_full_size_fp16_storage(name):
    """The fp16-storage form at full size (the benchmark's form): no
    elementwise bar (every stored value is rounded to fp16); on 32 sampled
    runs the fraction of rounded spins that differ from the FP64 oracle's (up
    to a global flip) stays below 2 % and the sample's best energy is within
    0.5 % of the oracle's."""
    M = _mars()
    w = I.workload(name, seed=1)
    R = w.runs
    announce("graph full size fp16", name, R)
    with M.Instance.from_inputs(w.instance) as g:
        out = g.solve_ex(R, w.schedule, 1, want_spins=True)
    S = out["spins"].cpu().numpy()
    E = out["energies"].cpu().numpy()
    mism, Eg, Eo = [], [], []
    for r0 in (0, R // 3, R // 2 + 5, R - 8):
        ref = O.solve(w.instance, R, w.schedule.replace(precision="fp64"), 1, run_begin=r0, run_count=8)
        d = np.mean(S[r0:r0 + 8] != ref["spins"], axis=1)
        d = np.minimum(d, np.mean(S[r0:r0 + 8] != -ref["spins"], axis=1))
        mism += d.tolist()
        Eg += E[r0:r0 + 8].tolist()
        Eo += ref["energy"].tolist()
    gap = (min(Eg) - min(Eo)) / abs(min(Eo))
    print("[fp16] %s: spin mismatch %.4f, best-energy gap %.2e" % (name, float(np.mean(mism)), gap), flush=True)
    assert np.mean(mism) <= 0.02 and gap <= 5e-3
    assert out["result"]["best_energy"] == E.min()


@pytest.mark.parametrize("lps", ["2", "4"])
@pytest.mark.parametrize("case", ["er_dense_isolated", "er_int8_dense", "er_field"])
def test_lane_split_variants(case, lps, monkeypatch):
    """The sparse solver with each slot's row split over 2 or 4 lanes
    (MARS_SPARSE_LPS), on long rows with isolated vertices, int8 weights and
    short rows with a field: one damped fp32 level (phased and synchronous)
    within 1e-5 of the oracle with a ragged run block, the fp16 storage bound
    of test_one_level_fp16_storage, and the paper's scheduler by replay (runs
    of one workgroup finishing levels at different sweeps)."""
    M = _mars()
    monkeypatch.setenv("MARS_SPARSE_LPS", lps)
    monkeypatch.delenv("MARS_SPARSE_VEC", raising=False)
    inst = CASES[case]()
    R = 1031
    for update in ("phased", "jacobi"):
        sch = _rel_sched(inst, precision="fp32", update=update, damping=0.5, level_count=1)
        announce("graph lane split damped", case, lps, update, R)
        with M.Instance.from_inputs(inst) as g:
            out = g.solve_ex(R, sch, 37, want_m=True)
        ref = O.solve(inst, R, sch, 37, run_count=R)
        err = np.max(np.abs(out["m"].cpu().numpy().astype(np.float64) - ref["m"]))
        assert err <= 1e-5, (update, err)
    test_one_level_fp16_storage(case, R)
    s = I.field_scale(inst)
    R = 2048
    sch = I.Schedule(kind="linear", T_lo=0.0, T_hi=2.0 * s, c_step=0.2 * s, max_sweeps=1000, d_min=1e-4,
                     precision="fp32")
    announce("graph lane split paper schedule", case, lps, R)
    with M.Instance.from_inputs(inst) as g:
        out = g.solve_ex(R, sch, 43, want_m=True, levels_cap=64)
    spl = out["sweeps_per_level"].cpu().numpy()
    assert out["result"]["sweeps_executed"] == int(spl.sum())
    sample = list(range(0, R, R // 32))[:32]
    check_replay(out["m"].cpu().numpy(), spl, inst, R, sch, 43, "fp32", sample,
                 label="%s lps=%s" % (case, lps))


@pytest.mark.parametrize("case", ["er_dense_isolated", "er_int8_dense"])
def test_lane_split_far_pairs(case, monkeypatch):
    """Two lanes per slot with at least eight run groups per workgroup (8200
    runs: 32 runs per workgroup, a ragged last block), where the two lanes of
    a pair sit eight lanes apart and exchange their partial fields by a row
    rotation: one damped fp32 level, phased and synchronous, within 1e-5 of
    the oracle, the fp16 storage bound, and the paper's scheduler by replay
    on 32 sampled runs (runs of one workgroup finishing levels at different
    sweeps)."""
    M = _mars()
    for name in ("MARS_SPARSE_LPS", "MARS_SPARSE_VEC", "MARS_SPARSE_RPW"):
        monkeypatch.delenv(name, raising=False)
    inst = CASES[case]()
    R = 8200
    for update in ("phased", "jacobi"):
        sch = _rel_sched(inst, precision="fp32", update=update, damping=0.5, level_count=1)
        announce("graph far pairs damped", case, update, R)
        with M.Instance.from_inputs(inst) as g:
            out = g.solve_ex(R, sch, 47, want_m=True)
        ref = O.solve(inst, R, sch, 47, run_count=R)
        err = np.max(np.abs(out["m"].cpu().numpy().astype(np.float64) - ref["m"]))
        assert err <= 1e-5, (update, err)
    test_one_level_fp16_storage(case, R)
    s = I.field_scale(inst)
    sch = I.Schedule(kind="linear", T_lo=0.0, T_hi=2.0 * s, c_step=0.2 * s, max_sweeps=1000, d_min=1e-4,
                     precision="fp32")
    announce("graph far pairs paper schedule", case, R)
    with M.Instance.from_inputs(inst) as g:
        out = g.solve_ex(R, sch, 53, want_m=True, levels_cap=64)
    spl = out["sweeps_per_level"].cpu().numpy()
    assert out["result"]["sweeps_executed"] == int(spl.sum())
    sample = list(range(0, R, R // 32))[:32]
    check_replay(out["m"].cpu().numpy(), spl, inst, R, sch, 53, "fp32", sample, label="%s far pairs" % case)
