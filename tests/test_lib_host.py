"""Library host code vs the oracle: symbolic bit-exact, host LDL^T to rounding."""

import numpy as np
import pytest

from oracle import factor, selinv, symbolic
from tests._ref import oracle_sym, workload
from workloads import random_pattern


def lib_ctx(w, relax, cap=None):
    from paper_1604_02528_amd import SelInv

    return SelInv(w.n, w.colptr, w.rowind, w.perm, dtype=w.dtype, batch=w.batch,
                  cap=cap or w.cap, relax=relax, device="cpu")


def assert_same_symbolic(lib, sym):
    assert lib["nsuper"] == sym.nsuper
    for key, ref in [("parent", sym.parent), ("colcount", sym.colcount), ("xsuper", sym.xsuper),
                     ("sparent", sym.sparent), ("seg_ptr", sym.seg_ptr), ("seg_super", sym.seg_super),
                     ("seg_start", sym.seg_start), ("seg_posoff", sym.seg_posoff), ("posarr", sym.posarr)]:
        assert np.array_equal(lib[key], ref), key
    rows = np.concatenate(sym.rows) if sym.rows else np.zeros(0, np.int64)
    assert np.array_equal(lib["rowind_L"], rows)
    assert lib["nnzL"] == sym.nnzL()


# the last three are the full benchmark sizes (40^3, 30^3 with 32 shifts, 64^3 with 8 shifts)
SYM_CASES = [("C1", None, None), ("C4s", None, None), ("C2", 16, None), ("C3", 10, 2), ("C5", 8, 1),
             ("C4", None, None), ("C2", None, None), ("C3", None, None), ("C5", None, None)]


@pytest.mark.parametrize("relax", [0.0, 0.05])
@pytest.mark.parametrize("name,scale,batch", SYM_CASES)
def test_symbolic_bit_exact(name, scale, batch, relax):
    w = workload(name, scale, batch)
    sym = oracle_sym(name, scale, batch, relax)
    assert_same_symbolic(lib_ctx(w, relax).symbolic(), sym)


@pytest.mark.parametrize("seed", range(30))
def test_symbolic_bit_exact_random(seed):
    rng = np.random.default_rng(1000 + seed)
    n = int(rng.integers(2, 200))
    colptr, rowind, vals = random_pattern(n, float(rng.uniform(0.005, 0.2)), rng)
    perm = rng.permutation(n).astype(np.int64)
    cap = int(rng.integers(1, 40))
    relax = float(rng.choice([0.0, 0.05, 0.3]))
    sym = symbolic.analyze(n, colptr, rowind, perm, cap=cap, relax=relax)
    from paper_1604_02528_amd import SelInv

    S = SelInv(n, colptr, rowind, perm, cap=cap, relax=relax, device="cpu")
    assert_same_symbolic(S.symbolic(), sym)


@pytest.mark.parametrize("relax", [0.0, 0.05])
@pytest.mark.parametrize("name,scale,batch", [("C1", None, None), ("C2", 12, None), ("C3", 8, 2), ("C5", 6, 2)])
def test_host_factor_matches_oracle(name, scale, batch, relax):
    w = workload(name, scale, batch)
    sym = oracle_sym(name, scale, batch, relax)
    S = lib_ctx(w, relax)
    P = S.factor_host(w.values)[:, S.packed_index()]
    mask = np.concatenate([np.tril(np.ones((sym.width(K) + sym.rows[K].shape[0], sym.width(K)), bool)).reshape(-1, order="F")
                           for K in range(sym.nsuper)])
    for l in range(w.batch):
        ref = selinv.flatten(sym, factor.factor(sym, w.values[l]))
        err = np.max(np.abs(P[l][mask] - ref[mask])) / np.max(np.abs(ref[mask]))
        assert err < 1e-13
        ld = S.logdet()[l]
        ref_ld = factor.logdet(sym, factor.factor(sym, w.values[l]))
        assert abs(ld - ref_ld) <= 1e-10 * max(1.0, abs(ref_ld))


@pytest.mark.parametrize("name,scale,batch,relax", [("C1", None, None, 0.0), ("C2", 12, None, 0.0),
                                                     ("C2", None, None, 0.05), ("C3", 8, 3, 0.05),
                                                     ("C5", 6, 2, 0.0), ("C3", None, None, 0.05),
                                                     ("H3", None, None, 0.05)])
def test_scheduler_plan_replay(name, scale, batch, relax):
    """Host replay of the persistent scheduler's protocol: every item becomes
    ready exactly once, after all of its dependencies, within queue capacity;
    and the normalization chunks of selinv_normalize_run cover every list and
    level launch in order, each launch after its nodes' chunk (the full C3 and
    H3 plans have several chunks)."""
    from paper_1604_02528_amd import capi

    w = workload(name, scale, batch)
    S = lib_ctx(w, relax)
    capi.selinv_check_plan(S.h)


@pytest.mark.parametrize("relax", [0.0, 0.05])
@pytest.mark.parametrize("scale,batch", [(6, 2), (10, 3)])
def test_host_factor_hermitian_matches_oracle(scale, batch, relax):
    """The library's host LDL^H (dtype h128) against the oracle's Hermitian
    factorization, and its log det (real for these positive definite shifts)."""
    from paper_1604_02528_amd import SelInv

    w = workload("H3", scale, batch)
    sym = oracle_sym("H3", scale, batch, relax)
    S = SelInv(w.n, w.colptr, w.rowind, w.perm, dtype="h128", batch=w.batch, cap=w.cap, relax=relax, device="cpu")
    P = S.factor_host(w.values)[:, S.packed_index()]
    mask = np.concatenate([np.tril(np.ones((sym.width(K) + sym.rows[K].shape[0], sym.width(K)), bool)).reshape(-1, order="F")
                           for K in range(sym.nsuper)])
    for l in range(w.batch):
        Pref = factor.factor(sym, w.values[l], herm=True)
        ref = selinv.flatten(sym, Pref)
        err = np.max(np.abs(P[l][mask] - ref[mask])) / np.max(np.abs(ref[mask]))
        assert err < 1e-13
        ld = S.logdet()[l]
        ref_ld = factor.logdet(sym, Pref)
        assert abs(ld.real - np.real(ref_ld)) <= 1e-10 * max(1.0, abs(ref_ld))
        assert abs(ld.imag) <= 1e-10


@pytest.mark.parametrize("seed", range(6))
def test_host_factor_hermitian_random_permuted(seed):
    """Random Hermitian patterns under random permutations: the entries that
    the permutation moves into the upper triangle enter conjugated."""
    from paper_1604_02528_amd import SelInv
    from tests.test_oracle_hermitian import hermitian_random
    from oracle import symbolic

    rng = np.random.default_rng(700 + seed)
    n = int(rng.integers(20, 120))
    colptr, rowind, v = hermitian_random(n, 0.08, rng, indefinite=bool(seed % 2))
    perm = rng.permutation(n).astype(np.int64)
    cap = int(rng.integers(2, 30))
    sym = symbolic.analyze(n, colptr, rowind, perm, cap=cap)
    S = SelInv(n, colptr, rowind, perm, dtype="h128", batch=1, cap=cap, relax=0.0, device="cpu")
    P = S.factor_host(v[None, :])[:, S.packed_index()]
    ref = selinv.flatten(sym, factor.factor(sym, v, herm=True))
    mask = np.concatenate([np.tril(np.ones((sym.width(K) + sym.rows[K].shape[0], sym.width(K)), bool)).reshape(-1, order="F")
                           for K in range(sym.nsuper)])
    assert np.max(np.abs(P[0][mask] - ref[mask])) <= 1e-13 * np.max(np.abs(ref[mask]))


def _lower_mask(sym):
    return np.concatenate([np.tril(np.ones((sym.width(K) + sym.rows[K].shape[0], sym.width(K)), bool)).reshape(-1, order="F")
                           for K in range(sym.nsuper)])


@pytest.mark.parametrize("relax", [0.0, 0.05])
@pytest.mark.parametrize("scale,batch", [(6, 2), (10, 2)])
def test_host_factor_lu_matches_oracle(scale, batch, relax):
    """The library's host L D U (dtype lu64): both panel sets against the
    oracle's factor_lu, and the log det."""
    from paper_1604_02528_amd import SelInv

    w = workload("U3", scale, batch)
    sym = oracle_sym("U3", scale, batch, relax)
    S = SelInv(w.n, w.colptr, w.rowind, w.perm, dtype="lu64", batch=w.batch, cap=w.cap, relax=relax, device="cpu")
    P = S.factor_host(w.values)[:, S.packed_index()]
    mask = _lower_mask(sym)
    half = mask.size
    for l in range(w.batch):
        PL, PU = factor.factor_lu(sym, w.lower_values[l], w.upper_values[l])
        for got, ref in ((P[l][:half], selinv.flatten(sym, PL)), (P[l][half:], selinv.flatten(sym, PU))):
            err = np.max(np.abs(got[mask] - ref[mask])) / np.max(np.abs(ref[mask]))
            assert err < 1e-13
        ld = S.logdet()[l]
        ref_ld = factor.logdet(sym, PL)
        assert abs(ld - np.real(ref_ld)) <= 1e-10 * max(1.0, abs(ref_ld))


@pytest.mark.parametrize("seed", range(6))
def test_host_factor_lu_random_permuted(seed):
    """Random unsymmetric values on random symmetric patterns under random
    permutations: an entry moved into B's upper triangle trades its value with
    its mirror."""
    from paper_1604_02528_amd import SelInv
    from tests.test_oracle_lu import unsymmetric_random

    rng = np.random.default_rng(1700 + seed)
    n = int(rng.integers(20, 120))
    colptr, rowind, lo, up = unsymmetric_random(n, 0.08, rng)
    perm = rng.permutation(n).astype(np.int64)
    cap = int(rng.integers(2, 30))
    sym = symbolic.analyze(n, colptr, rowind, perm, cap=cap)
    S = SelInv(n, colptr, rowind, perm, dtype="lu64", batch=1, cap=cap, relax=0.0, device="cpu")
    P = S.factor_host(np.concatenate([lo, up])[None, :])[:, S.packed_index()]
    PL, PU = factor.factor_lu(sym, lo, up)
    mask = _lower_mask(sym)
    half = mask.size
    for got, ref in ((P[0][:half], selinv.flatten(sym, PL)), (P[0][half:], selinv.flatten(sym, PU))):
        assert np.max(np.abs(got[mask] - ref[mask])) <= 1e-13 * np.max(np.abs(ref[mask]))


def test_lu_plan_replay_and_refusals():
    """An LU plan passes the scheduler replay; the paths the LU form does not
    have are refused (schedules other than levels at analyze time)."""
    from paper_1604_02528_amd import SelInv, capi

    w = workload("U3", 8, 2)
    S = SelInv(w.n, w.colptr, w.rowind, w.perm, dtype="lu64", batch=w.batch, cap=w.cap, relax=0.05, device="cpu")
    capi.selinv_check_plan(S.h)
    R = SelInv(w.n, w.colptr, w.rowind, w.perm, dtype="f64", batch=w.batch, cap=w.cap, relax=0.05, device="cpu")
    assert S.panel_elems == 2 * R.panel_elems  # two panel sets of the symmetric layout
    assert S.packed_index().size == 2 * R.packed_index().size
    for sched in ("persistent", "push"):
        with pytest.raises(capi.SelinvError) as ei:
            SelInv(w.n, w.colptr, w.rowind, w.perm, dtype="lu64", batch=w.batch, cap=w.cap, sched=sched, device="cpu")
        assert ei.value.status == 7


@pytest.mark.parametrize("sched", ["persistent", "push"])
@pytest.mark.parametrize("name,scale", [("C2", 12), ("C3", 8), ("H3", 8)])
def test_plan_check_other_schedules(name, scale, sched):
    """The plan check (ticket replay, normalization chunks) on the persistent
    and push plans too; they have a single normalization chunk."""
    from paper_1604_02528_amd import SelInv, capi

    w = workload(name, scale)
    S = SelInv(w.n, w.colptr, w.rowind, w.perm, dtype=w.dtype, batch=w.batch, cap=w.cap, relax=0.05, sched=sched,
               device="cpu", adjoint=False)
    capi.selinv_check_plan(S.h)
    assert len(capi.selinv_items(S.h, 3)) == 1
