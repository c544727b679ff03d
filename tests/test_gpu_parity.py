"""GPU selected inversion vs the CPU oracle (element by element on the panels)."""

import numpy as np
import pytest
import torch

from tests._ref import maxrel, oracle_x, workload

CASES = [
    # (name, scale, batch, relax)
    ("C1", None, None, 0.0),
    ("C4s", None, None, 0.0),
    ("C2", 12, None, 0.0),
    ("C2", 12, None, 0.05),
    ("C2", 20, None, 0.05),
    ("C3", 8, 2, 0.05),
    ("C5", 6, 2, 0.05),
]


@pytest.mark.gpu
@pytest.mark.parametrize("sched", ["levels", "persistent"])
@pytest.mark.parametrize("name,scale,batch,relax", CASES)
def test_selinv_matches_oracle(name, scale, batch, relax, sched):
    from paper_1604_02528_amd import SelInv

    w = workload(name, scale, batch)
    print(f"case {name} scale={scale} batch={batch} relax={relax} sched={sched}", flush=True)
    S = SelInv(w.n, w.colptr, w.rowind, w.perm, dtype="c128" if w.is_complex else "f64", batch=w.batch,
               cap=w.cap, relax=relax, sched=sched, watchdog_ms=20000)
    S.factor(w.values)
    S.run()
    S.sync()
    X = S.to_host("x")
    ref = oracle_x(name, scale, batch, relax)
    tol = 1e-9 if w.is_complex else 1e-10
    for l in range(w.batch):
        err = maxrel(X[l], ref[l])
        print(f"  matrix {l}: max-norm rel err {err:.3e}", flush=True)
        assert err <= tol
