"""Shared helpers for the tests: oracle results on the seeded workloads."""

import functools

import numpy as np

from oracle import factor, selinv, symbolic
from workloads import config


@functools.lru_cache(maxsize=None)
def workload(name, scale=None, batch=None):
    return config(name, scale=scale, batch=batch)


@functools.lru_cache(maxsize=None)
def oracle_sym(name, scale=None, batch=None, relax=0.0):
    w = workload(name, scale, batch)
    return symbolic.analyze(w.n, w.colptr, w.rowind, w.perm, cap=w.cap, relax=relax)


@functools.lru_cache(maxsize=None)
def oracle_x(name, scale=None, batch=None, relax=0.0):
    """Flattened oracle X panels [batch, panel_elems] (Alg. 1; for an LU
    workload the X set followed by the X^T set)."""
    w = workload(name, scale, batch)
    sym = oracle_sym(name, scale, batch, relax)
    h = w.is_hermitian
    out = []
    if w.is_lu:  # both panel sets: X on the pattern of L, then X^T (Alg. 1, LU form)
        for l in range(w.batch):
            PL, PU = factor.factor_lu(sym, w.lower_values[l], w.upper_values[l])
            XL, XU = selinv.alg1_lu(sym, *factor.normalize_lu(sym, PL, PU))
            out.append(np.concatenate([selinv.flatten(sym, XL), selinv.flatten(sym, XU)]))
        return np.stack(out)
    for l in range(w.batch):
        P = factor.factor(sym, w.values[l], herm=h)
        lh, dt = factor.normalize(sym, P, herm=h)
        out.append(selinv.flatten(sym, selinv.alg1(sym, lh, dt, herm=h)))
    return np.stack(out)


def maxrel(a, b):
    """max |a - b| / max |b| (complex modulus), the normwise max-norm error."""
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))
