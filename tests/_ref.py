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
    """Flattened oracle X panels [batch, panel_elems] (Alg. 1)."""
    w = workload(name, scale, batch)
    sym = oracle_sym(name, scale, batch, relax)
    h = w.is_hermitian
    out = []
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
