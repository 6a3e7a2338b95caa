"""Planted mistakes in the oracle must be caught by the pins.

Each case edits one expression of the oracle's source (a dropped term, a sign,
a transposed or conjugated operand), loads the edited copy as a separate
module on the CPU, and checks that the Petrov-Galerkin closed form (Table 1,
eq. 1.3) or the true-residual identity (section 2.2) rejects it.  The real
oracle is never modified.
"""
from __future__ import annotations

import itertools
import os
import sys
import types

import numpy as np
import pytest

from oracle import blk_oracle as O
from tests import pins

SRC = open(os.path.join(os.path.dirname(O.__file__), "blk_oracle.py")).read()

MUTANTS = [
    # (id, methods it affects, original text, replacement)
    ("conjugated-gram", ["cocg", "cocr", "cocg_rq", "cocr_rq"], "return Y.T @ Z", "return Y.conj().T @ Z"),
    ("x-update-drops-xi", ["cocg_rq", "cocr_rq"], "X = X + S @ (alpha @ xi)", "X = X + S @ alpha"),
    ("beta-drops-tauT", ["cocg_rq"], "beta = solve(gqq, tau.T @ gn)", "beta = solve(gqq, gn)"),
    ("beta-tau-not-transposed", ["cocr_rq"], "beta = solve(gqv, tau.T @ gn)", "beta = solve(gqv, tau @ gn)"),
    ("w-sign", ["cocr_rq"], "W = Q - U @ alpha", "W = Q + U @ alpha"),
    ("cocg-r-sign", ["cocg"], "R = R - Z @ alpha", "R = R + Z @ alpha"),
    ("cocr-u-drops-beta", ["cocr"], "U = Vn + U @ beta", "U = Vn + U"),
    ("cocg-swapped-solve", ["cocg"], "alpha = solve(gram_t(P, Z), rho)", "alpha = solve(rho, gram_t(P, Z))"),
    ("qr-r-transposed", ["cocg_rq", "cocr_rq"], "R = R / ph[:, None]", "R = R.T / ph[:, None]"),
    ("xi-order", ["cocg_rq", "cocr_rq"], "return Qn, tau, tau @ xi", "return Qn, tau, xi @ tau"),
    ("cocr-residual-wrong-block", ["cocr"], "Rn = R - U @ alpha", "Rn = R - V @ alpha"),
    ("cocg-beta-index", ["cocg"], "beta = solve(rho, rho_n)", "beta = solve(rho_n, rho)"),
]


_COUNTER = itertools.count()


def _load_mutant(old: str, new: str) -> types.ModuleType:
    assert SRC.count(old) >= 1, old
    name = f"blk_oracle_mutant_{next(_COUNTER)}"
    mod = types.ModuleType(name)
    sys.modules[name] = mod  # dataclasses resolve annotations through sys.modules
    exec(compile(SRC.replace(old, new), name, "exec"), mod.__dict__)
    return mod


def _pin_error(mod, method: str) -> float:
    n, p = 40, 2
    A = pins.well_conditioned_cs(n, 5)
    rng = np.random.default_rng(6)
    B = rng.standard_normal((n, p)) + 1j * rng.standard_normal((n, p))
    try:
        r = mod.solve_block(method, A, B, tol=1e-30, maxit=4, record=True)
    except Exception:
        return np.inf
    err = 0.0
    for m in range(len(r.Xs)):
        ref = pins.petrov_galerkin_iterate(A, B, np.zeros_like(B), m, method)
        err = max(err, pins.rel(r.Xs[m], ref))
        true = np.linalg.norm(B - A @ r.Xs[m]) / np.linalg.norm(B)
        if m < len(r.hist):
            err = max(err, abs(r.hist[m] - true) / true)
    if len(r.Xs) < 5:
        err = np.inf
    return err


@pytest.mark.parametrize("method", ["cocg", "cocr", "cocg_rq", "cocr_rq"])
def test_unmodified_oracle_passes(method):
    assert _pin_error(_load_mutant("", ""), method) < 1e-11


@pytest.mark.parametrize("mid,methods,old,new", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_mutant_is_caught(mid, methods, old, new):
    mod = _load_mutant(old, new)
    for method in methods:
        assert _pin_error(mod, method) > 1e-6, (mid, method)
