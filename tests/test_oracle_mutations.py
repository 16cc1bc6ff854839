"""Planted mistakes: a copy of an oracle module with one plausible slip
(transposed fold, dropped factor, wrong index, wrong key word) must fail the
pin that guards that part.  Mistakes are planted only in these CPU copies."""

import importlib.util
import os
import types

import numpy as np
import pytest

import oracle
import workloads as wk
from oracle import philox, plan, randorth, rounding, tt

ORACLE_DIR = os.path.dirname(oracle.__file__)


def _mutant(modname: str, old: str, new: str) -> types.ModuleType:
    src = open(os.path.join(ORACLE_DIR, modname + ".py")).read()
    assert src.count(old) == 1, f"mutation anchor not unique in {modname}: {old!r}"
    src = src.replace(old, new)
    mod = types.ModuleType(f"oracle._mutant_{modname}")
    mod.__package__ = "oracle"
    exec(compile(src, f"<mutant {modname}>", "exec"), mod.__dict__)
    return mod


def _pair(seed, n, r, s):
    rng = np.random.default_rng(seed)
    return (wk.gaussian_tt(rng, n, wk.feasible_ranks(n, r)),
            wk.gaussian_tt(rng, n, wk.feasible_ranks(n, s)))


def _hatt_vs_randorth(hmod, ell=5, n=(4, 5, 4, 5), r=3, s=3):
    y, z = _pair(3, list(n), r, s)
    l = plan.clamp_ell(tt.modes(y), tt.ranks(y), tt.ranks(z), ell)
    R = philox.sketch(2, tt.modes(y), l)
    return tt.rel_err(hmod.hatt(y, z, R), randorth.randorth(tt.pkp(y, z), R))


@pytest.mark.parametrize("old,new", [
    ('"xa,yb,abg->xyg"', '"xa,yb,bag->xyg"'),        # transposed U_gamma fold in HPCRL
    ('"gab,ax,by->gxy"', '"gba,ax,by->gxy"'),        # transposed M_gamma fold in the update
    ("rt[c][:, i, :]", "rt[c][:, n - 1 - i, :]"),    # wrong sketch slice in W_R
    ("m = q.T @ xm", "m = q.T @ (xm * 1.0001)"),     # perturbed projection
])
def test_hatt_mutants_break_randorth_identity(old, new):
    assert _hatt_vs_randorth(oracle.hatt) < 1e-13
    assert _hatt_vs_randorth(_mutant("hatt", old, new)) > 1e-8


@pytest.mark.parametrize("old,new", [
    ("(s[:rho, None] * vt[:rho, :])", "(vt[:rho, :])"),          # dropped Sigma
    ("if tail <= delta * delta:", "if tail <= delta:"),          # tolerance not squared
])
def test_rounding_mutants_break_tt_svd_agreement(old, new):
    y, z = wk.tiny_pair(5)
    a = tt.pkp(y, z)
    fz = tt.full(a)
    mod = _mutant("rounding", old, new)

    def bad(rmod):
        b = rmod.tt_round(a, tol=3e-2)
        c = rounding.tt_svd(fz, tol=3e-2)
        return tt.ranks(b) != tt.ranks(c) or np.linalg.norm(tt.full(b) - tt.full(c)) > 1e-10 * np.linalg.norm(fz)

    assert not bad(rounding)
    assert bad(mod)


def test_pkp_index_mutant_breaks_bruteforce():
    y, z = wk.tiny_pair(3)
    mod = _mutant("tt", "np.kron(y[:, i, :], z[:, i, :])", "np.kron(y[:, i, :], z[:, n - 1 - i, :])")
    fz = tt.full(y) * tt.full(z)
    assert np.allclose(tt.full(tt.pkp(y, z)), fz)
    assert not np.allclose(mod.full(mod.pkp(y, z)), fz)


def test_philox_key_mutant_breaks_known_answers():
    mod = _mutant("philox", "(hi1 ^ c1 ^ k0)", "(hi1 ^ c1 ^ k1)")
    v = [0x243F6A88, 0x85A308D3, 0x13198A2E, 0x03707344, 0xA4093822, 0x299F31D0]
    good = [int(o) for o in philox.philox4x32_10(*v)]
    bad = [int(o) for o in mod.philox4x32_10(*v)]
    assert good == [0xD16CFE09, 0x94FDCCEB, 0x5001E420, 0x24126EA1]
    assert bad != good
