"""Pins of the oracle's separate-component AMG for the displacement block
(Sec. 4.4: the mechanics AMG is built on the separate displacement component
approximation of A_uu, amg_unknown_based = 2).

* The F-relaxation AMG's level-0 operator is A_FF with every entry between
  unknowns of different field labels removed, checked against a numpy filter
  of the exported A_FF.
* Every level of that hierarchy stays decoupled by label (the unknown
  approach interpolates within a label, so the Galerkin products couple no
  two labels).
* With the couplings across labels removed from the system itself, options 1
  and 2 give the same hierarchy sizes and bit-identical applies (the filter is
  then the identity).
* The MGR_U solve with it converges on the fracturing system."""
import numpy as np
import pytest

import oracle as O
import workloads as W
from _systems import SMALL


def _mgr(s, aub, **kw):
    lv = [O.LevelOpts(fmask=7, frelax="amg", amg_unknown_based=aub, amg_agg_levels=kw.pop("agg", 0))]
    return O.MGR(s["b"], s["rp"], s["ci"], s["vals"], s["field"], lv, **kw)


def _f_labels(m, s):
    cf = m.export(0, 0, 0)          # 1 = C, 0 = F
    return np.asarray(s["field"])[np.flatnonzero(cf == 0)]


def _dense(c):
    A = np.zeros((c.nr, c.nc))
    for i in range(c.nr):
        A[i, c.ci[c.rp[i]:c.rp[i + 1]]] = c.v[c.rp[i]:c.rp[i + 1]]
    return A


def _pattern_labels_ok(c, lab):
    rows = np.repeat(np.arange(c.nr), np.diff(c.rp))
    return np.all(lab[rows] == lab[c.ci])


@pytest.mark.parametrize("agg", [0, 1])
def test_sdc_level0_is_filtered_aff(agg):
    s = SMALL["frac_12^3"]()
    m = _mgr(s, 2, agg=agg)
    assert m.status == 0
    aff = m.export(0, 0, 4)
    lab = _f_labels(m, s)
    a0 = m.export(2, 0, 1, sub=0)
    rows = np.repeat(np.arange(aff.nr), np.diff(aff.rp))
    keep = lab[rows] == lab[aff.ci]
    assert keep.sum() < len(keep)            # the block does couple the labels
    rp = np.concatenate([[0], np.cumsum(np.bincount(rows[keep], minlength=aff.nr))])
    assert np.array_equal(a0.rp, rp)
    assert np.array_equal(a0.ci, aff.ci[keep])
    assert np.array_equal(a0.v, aff.v[keep])


def test_sdc_hierarchy_decoupled_by_label():
    s = SMALL["frac_12^3"]()
    m = _mgr(s, 2, agg=1)
    lab = _f_labels(m, s)
    k = 0
    while True:
        try:
            a = m.export(2, k, 1, sub=0)
        except KeyError:
            break
        assert _pattern_labels_ok(a, lab), k
        try:
            cf = m.export(2, k, 0, sub=0)
        except KeyError:
            break
        p = m.export(2, k, 2, sub=0)
        lc = lab[np.flatnonzero(cf == 1)]
        rows = np.repeat(np.arange(p.nr), np.diff(p.rp))
        assert np.all(lab[rows] == lc[p.ci]), k   # interpolation within a label
        lab = lc
        k += 1
    assert k >= 2


def _decoupled_system(s):
    """The same system with the displacement block's couplings between different
    components removed (the pressure rows and columns untouched)."""
    b, rp, ci, vals = s["b"], np.asarray(s["rp"]), np.asarray(s["ci"]), np.asarray(s["vals"]).copy()
    field = np.asarray(s["field"])
    bl = vals.reshape(-1, b, b)
    for I in range(len(rp) - 1):
        for p in range(rp[I], rp[I + 1]):
            J = ci[p]
            for r in range(b):
                fr = field[I * b + r]
                for c in range(b):
                    fc = field[J * b + c]
                    if fr < 3 and fc < 3 and fr != fc:
                        bl[p, r, c] = 0.0
    return dict(s, vals=bl.reshape(-1))


def test_sdc_is_identity_without_cross_couplings():
    s = _decoupled_system(SMALL["frac_12^3"]())
    v = np.random.default_rng(2).standard_normal(s["n"])
    m1, m2 = _mgr(s, 1), _mgr(s, 2)
    assert m1.status == 0 and m2.status == 0
    assert m1.info() == m2.info()
    np.testing.assert_array_equal(m1.apply(v), m2.apply(v))


def test_sdc_converges_on_fracturing():
    s = SMALL["frac_18^3"]()
    m = _mgr(s, 2, agg=1, nu_pre=1, nu_post=1, smoother="hybrid-gs", chunk=32)
    x, info = m.solve(s["rhs"])
    A = W.csr_of(s)
    assert info.status == 0
    assert np.linalg.norm(s["rhs"] - A @ x) <= 1e-8 * np.linalg.norm(s["rhs"])
