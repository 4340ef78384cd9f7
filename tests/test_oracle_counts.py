"""Pins of the exact-integer triangle counts (oracle/counts.py) against brute-force enumeration.

The count of closed grid triangles of a bin triple (Sec. 3.2, the N_tri that Eq. iFT_I gives
as N^2 sum I1 I2 I3) is fixed by its definition: enumerate k1 in bin a and k2 in bin b, set
k3 = -(k1 + k2) mod the grid and test k3 in bin c.  oracle.brute does exactly that; the pair
convolution route must give the same integers, and so must the float64 triple-sum route of
the estimator after rounding.  A planted mistake (the mirror half of the grid left out of the
indicators) must make the comparison fail.
"""
import numpy as np
import pytest

from oracle import bins as ob
from oracle import brute as obr
from oracle import counts as oc
from oracle import estimator as oe
from paper_2506_10526_amd import synth


def _brute_count(bins, tri3, uv_unit=None):
    (f1, f2, f3), shape = obr.closed_triangles(bins, tri3)
    if uv_unit is None:
        return len(f1)
    m = obr.full_plane(np.asarray(uv_unit, dtype=np.complex128), bins.n).real
    if bins.kind == ob.SHELL_K:
        m = np.broadcast_to(m[None], shape)
    m = m.ravel()
    return int(np.sum(m[f1] * m[f2] * m[f3]))


def _random_uv_unit(n, seed):
    """Random 0/1 occupancy on the half plane, consistent on the self-conjugate column v = 0."""
    rng = np.random.default_rng(seed)
    m = (rng.random((n, n // 2 + 1)) < 0.8).astype(np.uint8)
    qu = ob.signed_index(n)
    m[:, 0] = np.maximum(m[:, 0], m[(-qu) % n, 0])
    return m


@pytest.mark.parametrize("mask", [False, True])
def test_shell_counts_match_brute_force(mask):
    n, nc = 12, 8
    edges = 2 * np.pi * np.geomspace(1 / n, 4.2 / n, 6)
    b = ob.make_bins(ob.SHELL_K, n, nc, edges, du=1.0, r_mpc=float(n), rprime=1.0, dnu=float(n) / nc)
    uv = _random_uv_unit(n, 3) if mask else None
    T, dev = oc.exact_counts(b, uv)
    assert dev < 1e-9
    ref = np.array([_brute_count(b, t, uv) for t in b.triangles], dtype=np.int64)
    assert np.array_equal(T, ref)
    assert (T > 0).sum() >= 5
    # the float64 triple-sum route of the estimator rounds to the same integers
    V = synth.make_cube(synth.small_workload(n, nc), seed=1)
    _, T3, _, _, dev3 = oe.estimate_3d(b, V, oe.Weights(uv_mask=uv))
    assert dev3 < 1e-6
    assert np.array_equal(T3, T)


@pytest.mark.parametrize("mask", [False, True])
def test_ring_counts_match_brute_force(mask):
    n = 16
    edges = np.geomspace(1.0, 6.0, 6)
    b = ob.make_bins(ob.RING_U, n, 4, edges)
    uv = _random_uv_unit(n, 5) if mask else None
    T, dev = oc.exact_counts(b, uv)
    assert dev < 1e-9
    ref = np.array([_brute_count(b, t, uv) for t in b.triangles], dtype=np.int64)
    assert np.array_equal(T, ref)
    # the MABS count of a channel triple with unit channel weights is the same T_perp
    V = synth.make_cube(synth.small_workload(n, 4), seed=2)
    _, N, _, _ = oe.estimate_mabs(b, V, oe.Weights(uv_mask=uv), nu1=[0])
    assert np.array_equal(N[:, 0, 1, 2], T)


def test_counts_with_aliasing_closure():
    """umax beyond (n - 1) / 3: closure is mod n, and the counts follow the cyclic definition."""
    n = 12
    edges = np.geomspace(1.0, 6.0, 5)
    b = ob.make_bins(ob.RING_U, n, 2, edges, umax=5.0)
    assert not b.true_closure
    T, _ = oc.exact_counts(b)
    ref = np.array([_brute_count(b, t) for t in b.triangles], dtype=np.int64)
    assert np.array_equal(T, ref)


def test_planted_missing_mirror_half_fails(monkeypatch):
    n, nc = 12, 8
    edges = 2 * np.pi * np.geomspace(1 / n, 4.2 / n, 6)
    b = ob.make_bins(ob.SHELL_K, n, nc, edges, du=1.0, r_mpc=float(n), rprime=1.0, dnu=float(n) / nc)
    ref = np.array([_brute_count(b, t) for t in b.triangles], dtype=np.int64)
    orig = oc.full_indicator

    def half_only(bins, j, uv_unit=None):
        x = orig(bins, j, uv_unit)
        x[..., bins.n // 2 + 1:] = 0.0
        return x

    monkeypatch.setattr(oc, "full_indicator", half_only)
    T, _ = oc.exact_counts(b)
    assert not np.array_equal(T, ref)
