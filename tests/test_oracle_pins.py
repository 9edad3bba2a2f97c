"""Pins of the CPU oracle to what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: numbers the
paper prints (golden fixtures), closed forms, exact invariants, special cases
that reduce to a textbook result, or an independent route (the paper's own
literal assembly, an eigendecomposition instead of expm).
"""
import math
import os
from itertools import combinations

import numpy as np
import pytest
import scipy.linalg as sla

from conftest import GOLDEN
from synth import ring, chain, two_site, cluster_2d, PulseParams, random_state
from oracle import (HubbardOracle, sector_states, apply_ladder, ladder_matrix,
                    pulse_A, ground_state, midpoint_step_exact, observables,
                    krylov_step_alg6, tridiag_expm_e1, canonical_map)
from oracle.fock import UP, DOWN, mode_index, docc_weights
from oracle.literal_csr import csr_upper, literal_H, alg2_structure
from oracle import freefermion as ff
from oracle.stepper import power_iteration_ground_state, expm_apply


def _read_table1():
    rows = []
    with open(os.path.join(GOLDEN, "table1_dimensions.txt")) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                ns, npsi, nnz = line.split()
                rows.append((int(ns), float(npsi), float(nnz)))
    return rows


def _round2(x):
    """Round to two significant digits as Table 1 prints them."""
    e = math.floor(math.log10(x))
    return round(x / 10 ** e, 1) * 10 ** e


# --------------------------------------------------------------------------
# basis and sparsity (Table 1, Eq. (statedim), Alg. 2)

@pytest.mark.parametrize("ns,npsi,nnz", [r for r in _read_table1() if r[0] <= 14])
def test_table1_sector_dimension(ns, npsi, nnz):
    dim = len(sector_states(ns, ns // 2, ns // 2)) if ns <= 12 else None
    if dim is None:  # 14 sites: count the tensor-product factors by enumeration
        dim = len(list(combinations(range(ns), ns // 2))) ** 2
    assert _round2(dim) == pytest.approx(npsi, rel=1e-12)


@pytest.mark.parametrize("ns,npsi,nnz", [r for r in _read_table1() if r[0] <= 8])
def test_table1_worst_case_nonzeros_from_alg2(ns, npsi, nnz):
    st = sector_states(ns, ns // 2, ns // 2)
    row, col = alg2_structure(st)
    assert row[-1] - 1 == len(col)
    assert _round2(len(col)) == pytest.approx(nnz, rel=1e-12)
    # every row's first stored entry is its diagonal (Sec. 3.2, Alg. 3 note)
    assert np.all(col[row[:-1] - 1] == np.arange(1, len(st) + 1))


def test_csr_worked_example():
    M = np.zeros((5, 5), dtype=complex)
    val_ref = col_ref = row_ref = None
    r = 0
    with open(os.path.join(GOLDEN, "csr_example.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            key, *nums = line.split()
            nums = [float(x) for x in nums]
            if key == "matrix":
                M[r] = [complex(nums[2 * k], nums[2 * k + 1]) for k in range(5)]
                r += 1
            elif key == "val":
                val_ref = np.array([complex(nums[2 * k], nums[2 * k + 1]) for k in range(len(nums) // 2)])
            elif key == "col":
                col_ref = np.array(nums, dtype=int)
            elif key == "row":
                row_ref = np.array(nums, dtype=int)
    assert np.allclose(M, M.conj().T)
    val, col, row = csr_upper(M)
    assert np.array_equal(val, val_ref)
    assert np.array_equal(col, col_ref)
    assert np.array_equal(row, row_ref)


# --------------------------------------------------------------------------
# ladder operators (Eq. (creation-annihilation))

def _full_fock(ns):
    return np.arange(4 ** ns, dtype=np.int64)


def test_ladder_anticommutators_full_fock():
    ns = 3
    st = _full_fock(ns)
    modes = range(2 * ns)
    c = {m: ladder_matrix(st, st, m, False).toarray() for m in modes}
    cd = {m: ladder_matrix(st, st, m, True).toarray() for m in modes}
    eye = np.eye(len(st))
    for a in modes:
        assert np.allclose(cd[a], c[a].T)  # real signs: c^dag is the transpose
        for b in modes:
            acomm = c[a] @ cd[b] + cd[b] @ c[a]
            assert np.array_equal(acomm, eye if a == b else 0 * eye)
            assert not np.any(c[a] @ c[b] + c[b] @ c[a])


def test_number_operator_and_docc_weights():
    ns = 3
    st = _full_fock(ns)
    w = docc_weights(st, ns)
    dsum = 0
    for i in range(ns):
        nu = (ladder_matrix(st, st, mode_index(i, UP), True)
              @ ladder_matrix(st, st, mode_index(i, UP), False)).toarray()
        nd = (ladder_matrix(st, st, mode_index(i, DOWN), True)
              @ ladder_matrix(st, st, mode_index(i, DOWN), False)).toarray()
        assert np.array_equal(np.diag(nu), (st >> mode_index(i, UP)) & 1)
        dsum = dsum + nu @ nd
    assert np.array_equal(np.diag(dsum), w)


def test_block_diagonal_on_full_fock_space():
    """Eq. (directsum): H only connects states with equal (n_up, n_down)."""
    ns = 4
    lat = ring(4).with_onsite([0.3, -0.2, 0.1, 0.0])
    full = HubbardOracle(lat, 3.0, 0, 0, states=_full_fock(ns))
    H = full.H(0.41).toarray()
    st = full.states
    nu = np.bitwise_count(st & 0x55).astype(int)
    nd = np.bitwise_count(st & 0xAA).astype(int)
    key = nu * 10 + nd
    assert not np.any(H[key[:, None] != key[None, :]])
    for (a, b) in [(2, 2), (1, 3), (3, 2)]:
        sec = HubbardOracle(lat, 3.0, a, b)
        idx = np.searchsorted(st, sec.states)
        assert np.allclose(H[np.ix_(idx, idx)], sec.H(0.41).toarray(), atol=0, rtol=0)


# --------------------------------------------------------------------------
# Hamiltonian closed forms and symmetries

def test_hermitian():
    h = HubbardOracle(cluster_2d(3, 2), 5.0, 3, 2)
    H = h.H(0.77).toarray()
    assert np.array_equal(H, H.conj().T)


@pytest.mark.parametrize("U,t,A", [(8.0, 1.0, 0.0), (4.0, 1.0, 0.3), (1.5, 0.7, -1.1), (0.0, 1.0, 0.5)])
def test_two_site_ground_energy(U, t, A):
    """Two sites, one electron of each spin: E0 = U/2 - sqrt(U^2/4 + 4 t^2)."""
    h = HubbardOracle(two_site(t), U, 1, 1)
    E0 = np.linalg.eigvalsh(h.H(A).toarray())[0]
    assert E0 == pytest.approx(U / 2 - math.sqrt(U * U / 4 + 4 * t * t), abs=1e-13)


@pytest.mark.parametrize("L,nu,nd,A", [(6, 3, 2, 0.0), (6, 2, 2, 0.37), (5, 2, 3, -0.8)])
def test_free_ring_spectrum_is_sum_of_plane_wave_levels(L, nu, nd, A):
    """U = 0 ring: one-particle levels -2t cos(k - A), k = 2 pi n / L (plane
    waves; fixes the Peierls sign convention); the many-body spectrum is every
    sum of n_up + n_down distinct-per-spin levels."""
    h = HubbardOracle(ring(L), 0.0, nu, nd)
    ev = np.sort(np.linalg.eigvalsh(h.H(A).toarray()))
    eps = [-2.0 * math.cos(2 * math.pi * n / L - A) for n in range(L)]
    sums = sorted(sum(eps[k] for k in cu) + sum(eps[k] for k in cd)
                  for cu in combinations(range(L), nu) for cd in combinations(range(L), nd))
    assert np.allclose(ev, sums, atol=1e-12)


def test_peierls_plane_wave_eigenvector():
    """A single up electron in plane wave k on a ring is an eigenstate with
    energy -2t cos(k - A) (and not cos(k + A))."""
    L, A, k = 7, 0.6, 2 * math.pi * 2 / 7
    h = HubbardOracle(ring(L), 3.0, 1, 0)
    x = np.array([np.exp(1j * k * i) for i in range(L)]) / math.sqrt(L)
    # basis states are single up electrons on site i = bit 2i; ascending order = site order
    assert np.array_equal(h.states, [1 << (2 * i) for i in range(L)])
    y = h.apply(A, x)
    assert np.allclose(y, -2 * math.cos(k - A) * x, atol=1e-14)


def test_no_hopping_spectrum_is_U_times_doublons():
    lat = cluster_2d(3, 2).with_hopping(0.0)
    h = HubbardOracle(lat, 6.5, 3, 3)
    ev = np.sort(np.linalg.eigvalsh(h.H(0.9).toarray()))
    assert np.allclose(ev, np.sort(6.5 * docc_weights(h.states, 6)), atol=1e-13)


@pytest.mark.parametrize("lat,A", [(ring(6), 0.0), (chain(6), 0.83), (ring(4), 0.0)])
def test_half_filled_bipartite_spectrum_symmetric(lat, A):
    """Particle-hole symmetry at half filling on a bipartite lattice (a ring
    only at A = 0): the spectrum is symmetric about U Ns / 4."""
    ns, U = lat.n_sites, 5.0
    h = HubbardOracle(lat, U, ns // 2, ns // 2)
    ev = np.sort(np.linalg.eigvalsh(h.H(A).toarray()))
    c = U * ns / 4
    assert np.allclose(ev - c, -(ev - c)[::-1], atol=1e-11)


def test_open_chain_constant_field_is_pure_gauge():
    h = HubbardOracle(chain(6), 4.0, 3, 2)
    e0 = np.linalg.eigvalsh(h.H(0.0).toarray())
    for A in (0.4, 1.3, -2.2):
        assert np.allclose(np.linalg.eigvalsh(h.H(A).toarray()), e0, atol=1e-12)


def test_ring_spectrum_flux_period_and_parity():
    L = 6
    h = HubbardOracle(ring(L), 4.0, 3, 3)
    A = 0.29
    e = np.linalg.eigvalsh(h.H(A).toarray())
    assert np.allclose(np.linalg.eigvalsh(h.H(A + 2 * math.pi / L).toarray()), e, atol=1e-11)
    assert np.allclose(np.linalg.eigvalsh(h.H(-A).toarray()), e, atol=1e-11)
    # the pulse does something: a generic A changes the spectrum
    assert not np.allclose(np.linalg.eigvalsh(h.H(0.0).toarray()), e, atol=1e-6)


@pytest.mark.parametrize("lat", [ring(6), cluster_2d(3, 2), chain(5)])
def test_literal_alg2_alg3_assembly_matches_ladder_products(lat):
    """The paper's own assembly route (Alg. 2 pattern, Alg. 3 values with the
    sign of Eq. (sign-explanation), split of Eq. (hamimplementation)) gives
    the same matrix as products of ladder operators."""
    ns = lat.n_sites
    h = HubbardOracle(lat, 2.5, ns // 2, (ns + 1) // 2)
    for A in (0.0, 0.61):
        Hl, _ = literal_H(h.states, ns, 2.5, lat.bonds, A)
        assert np.allclose(Hl, h.H(A).toarray(), atol=1e-15)


def test_hamiltonian_row_matches_matrix():
    h = HubbardOracle(cluster_2d(3, 2), 4.0, 3, 3)
    H = h.H(0.7).toarray()
    for k in (0, 17, 199, h.dim - 1):
        cols, vals = h.row(0.7, k)
        r = np.zeros(h.dim, dtype=complex)
        np.add.at(r, cols, vals)
        assert np.allclose(r, H[k], atol=1e-15)


def test_norm_inf_time_independent():
    h = HubbardOracle(cluster_2d(3, 4).with_hopping(1.0), 8.0, 2, 2)
    n0 = np.abs(h.H(0.0).toarray()).sum(axis=1).max()
    n1 = np.abs(h.H(0.9).toarray()).sum(axis=1).max()
    assert n0 == pytest.approx(n1) == pytest.approx(h.norm_inf())


# --------------------------------------------------------------------------
# layout map to the spin-separated tile

@pytest.mark.parametrize("lat,nu,nd", [(ring(5), 2, 3), (cluster_2d(3, 2), 3, 3), (chain(4), 2, 1)])
def test_canonical_map_gives_tensor_product_structure(lat, nu, nd):
    """With the sign S of the interleaved -> separated reordering, H becomes
    T_up (x) 1 + 1 (x) T_dn + D on the (a, b) tile, where T_up (T_dn) is the
    Hamiltonian of the up-only (down-only) sector; without S it does not."""
    A = 0.53
    ns = lat.n_sites
    h = HubbardOracle(lat, 3.0, nu, nd)
    flat, sign, du, dd, _, _ = canonical_map(h.states, ns)
    P = np.zeros((h.dim, h.dim))
    P[flat, np.arange(h.dim)] = sign
    Hc = P @ h.H(A).toarray() @ P.T
    Tu = HubbardOracle(lat, 0.0, nu, 0).H(A).toarray()
    Td = HubbardOracle(lat, 0.0, 0, nd).H(A).toarray()
    D = np.diag((P @ np.diag(h.diag) @ P.T).diagonal())
    expect = np.kron(Tu, np.eye(dd)) + np.kron(np.eye(du), Td) + D
    assert np.allclose(Hc, expect, atol=1e-15)
    P0 = np.abs(P)
    Hn = P0 @ h.H(A).toarray() @ P0.T
    if nu > 0 and nd > 0 and ns > 2:
        assert not np.allclose(Hn, expect, atol=1e-6)


# --------------------------------------------------------------------------
# pulse

def test_pulse_shape_properties():
    p = PulseParams(0, 0.5, 8.0, 1.0, 0.3)
    assert pulse_A(p, 1.0) == 0.0
    for s in (0.05, 0.1, 0.37):
        assert pulse_A(p, 1.0 + s) == pytest.approx(-pulse_A(p, 1.0 - s), abs=1e-15)
    ts = np.linspace(-2, 4, 20001)
    a = np.array([pulse_A(p, t) for t in ts])
    assert np.max(np.abs(a)) <= 0.5
    # zero crossings at t0 + k pi / omega
    for k in (1, 2, 3):
        assert abs(pulse_A(p, 1.0 + k * math.pi / 8.0)) < 1e-15
    # far from the centre the envelope has decayed
    assert abs(pulse_A(p, 1.0 + 3.0)) < 1e-20
    # kind 1 with b = cos(omega t_p) starts at zero phase (f(0) = 1)
    q = PulseParams(1, 0.8, 3.0, 6.0, 2.0, math.cos(3.0 * 6.0))
    assert abs(pulse_A(q, 0.0)) < 1e-15


# --------------------------------------------------------------------------
# stepper

def _small():
    lat = ring(6)
    return lat, HubbardOracle(lat, 4.0, 3, 3), PulseParams(0, 0.7, 5.0, 0.3, 0.2)


def test_exact_step_matches_eigendecomposition_and_sparse_route():
    lat, h, p = _small()
    v = random_state(h.dim, seed=3)[0]
    t, tau = 0.21, 0.05
    H = h.H(pulse_A(p, t + tau / 2)).toarray()
    w, U = np.linalg.eigh(H)
    ref = U @ (np.exp(-1j * tau * w) * (U.conj().T @ v))
    out = midpoint_step_exact(h, v, t, tau, p)
    assert np.allclose(out, ref, atol=1e-13)
    import scipy.sparse.linalg as spla
    out2 = spla.expm_multiply(-1j * tau * h.H(pulse_A(p, t + tau / 2)), v)
    assert np.allclose(out2, ref, atol=1e-13)


def test_stationary_ground_state_evolution():
    """Sec. 3.9 / Fig. 3: from the ground state of a time-independent H the
    state only picks up the phase exp(-i E0 t); d and E stay constant."""
    h = HubbardOracle(chain(6), 4.0, 3, 3)
    E0, E1, g = ground_state(h, 0.0)
    p = PulseParams(0, 0.0, 1.0, 0.0, 1.0)
    v = g.copy()
    n0, e0, d0, _ = observables(h, g, 0.0)
    for n in range(20):
        v = midpoint_step_exact(h, v, n * 0.1, 0.1, p)
    assert np.allclose(v, np.exp(-1j * E0 * 2.0) * g, atol=1e-12)
    n1, e1, d1, _ = observables(h, v, 0.0)
    assert e1 == pytest.approx(e0, abs=1e-12) and d1 == pytest.approx(d0, abs=1e-12)
    assert e0 == pytest.approx(E0 / 6, abs=1e-12)


def test_norm_and_energy_conservation_without_field():
    h = HubbardOracle(ring(6), 4.0, 3, 2)
    v = random_state(h.dim, seed=5)[0]
    p = PulseParams(0, 0.0, 1.0, 0.0, 1.0)
    _, e0, _, _ = observables(h, v, 0.0)
    for n in range(10):
        v = midpoint_step_exact(h, v, n * 0.2, 0.2, p)
    n1, e1, _, _ = observables(h, v, 0.0)
    assert n1 == pytest.approx(1.0, abs=1e-13)
    assert e1 == pytest.approx(e0, abs=1e-12)


def test_no_hopping_evolution_is_diagonal_phase():
    lat = cluster_2d(3, 2).with_hopping(0.0)
    h = HubbardOracle(lat, 7.0, 3, 2)
    v0 = random_state(h.dim, seed=9)[0]
    p = PulseParams(0, 0.9, 6.0, 0.2, 0.3)
    v = v0.copy()
    for n in range(8):
        v = midpoint_step_exact(h, v, n * 0.05, 0.05, p)
    assert np.allclose(v, np.exp(-1j * 7.0 * docc_weights(h.states, 6) * 0.4) * v0, atol=1e-13)


def test_free_fermion_reduction_with_pulse():
    """U = 0: the many-body stepper equals propagating the orbitals of a
    Slater determinant (open-shell filling on purpose)."""
    lat = ring(6)
    h = HubbardOracle(lat, 0.0, 2, 3)
    p = PulseParams(0, 0.8, 4.0, 0.25, 0.2)
    rng = np.random.default_rng(2)
    phis = [np.linalg.qr(rng.standard_normal((6, 2)) + 1j * rng.standard_normal((6, 2)))[0],
            np.linalg.qr(rng.standard_normal((6, 3)) + 1j * rng.standard_normal((6, 3)))[0]]
    v = ff.slater_vector(phis[0], phis[1], h)
    assert np.linalg.norm(v) == pytest.approx(1.0, abs=1e-13)
    tau = 0.04
    for n in range(12):
        v = midpoint_step_exact(h, v, n * tau, tau, p)
        phis = ff.step(lat, phis, n * tau, tau, p)
    A = pulse_A(p, 12 * tau)
    _, e_mb, d_mb, site_mb = observables(h, v, A)
    e_ff, d_ff, site_ff = ff.observables(lat, phis, A)
    assert e_mb == pytest.approx(e_ff, abs=1e-12)
    assert d_mb == pytest.approx(d_ff, abs=1e-12)
    assert np.allclose(site_mb, site_ff, atol=1e-12)
    assert np.allclose(v, ff.slater_vector(phis[0], phis[1], h), atol=1e-12)


def test_time_reversal():
    lat, h, p = _small()
    v0 = random_state(h.dim, seed=4)[0]
    v = v0.copy()
    tau, n = 0.05, 10
    for k in range(n):
        v = midpoint_step_exact(h, v, k * tau, tau, p)
    for k in reversed(range(n)):
        v = midpoint_step_exact(h, v, (k + 1) * tau, -tau, p)
    assert np.allclose(v, v0, atol=1e-12)


def test_midpoint_rule_is_second_order():
    """The exponential midpoint rule is the second-order Magnus integrator;
    halving tau divides the global error by about 4."""
    h = HubbardOracle(ring(4), 4.0, 1, 2)
    p = PulseParams(0, 0.7, 5.0, 0.3, 0.2)
    v0 = random_state(h.dim, seed=6)[0]
    T = 0.6

    def run(tau):
        v = v0.copy()
        for k in range(int(round(T / tau))):
            v = midpoint_step_exact(h, v, k * tau, tau, p)
        return v

    ref = run(T / 960)
    errs = [np.linalg.norm(run(T / n) - ref) for n in (30, 60, 120)]
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 3.6 < r1 < 4.4 and 3.6 < r2 < 4.4


# --------------------------------------------------------------------------
# Krylov step (Alg. 6) and the small exponential

def test_tridiag_expm_matches_eigendecomposition():
    rng = np.random.default_rng(0)
    for j in (1, 2, 5, 17, 30):
        a = rng.uniform(-10, 10, j)
        b = rng.uniform(0.1, 8, max(j - 1, 1))[: max(j - 1, 0)]
        T = np.diag(a) + np.diag(b, 1) + np.diag(b, -1)
        w, Q = np.linalg.eigh(T)
        ref = Q @ (np.exp(-1j * 0.07 * w) * Q[0, :])
        assert np.allclose(tridiag_expm_e1(a, b, 0.07), ref, atol=1e-14)


def test_alg6_reaches_tolerance_against_exact_step():
    lat = cluster_2d(3, 2)
    h = HubbardOracle(lat, 8.0, 3, 3)
    v = random_state(h.dim, seed=11)[0]
    A, tau = 0.4, 0.01
    exact = expm_apply(h.H(A), v, tau)
    ms = []
    for tol in (1e-6, 1e-10, 1e-13):
        out, info = krylov_step_alg6(lambda x: h.apply(A, x), v, tau, 30, tol, h.norm_inf())
        assert info["converged"]
        # the estimate undershoots the error by about an order of magnitude (Fig. 2)
        assert np.linalg.norm(out - exact) < 100 * tol
        ms.append(info["m"])
    assert ms[0] <= ms[1] <= ms[2] and ms[0] < ms[2]


def test_alg6_eigenvector_start_breaks_down_immediately():
    h = HubbardOracle(ring(6), 4.0, 3, 3)
    E0, _, g = ground_state(h, 0.0)
    out, info = krylov_step_alg6(lambda x: h.apply(0.0, x), g, 0.1, 30, 1e-12, h.norm_inf())
    assert info["m"] == 1 and info["breakdown"]
    assert np.allclose(out, np.exp(-1j * 0.1 * E0) * g, atol=1e-12)


def test_alg6_not_converged_flag():
    h = HubbardOracle(cluster_2d(3, 2), 8.0, 3, 3)
    v = random_state(h.dim, seed=12)[0]
    out, info = krylov_step_alg6(lambda x: h.apply(0.2, x), v, 0.05, 3, 1e-14, h.norm_inf())
    assert not info["converged"] and info["m"] == 3


def test_alg6_estimate_tracks_error_rate():
    """Fig. 2: the a-posteriori estimate decreases with m at the rate of the
    true error (checked as a log-log slope within a factor)."""
    h = HubbardOracle(ring(8), 8.0, 4, 4)
    v = random_state(h.dim, seed=13)[0]
    A, tau = 0.3, 0.05
    exact = expm_apply(h.H(A), v, tau)
    est, err = [], []
    for m in range(3, 12):
        out, info = krylov_step_alg6(lambda x: h.apply(A, x), v, tau, m, 1e-30, h.norm_inf())
        est.append(info["eps"])
        err.append(np.linalg.norm(out - exact))
    le, lr = np.log(est), np.log(err)
    se = np.polyfit(range(len(le)), le, 1)[0]
    sr = np.polyfit(range(len(lr)), lr, 1)[0]
    assert se < 0 and sr < 0 and 0.5 < se / sr < 2.0


# --------------------------------------------------------------------------
# ground state and observables

def test_ground_state_sparse_matches_dense_and_power_iteration():
    h = HubbardOracle(ring(8), 8.0, 4, 4)
    E0, E1, g = ground_state(h, 0.0)           # dense (dim 4900 > limit -> sparse)
    w = np.linalg.eigvalsh(h.H(0.0).toarray())
    assert E0 == pytest.approx(w[0], abs=1e-11) and E1 == pytest.approx(w[1], abs=1e-10)
    assert E1 - E0 > 1e-3  # unique ground state on the half-filled bipartite ring
    hs = HubbardOracle(two_site(), 4.0, 1, 1)
    Ep, _ = power_iteration_ground_state(hs, 0.0, tol=1e-13)
    assert Ep == pytest.approx(2 - math.sqrt(4 + 4), abs=1e-9)


def test_observables_free_half_filled_ring_and_bounds():
    h0 = HubbardOracle(ring(6), 0.0, 3, 3)
    _, _, g0 = ground_state(h0, 0.0)
    _, e, d, site = observables(h0, g0, 0.0)
    assert d == pytest.approx(0.25, abs=1e-12)
    assert np.allclose(site, 0.25, atol=1e-12)
    # free-fermion energy per site: occupied levels -2cos(2 pi n/6) for n = 0, +-1, twice
    assert e == pytest.approx(2 * (-2 - 2 * 0.5 - 2 * 0.5) / 6, abs=1e-12)
    for U in (2.0, 8.0, 40.0):
        h = HubbardOracle(ring(6), U, 3, 3)
        _, _, g = ground_state(h, 0.0)
        _, _, dU, s = observables(h, g, 0.0)
        assert 0 < dU < 0.25 and s.sum() / 6 == pytest.approx(dU)
    assert dU < 0.01


def test_onsite_energy_enters_with_plus_sign():
    """One electron, no hopping: the energies are the on-site epsilon_i."""
    eps = [0.5, -1.25, 2.0]
    lat = chain(3).with_hopping(0.0).with_onsite(eps)
    for nu, nd in ((1, 0), (0, 1)):
        h = HubbardOracle(lat, 3.0, nu, nd)
        assert np.allclose(np.sort(np.linalg.eigvalsh(h.H(0.3).toarray())), np.sort(eps))
    h2 = HubbardOracle(lat, 3.0, 1, 1)
    ev = np.sort(np.linalg.eigvalsh(h2.H(0.0).toarray()))
    ref = sorted(eps[i] + eps[j] + (3.0 if i == j else 0.0) for i in range(3) for j in range(3))
    assert np.allclose(ev, ref)


# --------------------------------------------------------------------------
# Green's functions (Eq. (Glg))

def test_greens_equal_time_sum_rule():
    """G^>(t,t) - G^<(t,t) = -i <{c, c^dag}> = -i for a normalised state."""
    from oracle.greens import greens_diag
    lat = ring(6)
    h = HubbardOracle(lat, 4.0, 3, 3)
    psi = random_state(h.dim, seed=31)[0]
    p = PulseParams(0, 0.5, 6.0, 0.1, 0.2)
    for site, spin in ((0, UP), (3, DOWN)):
        ol = greens_diag(h, psi, p, 0.0, 0.05, 2, 0, site, spin, dagger=False)
        og = greens_diag(h, psi, p, 0.0, 0.05, 2, 0, site, spin, dagger=True)
        assert (-1j * og[0]) - (1j * ol[0]) == pytest.approx(-1j, abs=1e-13)


def test_greens_equilibrium_matches_lehmann():
    """A = 0 from the ground state: the propagated overlap equals the Lehmann
    sum over the eigenstates of the N-1 (N+1) sector, up to the midpoint
    stepper being exact for time-independent H."""
    from oracle.greens import greens_diag, lehmann_overlap
    lat = ring(6)
    h = HubbardOracle(lat, 4.0, 3, 3)
    E0, _, g = ground_state(h, 0.0)
    p = PulseParams(0, 0.0, 1.0, 0.0, 1.0)
    for dagger, tgt in ((False, (2, 3)), (True, (4, 3))):
        ht = HubbardOracle(lat, 4.0, *tgt)
        o = greens_diag(h, g, p, 0.0, 0.1, 0, 15, 0, UP, dagger, ham_target=ht)
        ref = lehmann_overlap(h, g, E0, ht, 0, UP, dagger, 0.1 * np.arange(16))
        assert np.allclose(o, ref, atol=1e-12)
    # half filling: G^<_ii(t,t) = i/2 on the ring
    o = greens_diag(h, g, p, 0.0, 0.1, 0, 0, 2, DOWN, False)
    assert 1j * o[0] == pytest.approx(0.5j, abs=1e-12)


def test_greens_free_fermion_closed_form_with_pulse():
    """U = 0: G^<_ii(t, t') = i sum_occupied Phi_k,i(t) conj(Phi_k,i(t')) with
    the orbitals propagated by the same midpoint steps."""
    from oracle.greens import greens_diag
    lat = ring(6)
    h = HubbardOracle(lat, 0.0, 2, 3)
    p = PulseParams(0, 0.7, 5.0, 0.2, 0.25)
    rng = np.random.default_rng(4)
    phis = [np.linalg.qr(rng.standard_normal((6, 2)) + 1j * rng.standard_normal((6, 2)))[0],
            np.linalg.qr(rng.standard_normal((6, 3)) + 1j * rng.standard_normal((6, 3)))[0]]
    psi0 = ff.slater_vector(phis[0], phis[1], h)
    dt, start, nrel, site = 0.05, 3, 10, 4
    for spin in (UP, DOWN):
        o = greens_diag(h, psi0, p, 0.0, dt, start, nrel, site, spin, False)
        ph = [q.copy() for q in phis]
        hist = []
        for n in range(start + nrel + 1):
            hist.append(ph[spin][site, :].copy())
            ph = ff.step(lat, ph, n * dt, dt, p)
        ref = [np.sum(hist[start + s] * np.conj(hist[start])) for s in range(nrel + 1)]
        # o(s) = <c psi(t'+s)| U c psi(t')> = <c^dag(t'+s) c(t')> = sum_k Phi(t') conj(Phi(t'+s))
        assert np.allclose(o, np.conj(ref), atol=1e-12)
