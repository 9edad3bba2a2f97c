"""Creation/annihilation operators, overlaps and diagonal Green's functions
(Eq. (Glg)) of the HIP path against the CPU oracle."""
import numpy as np
import pytest

import paper_2005_13498_amd as hub
from synth import ring, cluster_2d, PulseParams, random_state, workloads
from oracle import HubbardOracle, to_canonical, ladder_matrix, pulse_A
from oracle.fock import UP, DOWN, mode_index
from oracle.greens import greens_diag

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _dev(x, dtype=torch.complex128):
    return torch.from_numpy(np.ascontiguousarray(x)).to(DEV).to(dtype)


@pytest.mark.parametrize("site,spin,dagger", [(0, 0, False), (3, 0, True), (2, 1, False), (5, 1, True),
                                              (4, 0, False), (1, 1, True)])
def test_apply_cop_matches_ladder_operator(site, spin, dagger):
    lat = cluster_2d(3, 2)
    nu, nd = 3, 2
    d = 1 if dagger else -1
    tu, td = (nu + d, nd) if spin == 0 else (nu, nd + d)
    hs, ht = HubbardOracle(lat, 4.0, nu, nd), HubbardOracle(lat, 4.0, tu, td)
    Bs, Bt = hub.Basis(lat, 4.0, nu, nd), hub.Basis(lat, 4.0, tu, td)
    xs = random_state(hs.dim, seed=5, nvec=2)
    Op = ladder_matrix(hs.states, ht.states, mode_index(site, spin), dagger)
    ref = np.stack([to_canonical(Op @ v, ht.states, 6) for v in xs])
    x = _dev(np.concatenate([to_canonical(v, hs.states, 6) for v in xs]))
    y = torch.empty(2 * Bt.dim, dtype=torch.complex128, device=DEV)
    hub.hub_apply_cop(Bs.handle, Bt.handle, site, spin, dagger, x, y, nvec=2)
    assert np.allclose(y.cpu().numpy().reshape(2, -1), ref, atol=1e-15)
    Bs.close()
    Bt.close()


def test_apply_cop_wrong_sector_rejected():
    lat = ring(6)
    Bs, Bt = hub.Basis(lat, 4.0, 3, 3), hub.Basis(lat, 4.0, 3, 2)
    x = torch.zeros(Bs.dim, dtype=torch.complex128, device=DEV)
    y = torch.zeros(Bt.dim, dtype=torch.complex128, device=DEV)
    with pytest.raises(hub.HubError) as e:
        hub.hub_apply_cop(Bs.handle, Bt.handle, 0, 0, False, x, y)   # c_up needs (2, 3)
    assert e.value.status == hub.HUB_E_SECTOR
    Bs.close()
    Bt.close()


def test_dot_batched():
    B = hub.Basis(ring(6), 4.0, 3, 2)
    a = random_state(B.dim, seed=1, nvec=3)
    b = random_state(B.dim, seed=2, nvec=3)
    got = hub.hub_dot(B.handle, _dev(a.ravel()), _dev(b.ravel()), nvec=3)
    assert np.allclose(got, [np.vdot(a[k], b[k]) for k in range(3)], atol=1e-15)
    B.close()


def _greens_case(lat, U, nu, nd, members, n_rel, dt, pulse, prec, tol, seed=9, path=-1):
    ham = HubbardOracle(lat, U, nu, nd)
    psi0 = random_state(ham.dim, seed=seed)[0]
    B = hub.Basis(lat, U, nu, nd)
    hub.hub_set_greens_path(B.handle, path)
    sectors = sorted({((nu + (1 if m[2] else -1), nd) if m[1] == 0 else (nu, nd + (1 if m[2] else -1)))
                      for m in members})
    T = [hub.Basis(lat, U, *sec) for sec in sectors]
    dtype = torch.complex128 if prec == hub.HUB_C128 else torch.complex64
    psi = _dev(to_canonical(psi0, ham.states, lat.n_sites), dtype)
    got = hub.hub_greens_diag(B.handle, [t.handle for t in T], pulse, 0.0, dt, n_rel,
                              hub.make_opts(tol=tol, m_max=30), members, psi)
    oh = {sec: HubbardOracle(lat, U, *sec) for sec in sectors}
    for k, (site, spin, dagger, start) in enumerate(members):
        sec = (nu + (1 if dagger else -1), nd) if spin == 0 else (nu, nd + (1 if dagger else -1))
        ref = greens_diag(ham, psi0, pulse, 0.0, dt, start, n_rel, site, spin, bool(dagger), ham_target=oh[sec])
        yield k, got[k], ref
    B.close()
    for t in T:
        t.close()


# path 0: members batched per sector; path 1: the persistent member stepper
_PATHS = pytest.mark.parametrize("path", [0, 1])


@_PATHS
def test_greens_diag_c128_matches_oracle(path):
    members = [(0, 0, 0, 0), (2, 1, 1, 3), (3, 0, 0, 2), (1, 0, 1, 0), (4, 1, 0, 1), (5, 1, 0, 2)]
    p = PulseParams(0, 0.6, 6.0, 0.2, 0.2)
    for k, got, ref in _greens_case(ring(6), 4.0, 3, 3, members, 12, 0.05, p, hub.HUB_C128, 1e-13, path=path):
        assert np.max(np.abs(got - ref)) < 1e-10, (k, np.max(np.abs(got - ref)))


@_PATHS
def test_greens_diag_c64_within_1e5(path):
    members = [(0, 0, 0, 0), (2, 1, 1, 3), (3, 0, 1, 2), (4, 1, 0, 1)]
    p = PulseParams(0, 0.6, 6.0, 0.2, 0.2)
    for k, got, ref in _greens_case(ring(8), 8.0, 4, 4, members, 20, 0.02, p, hub.HUB_C64, 1e-8, path=path):
        assert np.max(np.abs(got - ref)) < 1e-5, (k, np.max(np.abs(got - ref)))


@_PATHS
def test_greens_ring10_workload_sampled(path):
    """10-site ring, U = 8, 5/5 (dim 63,504), members in the (4,5), (6,5),
    (5,4), (5,6) sectors (dim 52,920) with staggered starts, complex64 apply
    with FP64 Lanczos scalars; first 15 relative steps against the oracle."""
    w = workloads()["ring10_greens"]
    members = [(0, 0, 0, 0), (3, 0, 1, 5), (6, 1, 0, 10), (9, 1, 1, 0)]
    for k, got, ref in _greens_case(w.lattice, w.U, 5, 5, members, 15, w.dt, w.pulse, hub.HUB_C64, 1e-8,
                                    path=path):
        assert np.max(np.abs(got - ref)) < 1e-5, (k, np.max(np.abs(got - ref)))


_STARTS = (50, 100)
_SIXTEEN = [(site, spin, dagger, st) for spin, dagger in ((0, 1), (1, 1), (0, 0), (1, 0))
            for site in (0, 6) for st in _STARTS]
_N_REL16 = 30


@pytest.fixture(scope="module")
def sixteen_reference():
    """Oracle overlaps of the 16 members: psi propagated once to each t',
    each member from there (shared by both precisions)."""
    w = workloads()["ring10_greens"]
    ham = HubbardOracle(w.lattice, w.U, 5, 5)
    psi0 = random_state(ham.dim, seed=10)[0]
    from oracle.stepper import midpoint_step_exact
    psi_at = {}
    v = psi0.copy()
    for n in range(max(_STARTS) + 1):
        if n in _STARTS:
            psi_at[n] = v.copy()
        v = midpoint_step_exact(ham, v, n * w.dt, w.dt, w.pulse)
    oh = {}
    ref = []
    for site, spin, dagger, st in _SIXTEEN:
        sec = (5 + (1 if dagger else -1), 5) if spin == 0 else (5, 5 + (1 if dagger else -1))
        if sec not in oh:
            oh[sec] = HubbardOracle(w.lattice, w.U, *sec)
        ref.append(greens_diag(ham, psi_at[st], w.pulse, st * w.dt, w.dt, 0, _N_REL16, site, spin, bool(dagger),
                               ham_target=oh[sec]))
    return w, ham, psi0, ref


@_PATHS
@pytest.mark.parametrize("prec,tol,bar", [(hub.HUB_C64, 1e-8, 1e-5), (hub.HUB_C128, 1e-13, 1e-10)])
def test_greens_ring10_sixteen_members(sixteen_reference, prec, tol, bar, path):
    """The 10-site ring workload from a seeded state: all four operators (c
    and c^dag of both spins) at sites 0 and 6, from t' = 0.5 and 1.0 (16
    members, four per sector with two start times each), 30 relative steps;
    every member and step against the oracle."""
    w, ham, psi0, ref = sixteen_reference
    lat, U = w.lattice, w.U
    B = hub.Basis(lat, U, 5, 5)
    hub.hub_set_greens_path(B.handle, path)
    T = [hub.Basis(lat, U, *sec) for sec in [(4, 5), (6, 5), (5, 4), (5, 6)]]
    try:
        dtype = torch.complex128 if prec == hub.HUB_C128 else torch.complex64
        psi = _dev(to_canonical(psi0, ham.states, 10), dtype)
        got = hub.hub_greens_diag(B.handle, [t.handle for t in T], w.pulse, 0.0, w.dt, _N_REL16,
                                  hub.make_opts(tol=tol, m_max=30), _SIXTEEN, psi)
        for k in range(len(_SIXTEEN)):
            assert np.max(np.abs(got[k] - ref[k])) < bar, (k, np.max(np.abs(got[k] - ref[k])))
    finally:
        B.close()
        for t in T:
            t.close()


@_PATHS
def test_greens_onsite_energies_and_a_spin_without_hops(path):
    """On-site energies (seeded, both spins) and sectors whose down spin is
    empty (one string, no hops): 6-site ring, psi in (2, 0), members c_up
    into (1, 0) and c^dag_down into (2, 1); then psi in (3, 2) with members in
    all four neighbouring sectors.  Both steppers against the oracle (c128,
    1e-10)."""
    lat = ring(6).with_onsite(list(np.random.default_rng(66).uniform(-1.0, 1.0, 6)))
    p = PulseParams(0, 0.6, 6.0, 0.2, 0.2)
    for (nu, nd), members in (((2, 0), [(1, 0, 0, 2), (4, 1, 1, 0), (3, 0, 0, 0)]),
                              ((3, 2), [(0, 0, 0, 1), (2, 0, 1, 0), (5, 1, 0, 2), (1, 1, 1, 3)])):
        for k, got, ref in _greens_case(lat, 4.0, nu, nd, members, 10, 0.05, p, hub.HUB_C128, 1e-13, path=path):
            assert np.max(np.abs(got - ref)) < 1e-10, ((nu, nd), k, np.max(np.abs(got - ref)))


def test_greens_member_stepper_stops_at_m_max():
    """m_max too small for the tolerance in the members' steps only: at U = 0
    psi = (plane wave k = 1 up) x (plane wave k = 2 down) on the 6-site ring
    is an eigenstate of H(A) for every A (one Lanczos vector per step),
    while the member c^dag_{1,up} psi needs more than three Krylov vectors
    for a step of 0.5.  Both steppers report HUB_E_NOT_CONVERGED."""
    lat = ring(6)
    B = hub.Basis(lat, 0.0, 1, 1)
    T = [hub.Basis(lat, 0.0, 2, 1)]
    up, dn = hub.hub_basis_states(B.handle)
    site = lambda s: int(s).bit_length() - 1
    pw = lambda k, strings: np.array([np.exp(2j * np.pi * k * site(s) / 6) for s in strings]) / np.sqrt(6)
    psi = _dev(np.outer(pw(1, up), pw(2, dn)).ravel(), torch.complex128)
    try:
        for path in (0, 1):
            hub.hub_set_greens_path(B.handle, path)
            with pytest.raises(hub.HubError) as e:
                hub.hub_greens_diag(B.handle, [t.handle for t in T], PulseParams(0, 0.6, 6.0, 0.2, 0.2), 0.0, 0.5, 6,
                                    hub.make_opts(tol=1e-14, m_max=3), [(1, 0, 1, 2)], psi.clone())
            assert e.value.status == hub.HUB_E_NOT_CONVERGED
    finally:
        B.close()
        for t in T:
            t.close()


def test_greens_member_stepper_needs_three_term_recurrence():
    """Forcing the persistent stepper with full reorthogonalisation is an
    error; the automatic choice falls back to the per-sector path."""
    lat = ring(6)
    p = PulseParams(0, 0.6, 6.0, 0.2, 0.2)
    B = hub.Basis(lat, 4.0, 3, 3)
    T = [hub.Basis(lat, 4.0, 2, 3)]
    psi = _dev(random_state(B.dim, seed=4)[0], torch.complex128)
    opts = hub.make_opts(tol=1e-12, m_max=30, reorth=1)
    try:
        hub.hub_set_greens_path(B.handle, 1)
        with pytest.raises(hub.HubError) as e:
            hub.hub_greens_diag(B.handle, [T[0].handle], p, 0.0, 0.05, 4, opts, [(1, 0, 0, 0)], psi.clone())
        assert e.value.status == hub.HUB_E_INVALID
        hub.hub_set_greens_path(B.handle, -1)
        a = hub.hub_greens_diag(B.handle, [T[0].handle], p, 0.0, 0.05, 4, opts, [(1, 0, 0, 0)], psi.clone())
        hub.hub_set_greens_path(B.handle, 0)
        b = hub.hub_greens_diag(B.handle, [T[0].handle], p, 0.0, 0.05, 4, opts, [(1, 0, 0, 0)], psi.clone())
        assert np.array_equal(a, b)
    finally:
        B.close()
        for t in T:
            t.close()


@pytest.fixture(scope="module")
def c3_reference():
    """Oracle overlaps of all 64 members of the 10-site ring workload (c and
    c^dag of both spins at sites 0, 3, 6, 9 from t' = 0.5, 1.0, 1.5, 2.0) for 6
    relative steps, psi from a seeded state propagated once to every t'."""
    w = workloads()["ring10_greens"]
    ham = HubbardOracle(w.lattice, w.U, 5, 5)
    psi0 = random_state(ham.dim, seed=11)[0]
    from oracle.stepper import midpoint_step_exact
    members = [(site, spin, dagger, int(round(tp / w.dt)))
               for spin, dagger in ((0, 1), (1, 1), (0, 0), (1, 0))
               for site in w.extra["sites"] for tp in w.extra["t_primes"]]
    starts = sorted({m[3] for m in members})
    psi_at, v = {}, psi0.copy()
    for n in range(max(starts) + 1):
        if n in starts:
            psi_at[n] = v.copy()
        v = midpoint_step_exact(ham, v, n * w.dt, w.dt, w.pulse)
    oh, ref = {}, []
    for site, spin, dagger, st in members:
        sec = (5 + (1 if dagger else -1), 5) if spin == 0 else (5, 5 + (1 if dagger else -1))
        if sec not in oh:
            oh[sec] = HubbardOracle(w.lattice, w.U, *sec)
        ref.append(greens_diag(ham, psi_at[st], w.pulse, st * w.dt, w.dt, 0, 6, site, spin, bool(dagger),
                               ham_target=oh[sec]))
    return w, ham, psi0, members, ref


@_PATHS
def test_greens_ring10_all_64_members(c3_reference, path):
    """The batched Green's-function configuration at full size: all 64 members
    in one call (complex64 apply, Krylov tol 1e-8), every member and step
    against the oracle within 1e-5."""
    w, ham, psi0, members, ref = c3_reference
    B = hub.Basis(w.lattice, w.U, 5, 5)
    hub.hub_set_greens_path(B.handle, path)
    T = [hub.Basis(w.lattice, w.U, *sec) for sec in [(4, 5), (6, 5), (5, 4), (5, 6)]]
    try:
        psi = _dev(to_canonical(psi0, ham.states, 10), torch.complex64)
        got = hub.hub_greens_diag(B.handle, [t.handle for t in T], w.pulse, 0.0, w.dt, 6,
                                  hub.make_opts(tol=1e-8, m_max=30), members, psi)
        err = max(float(np.max(np.abs(got[k] - ref[k]))) for k in range(len(members)))
        assert err < 1e-5, err
    finally:
        B.close()
        for t in T:
            t.close()
