"""14-site ring at half filling (dim 11,778,624): the apply at full size on
sampled rows, and the complex64 block path against the complex128
single-vector path (the block workload's reference)."""
import numpy as np
import pytest

import paper_2005_13498_amd as hub
from synth import workloads, PulseParams
from oracle import HubbardOracle
from oracle.fock import sector_states

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _canon(state, ns, up_rank, dn_rank, dim_dn):
    """(flat tile index, sign S) of one interleaved basis state."""
    ups = sum(((state >> (2 * i)) & 1) << i for i in range(ns))
    dns = sum(((state >> (2 * i + 1)) & 1) << i for i in range(ns))
    cross = sum(1 for j in range(ns) if (dns >> j) & 1 for i in range(j + 1, ns) if (ups >> i) & 1)
    return up_rank[ups] * dim_dn + dn_rank[dns], (-1.0) ** cross


class _RowOracle:
    """The oracle's Hamiltonian rows without assembling the full matrix."""

    def __init__(self, lat, U, n):
        self.lat, self.U, self.n = lat, U, n
        self.states = sector_states(lat.n_sites, n, n)
        self.ham = HubbardOracle.__new__(HubbardOracle)
        self.ham.lattice, self.ham.n_sites, self.ham.U = lat, lat.n_sites, U
        self.ham.states = self.states
        from oracle.fock import docc_weights
        self.ham.diag = None
        self._docc = docc_weights

    def row(self, A, k):
        st = self.states[k:k + 1]
        self.ham.diag = {k: self.U * float(self._docc(st, self.lat.n_sites)[0])}
        return HubbardOracle.row(self.ham, A, k)


def test_ring14_apply_sampled_rows():
    w = workloads()["ring14_block"]
    lat, U = w.lattice, w.U
    B = hub.Basis(lat, U, 7, 7)
    up, dn = hub.hub_basis_states(B.handle)
    up_rank = {int(s): i for i, s in enumerate(up)}
    dn_rank = {int(s): i for i, s in enumerate(dn)}
    g = torch.Generator(device=DEV).manual_seed(3)
    x = torch.randn(B.dim, dtype=torch.complex128, device=DEV, generator=g)
    y = torch.empty_like(x)
    A = 0.37
    hub.hub_apply_H(B.handle, [A], x, y)
    RO = _RowOracle(lat, U, 7)
    rng = np.random.default_rng(0)
    xc = x.cpu().numpy()
    yc = y.cpu().numpy()
    for k in rng.integers(0, len(RO.states), 40):
        cols, vals = RO.row(A, int(k))
        ik, sk = _canon(int(RO.states[k]), 14, up_rank, dn_rank, len(dn))
        acc = 0j
        for c, v in zip(cols, vals):
            ic, sc = _canon(int(RO.states[c]), 14, up_rank, dn_rank, len(dn))
            acc += v * sc * xc[ic]
        assert abs(yc[ik] - sk * acc) < 1e-12 * (1 + abs(acc))
    B.close()


def test_ring14_c64_block_vs_c128_single():
    w = workloads()["ring14_block"]
    B = hub.Basis(w.lattice, w.U, 7, 7)
    pulses = [PulseParams(0, a, 8.0, 0.0, 0.3) for a in w.extra["A0_batch"]]
    g = torch.Generator(device=DEV).manual_seed(7)
    v0 = torch.randn(B.dim, dtype=torch.complex128, device=DEV, generator=g)
    v0 /= torch.linalg.vector_norm(v0)
    n = 4
    opts64 = hub.make_opts(tol=1e-8, m_max=30)
    blk = v0.to(torch.complex64).repeat(len(pulses)).contiguous()
    st, o64, _ = hub.hub_propagate(B.handle, pulses, 0.0, w.dt, n, opts64, blk)
    opts128 = hub.make_opts(tol=1e-12, m_max=30)
    for k in (0, 5, 7):
        v = v0.clone()
        st, o128, _ = hub.hub_propagate(B.handle, [pulses[k]], 0.0, w.dt, n, opts128, v)
        got = blk[k * B.dim:(k + 1) * B.dim].to(torch.complex128)
        err = float(torch.linalg.vector_norm(got - v))
        assert err < 2e-5, err
        assert np.max(np.abs(o64[:, k, 3] - o128[:, 0, 3])) < 1e-5
        assert np.max(np.abs(o64[:, k, 2] - o128[:, 0, 2])) < 1e-5
    B.close()


@pytest.mark.parametrize("dtype,tol", [(torch.complex64, 2e-5), (torch.complex128, 1e-12)])
def test_ring14_two_pass_single_copy(dtype, tol):
    """14 sites: the column pass stages one copy of its columns (two do not
    fit LDS; complex64 4 columns, complex128 2) and takes the sign from the
    index.  Plain apply bit-identical to the one-pass kernel; fused Lanczos
    steps within rounding of the one-pass path."""
    w = workloads()["ring14_block"]
    B = hub.Basis(w.lattice, w.U, 7, 7)
    try:
        g = torch.Generator(device=DEV).manual_seed(11)
        x = torch.randn(B.dim, dtype=torch.complex128, device=DEV, generator=g)
        x = (x / torch.linalg.vector_norm(x)).to(dtype)
        ys = []
        for path in (0, 1):
            hub.hub_set_apply_path(B.handle, path)
            y = torch.empty_like(x)
            hub.hub_apply_H(B.handle, [0.37], x, y)
            ys.append(y)
        assert torch.equal(ys[0], ys[1])
        res = []
        for path in (0, -1):  # -1: automatic, the two-pass kernels for complex64 here
            hub.hub_set_apply_path(B.handle, path)
            v = x.clone()
            opts = hub.make_opts(tol=1e-6 if dtype == torch.complex64 else 1e-12, m_max=30)
            st, obs, log = hub.hub_propagate(B.handle, [w.pulse], 0.0, w.dt, 3, opts, v)
            res.append((v.to(torch.complex128).cpu().numpy(), obs))
        d = np.linalg.norm(res[1][0] - res[0][0]) / np.linalg.norm(res[0][0])
        assert d < tol, d
        assert np.max(np.abs(res[1][1] - res[0][1])) < tol
    finally:
        hub.hub_set_apply_path(B.handle, -1)
        B.close()
