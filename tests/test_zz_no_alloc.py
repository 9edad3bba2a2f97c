"""hub_observables_noalloc (the entry point for callers that cannot allocate
device memory) against hub_observables through the C ABI: two calls in a
row, the second on a smaller input, each equal bit for bit to the
allocating entry point's results; a sector beyond the static buffer is
rejected before any launch."""
import numpy as np
import pytest

import paper_2005_13498_amd as hub
from synth import workloads, ring, chain, random_state

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _both(B, As, x):
    ref, sref = hub.hub_observables(B.handle, As, x, site=True)
    got, sgot = hub.hub_observables(B.handle, As, x, site=True, noalloc=True)
    return ref, sref, got, sgot


@pytest.mark.parametrize("dtype", [torch.complex128, torch.complex64])
def test_noalloc_observables_equal_allocating(dtype):
    w = workloads()["cluster3x4"]
    big = hub.Basis(w.lattice, w.U, 6, 6)
    small = hub.Basis(ring(6), 4.0, 3, 2)
    try:
        # first call: 12 sites, 3 vectors
        xs = random_state(big.dim, seed=31, nvec=3) * np.array([[1.0], [0.7], [2.0]])
        x = torch.from_numpy(xs.ravel()).to(DEV).to(dtype)
        ref, sref, got, sgot = _both(big, [0.3, -0.5, 1.2], x)
        assert np.array_equal(ref, got) and np.array_equal(sref, sgot)
        assert np.all(np.isfinite(got)) and abs(got[1, 1] - 0.7) < 1e-5
        # second call: a smaller sector and fewer vectors (stale contents of
        # the larger call must not leak into the result)
        xs2 = random_state(small.dim, seed=32, nvec=1)
        x2 = torch.from_numpy(xs2.ravel()).to(DEV).to(dtype)
        ref2, sref2, got2, sgot2 = _both(small, [0.9], x2)
        assert np.array_equal(ref2, got2) and np.array_equal(sref2, sgot2)
        assert abs(got2[0, 1] - 1.0) < 1e-5
    finally:
        big.close()
        small.close()


def test_noalloc_rejects_sector_beyond_scratch():
    B = hub.Basis(chain(16), 4.0, 8, 8)  # apply partials alone exceed 512 KiB
    try:
        x = torch.zeros(B.dim, dtype=torch.complex128, device=DEV)
        with pytest.raises(hub.HubError) as e:
            hub.hub_observables(B.handle, [0.0], x, noalloc=True)
        assert e.value.status == hub.HUB_E_INVALID and "static buffer" in str(e.value)
        del x
    finally:
        B.close()
        torch.cuda.empty_cache()
