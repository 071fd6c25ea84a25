"""The allocation-free encounter test (mx_flag_pairs_noalloc) against the
allocating entry point (mx_flag_pairs), through the C ABI: the same sorted pair
list and count, bit for bit, on two calls in a row, the second with fewer bodies
and fewer massive bodies (the scratch array keeps the first call's contents);
sizes beyond its limits are refused with MX_ECAPACITY."""
import numpy as np
import pytest

from synth import ic

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mx():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2601_16791_amd as m
    m.lib()
    return m


def _inputs(seed, nb, ns, h):
    """Massive and massless bodies on nearby orbits, drifted over h on their own
    Kepler orbits by the library's drift entry point."""
    import torch
    import paper_2601_16791_amd as m
    rng = np.random.default_rng(seed)
    n = nb + ns
    a = np.concatenate([rng.uniform(3.0, 3.5, nb), rng.uniform(2.8, 3.7, ns)])
    e = rng.uniform(0, 0.05, n)
    inc = rng.uniform(0, 0.01, n)
    M = np.concatenate([rng.uniform(0, 0.5, nb), rng.normal(0.25, 0.05, ns)])
    x0, u0 = ic.el2x(ic.G, a, e, inc, np.full(n, 0.3), np.full(n, 1.1), M)
    x1, u1 = m.kepler_drift(ic.G, x0, u0, h)
    torch.cuda.synchronize()
    return x0, u0, x1.cpu().numpy(), u1.cpu().numpy()


def test_noalloc_flag_pairs_equals_allocating_entry_point(mx):
    h = 20.0
    for seed, nb, ns, cap in ((1, 40, 6000, 1 << 14), (2, 7, 900, 1 << 10)):
        x0, u0, x1, u1 = _inputs(seed, nb, ns, h)
        rcrit = np.random.default_rng(seed + 10).uniform(0.05, 0.12, nb)
        ref = mx.flag_pairs(nb, rcrit, x0, u0, x1, u1, h, cap=cap)
        got = mx.flag_pairs(nb, rcrit, x0, u0, x1, u1, h, cap=cap, noalloc=True)
        assert len(ref) > 10, (seed, len(ref))
        assert np.array_equal(got, ref), (seed, len(got), len(ref))
    with pytest.raises(mx.MxError) as e:
        mx.flag_pairs(nb, rcrit, x0, u0, x1, u1, h, cap=1 << 17, noalloc=True)
    assert e.value.code == -7
