"""mplu_zgesv_noalloc (the gesv that takes its workspace from the library's static
scratch) against mplu_zgesv on the same inputs: factors, pivots, info and X bit for bit,
on consecutive calls whose second input is smaller (the scratch keeps the first call's
contents, so everything the second call needs zeroed must be cleared by it)."""
import numpy as np
import pytest

import synthgen
from helpers import to_dev, to_host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mp():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2403_16013_amd as m

    m.lib()
    return m


def _pair(mp, orc, C, n, nrhs, seed, **kw):
    import torch

    A = orc.canon(synthgen.uniform(n, n, C, seed))
    B = orc.canon(synthgen.uniform(n, nrhs, C, seed + 1))
    Ta, Xa = to_dev(A), to_dev(B)
    ipa, infa = mp.gesv_noalloc(Ta, Xa, **kw)
    torch.cuda.synchronize()
    Tb, Xb = to_dev(A), to_dev(B)
    ipb, infb = mp.gesv(Tb, Xb, **kw)
    torch.cuda.synchronize()
    assert int(infa.item()) == int(infb.item()) == 0
    assert np.array_equal(ipa.cpu().numpy(), ipb.cpu().numpy())
    assert np.array_equal(to_host(Ta), to_host(Tb))
    assert np.array_equal(to_host(Xa), to_host(Xb))
    # and the solution is a solution: eta from the oracle's exact residual
    eta = orc.backward_error(A, to_host(Xa), B)
    assert eta <= 10 * n * {2: 2.0 ** -104, 3: 2.0 ** -157, 4: 2.0 ** -209}[C]


@pytest.mark.parametrize("C,method,panel", [(2, "3m", 64), (3, "4m", 32), (4, "3m", 128)])
def test_noalloc_equals_gesv_two_calls(mp, orc, C, method, panel):
    _pair(mp, orc, C, 300, 3, 40, panel=panel, method=method)
    _pair(mp, orc, C, 130, 2, 42, panel=panel, method=method)   # smaller second call


def test_noalloc_split_small_and_repeat(mp, orc):
    _pair(mp, orc, 2, 96, 1, 50, panel=32, method="split_i8")
    _pair(mp, orc, 2, 70, 1, 52, panel=32, method="split_i8")


def test_noalloc_rejects_beyond_scratch(mp):
    import torch

    n, nrhs = 1024, 300   # QD: the copy of B alone is 2*4*8*1024*300 bytes = 19.7 MB
    A = torch.zeros((2, 4, n, n), dtype=torch.float64, device="cuda")
    B = torch.zeros((2, 4, nrhs, n), dtype=torch.float64, device="cuda")
    with pytest.raises(mp.MPLUError, match="-103"):
        mp.gesv_noalloc(A, B)
