"""GPU parity on the synthetic families of the size and density sweeps (Sec. 4:
Rmat-er with (0.25, 0.25, 0.25, 0.25) and Rmat-g with (0.45, 0.15, 0.15, 0.25)), at
sizes the oracle finishes in seconds, both conflict rules.  Exact equality."""
import pytest

from paper_1606_06025_amd import graphs as gg
from tests.test_parity_gpu import _assert_parity

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1606_06025_amd import _lib
    _lib.load()
    return torch.device("cuda:0")


@pytest.mark.parametrize("abcd", [gg.RMAT_ER, gg.RMAT_G])
@pytest.mark.parametrize("n,d", [(3000, 2), (100_000, 10), (300_000, 10), (65_536, 40), (20_000, 80)])
def test_sweep_family_parity(dev, abcd, n, d):
    g = gg.rmat_n(n, d, 3, abcd=abcd)
    _assert_parity(g, dev)
    _assert_parity(g, dev, rule=1)
