"""P9 on the GPU: Stokes drag on a fixed D = 12 sphere in a periodic 96^3
box driven by a uniform force, against Hasimoto's simple-cubic-array law
F = 6 pi mu a U K(phi), with the multilinear and the cubic interpolation of
Eq. (lbm6)."""
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gpu():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1502_01159_amd import pibm

    pibm.lib()
    return pibm


@pytest.mark.parametrize("order", [2, 4])
def test_stokes_drag_hasimoto(gpu, order):
    """Re << 1, quasi-steady (the hydrodynamic radius changes by < 1% over the
    last 1000 steps), and the diffuse body's hydrodynamic radius lies between
    the point radius and one lattice unit beyond it, within 10% of R."""
    from paper_1502_01159_amd import stokes

    r = stokes.run(gpu, L=96, R=6.0, interp_order=order)
    print(r, flush=True)
    assert r["Re"] < 0.1
    assert r["drift"] < 1e-2
    assert r["R"] <= r["a"] <= r["R"] + 1.0
    assert abs(r["a_over_R"] - 1.0) <= 0.1
