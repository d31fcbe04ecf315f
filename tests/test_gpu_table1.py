"""Table 1 (Sec. 3.1) on the GPU: the cavity with a concentric hot cylinder
run to a steady state, against the oracle's steady state (64^2) and against
the printed Nusselt numbers on the paper's 250^2 mesh."""
import os

import pytest

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def printed():
    rows = (l.split() for l in open(os.path.join(GOLDEN, "table1_nu.txt")) if l.strip() and not l.startswith("#"))
    return {(float(r), float(a)): float(v) for r, a, v in rows}


@pytest.fixture(scope="module")
def gpu():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1502_01159_amd import pibm

    pibm.lib()
    return pibm


def test_steady_nusselt_64_matches_oracle(gpu):
    """FP32 storage on the GPU and the FP64 oracle reach the same steady
    Nusselt number (the oracle's value is stored by
    tests/golden/make_table1_oracle.py)."""
    from paper_1502_01159_amd import table1

    stored = float([l for l in open(os.path.join(GOLDEN, "table1_oracle_64.txt")) if not l.startswith("#")][0])
    nu, steps, ok, _ = table1.run_case(gpu, 64, 1e4, 2.5, chunk=2500, tol=1e-5, max_steps=80000)
    print(f"n=64 Ra=1e4 Ar=2.5: Nu={nu:.6f} after {steps} steps (oracle {stored:.6f})", flush=True)
    assert ok
    assert abs(nu - stored) <= 1e-3 * stored, (nu, stored)


@pytest.mark.parametrize("Ra", [1e4, 1e5, 1e6])
@pytest.mark.parametrize("Ar", [5.0, 2.5, 1.67])
def test_table1_printed_nusselt_250(gpu, Ra, Ar):
    """All nine cases of Table 1: steady Nu on the paper's 250^2 mesh within
    5% of the printed "Present" value."""
    from paper_1502_01159_amd import table1

    nu, steps, ok, sec = table1.run_case(gpu, 250, Ra, Ar, chunk=5000, tol=2e-5, max_steps=600000)
    ref = printed()[(Ra, Ar)]
    print(f"n=250 Ra={Ra:g} Ar={Ar:g}: Nu={nu:.4f} printed {ref} after {steps} steps ({sec:.1f} s)", flush=True)
    assert ok
    assert abs(nu / ref - 1.0) <= 0.05, (nu, ref)
