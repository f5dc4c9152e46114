"""The set-up tuning cache: a first set-up times its choices (the fused
Chebyshev step's variant, the V(2,2) smoothing launch pattern) and records
them; a second set-up of the same problem reads them instead of timing, makes
the same choices and so solves bit for bit the same."""
import os

import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from paper_2303_10233_amd import eth  # noqa: E402


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    eth.load_library()


@pytest.mark.parametrize("n,prec", [(128, eth.MIXED), (64, eth.FP64)])
def test_second_setup_reads_the_cache(n, prec, tmp_path, monkeypatch):
    import time
    path = tmp_path / "tune.txt"
    monkeypatch.setenv("ETH_TUNE_CACHE", str(path))
    print(f"[tuning cache] n={n} prec={prec}", flush=True)
    t0 = time.perf_counter()
    P = eth.Problem(n, precision=prec)
    torch.cuda.synchronize()
    cold = time.perf_counter() - t0
    timed, cached = P.tuning_source()
    assert timed >= 2 and cached == 0, (timed, cached)
    lines = path.read_text().splitlines()
    assert any(" mq_cheb_fused " in ln for ln in lines) and any(" vcycle_smoothing " in ln for ln in lines)
    t0 = time.perf_counter()
    Q = eth.Problem(n, precision=prec)
    torch.cuda.synchronize()
    warm = time.perf_counter() - t0
    assert Q.tuning_source() == (0, timed)
    assert Q.mq_variant() == P.mq_variant()
    print(f"  set-up cold {cold:.3f} s, warm {warm:.3f} s, choices {lines}", flush=True)
    b = P.assemble_rhs()
    xp, ip = P.solve(b, rtol=1e-8, maxit=500, use_graph=True)
    xq, iq = Q.solve(Q.assemble_rhs(), rtol=1e-8, maxit=500, use_graph=True)
    assert ip[0]["iterations"] == iq[0]["iterations"]
    assert torch.equal(xp, xq)
    # an empty path disables the cache: everything is timed again
    monkeypatch.setenv("ETH_TUNE_CACHE", "")
    R = eth.Problem(n, precision=prec)
    assert R.tuning_source() == (timed, 0)
    P.close()
    Q.close()
    R.close()
