"""The per-pass timing module (python -m paper_1106_0557_amd.timing): one JSON line per
mesh with the time of every active pass, their sum and the solve's bytes over it."""
import json

import pytest
import torch

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    yield


@pytest.mark.parametrize("dtype,sizes", [("fp32", [32, 40, 60]), ("fp64", [128])])
def test_timing_lines(capsys, dtype, sizes):
    from paper_1106_0557_amd import Plan, timing

    assert timing.main(["--n", *map(str, sizes), "--dtype", dtype, "--reps", "2"]) == 0
    lines = [json.loads(l) for l in capsys.readouterr().out.splitlines() if l.startswith("{")]
    assert [d["n"] for d in lines] == sizes
    for d in lines:
        assert d["dtype"] == dtype and d["reps"] == 2
        passes = d["pass_ms"]
        n = d["n"]
        plan = Plan(n, n, n, h=1.0 / n, dtype=torch.float32 if dtype == "fp32" else torch.float64)
        fused = plan.fused
        plan.close()
        # fused plans (nx == ny, plane in LDS) skip the y passes; five-pass plans run all five
        want = {"x_fwd", "z_conv", "x_inv"} if fused else {"x_fwd", "y_fwd", "z_conv", "y_inv", "x_inv"}
        assert set(passes) == want
        assert all(v > 0 for v in passes.values())
        assert d["solve_ms"] == pytest.approx(sum(passes.values()), rel=1e-3, abs=1e-3)
        assert d["algorithmic_GBps"] > 0
