"""The paper's pure-LBM protocol (Sec. III-A set-up, Sec. III-C steps) run
through the library, against the FP64 oracle taking the same steps."""
import numpy as np
import pytest

import oracle
from paper_2504_10539_amd import inputs
from tests.gpu_helpers import lbm, need_gpu

pytestmark = pytest.mark.gpu

KEYS = ("Gmax", "drho", "W_eff", "E_int")


@pytest.fixture(autouse=True)
def _gpu():
    need_gpu()


def _close(m, ref, n, rel):
    for k in KEYS:
        assert m[k] == pytest.approx(ref[k], rel=rel), k
    assert abs(m["W"] - ref["W"]) * n * n <= 2  # at most two cells across the threshold


def test_paper_protocol_matches_oracle(nthreads):
    from paper_2504_10539_amd import preset
    L = lbm()
    n, seg, every = 48, 100, 50
    r = preset.run(nx=n, segment=seg, every=every, fork_storage=L.LBM_F16_SHIFTED)
    assert [m["step"] for m in r["init_series"]] == list(range(0, 500, every))
    assert len(r["evolution_series"]) == 5 * (seg // every)
    assert [m["step"] for m in r["segment_ends"]] == [500 + seg * (k + 1) for k in range(5)]
    f = oracle.droplet_state(n, n, inputs.single_droplet(n, n / 6.0), seed=1)
    f = oracle.step(f, -5.5, 1.0, 500, nthreads)
    _close(r["after_init"], oracle.metrics(oracle.density(f)), n, 1e-5)
    for k in range(5):
        f = oracle.step(f, -5.5, 1.0, seg, nthreads)
        _close(r["segment_ends"][k], oracle.metrics(oracle.density(f)), n, 1e-5)
    final = oracle.metrics(oracle.density(f))
    for k in ("Gmax", "drho"):
        assert r["table_I"][k] == pytest.approx(final[k], rel=1e-5)
    for k in ("W_eff", "E_int"):
        assert r["table_II"][k] == pytest.approx(final[k], rel=1e-5)
    # the FP16-shifted fork from the common initialised state: metrics within 2%
    for k in ("Gmax", "drho"):
        assert r["fork"]["table_I"][k] == pytest.approx(final[k], rel=0.02)
    for k in ("W_eff", "E_int"):
        assert r["fork"]["table_II"][k] == pytest.approx(final[k], rel=0.02)
    assert np.isfinite([m["mass"] for m in r["evolution_series"]]).all()


def test_paper_protocol_with_the_pinn_branch():
    """The PINN-LBM branch of the protocol (Sec. III-C) forks from the same
    initialised state, trains and corrects before each of the five segments,
    and reports both columns of Tables I and II."""
    from paper_2504_10539_amd import preset
    r = preset.run(nx=48, segment=40, every=20, pinn_beta=0.5)
    assert len(r["pinn"]["segment_ends"]) == 5
    assert all(m["finite"] == 1 for m in r["pinn"]["segment_ends"])
    # the fork is a new run whose step count starts at the fork
    assert r["pinn"]["segment_ends"][-1]["step"] == 5 * 40
    assert r["segment_ends"][-1]["step"] == 500 + 5 * 40
    for k in ("W", "Gmax", "drho"):
        assert np.isfinite(r["pinn"]["table_I"][k])
    # the corrections changed the run
    assert r["pinn"]["table_II"]["E_int"] != r["table_II"]["E_int"]
