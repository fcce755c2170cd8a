"""The many-droplet workload as specified (G = -5.5, tau = 0.8) is unstable in
the FP64 oracle itself; tau = 1.0, the paper's Sec. III-A relaxation time,
is not.  This records the reading under which the benchmark runs that field at
tau = 1.0 (same geometry, same G)."""
import numpy as np

import oracle
from paper_2504_10539_amd import inputs


def _window(n):
    drops = inputs.many_droplets(4096, 2000, 8, 48, seed=3)
    return oracle.droplet_state(n, n, drops, seed=3, period=(4096, 4096))


def test_tau_0_8_window_goes_nonfinite_within_100_steps(nthreads):
    f = oracle.step(_window(512), -5.5, 0.8, 100, nthreads)
    assert not np.isfinite(oracle.density(f)).all()


def test_tau_1_0_window_stays_bounded(nthreads):
    f = oracle.step(_window(512), -5.5, 1.0, 100, nthreads)
    rho = oracle.density(f)
    assert np.isfinite(rho).all()
    # the initial transient overshoots the coexistence pair of G = -5.5
    # (0.105 / 2.31) to about 3.2 at step 100 and settles back below 2.6
    assert 0.05 < rho.min() and rho.max() < 4.0
