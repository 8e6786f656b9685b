"""Long-time precession under uniaxial anisotropy on the HIP path (Results A:
the Kittel-mode benchmark of a 128-spin bcc Fe block, 20 degrees from the
easy axis, weak damping).

A uniform ferromagnet feels no exchange torque, so every spin follows the
single-spin LLG in the anisotropy field H_K cos(theta) z, H_K = 2K/(mu mu_B):
cot(theta) = cot(theta_0) e^{lam t} with lam = alpha gamma' H_K, and the
azimuth phi = (asinh(cot theta) - asinh(cot theta_0)) / alpha, where
gamma' = gamma / (1 + alpha^2).  The colour sweep keeps the block uniform
only up to its splitting error, which this test bounds over 25 periods (the
FP64 oracle gives 1.7e-3 at a 0.5 fs step and 4.3e-4 at 0.25 fs).
"""
import math
import sys

import numpy as np
import pytest

from paper_2608_18541_amd import inputs as I

pytestmark = pytest.mark.gpu

MUB = 5.7883818060e-5
HBAR = 6.582119569e-4
GAMMA = 2.0 * MUB / HBAR


@pytest.fixture(scope="module")
def N():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2608_18541_amd import native
    native.lib()
    return native


def _kittel_errors(N, prec, dt):
    """Relative phase error at the end and largest cone-amplitude error of
    the block's magnetisation against the closed form over 25 periods."""
    K, alpha, mu = 1.0e-3, 0.01, 2.2
    th0 = math.radians(20.0)
    spec = I.fe_bcc_spec(L=4, lattice_mode=0, ttm_mode=0, Te0=0.0, B=(0.0, 0.0, 0.0), alpha=alpha,
                         K=(K, 0.0, 0.0, 0.0), dt=dt)
    n = spec.n_sites
    assert n == 128
    HK = 2.0 * K / (mu * MUB)
    gp = GAMMA / (1.0 + alpha ** 2)
    period = 2.0 * math.pi / (gp * HK * math.cos(th0))
    steps = int(math.ceil(25 * period / dt / 20.0)) * 20
    spins = np.tile([math.sin(th0), 0.0, math.cos(th0)], (n, 1))
    st = I.InitialState(species=np.zeros(n, dtype=np.int8), spins=spins, vel=np.zeros((n, 3)))
    print("kittel: prec=%d dt=%g steps=%d period=%.3f ps" % (prec, dt, steps, period), flush=True)
    sys.stdout.flush()
    s = N.System(spec, st, precision=prec, obs_every=20, obs_capacity=steps // 20 + 2)
    s.step(steps)
    obs = s.observables()
    s.close()
    t = np.array([o["t"] for o in obs])
    M = np.array([o["M"][0] for o in obs])
    assert len(t) == steps // 20 + 1
    # the block stays uniform: |m| = 1 to the splitting error
    assert np.abs(np.linalg.norm(M, axis=1) - 1.0).max() < 1e-6
    th = np.arccos(np.clip(M[:, 2] / np.linalg.norm(M, axis=1), -1.0, 1.0))
    phi = np.unwrap(np.arctan2(M[:, 1], M[:, 0]))
    lam = alpha * gp * HK
    cot_ref = (1.0 / math.tan(th0)) * np.exp(lam * t)
    th_ref = np.arctan2(1.0, cot_ref)
    phi_ref = (np.arcsinh(cot_ref) - math.asinh(1.0 / math.tan(th0))) / alpha
    # about 25 turns and a visible decay of the cone angle
    assert phi_ref[-1] / (2 * math.pi) > 24.0 and th_ref[-1] < 0.3 * th0
    e_phase = abs(phi[-1] - phi_ref[-1]) / phi_ref[-1]
    e_env = np.abs(np.sin(th) - np.sin(th_ref)).max() / math.sin(th0)
    print("kittel: prec=%d dt=%g phase rel err %.3e, envelope rel err %.3e"
          % (prec, dt, e_phase, e_env), flush=True)
    return e_phase, e_env


def test_kittel_precession_fp64_second_order(N):
    """FP64 at two step sizes: both within the paper's 1e-2 on the frequency
    and the envelope, and the error falls by four when the step halves (the
    palindromic colour sweep is second order)."""
    a = _kittel_errors(N, 0, 5.0e-4)
    b = _kittel_errors(N, 0, 2.5e-4)
    for e in a + b:
        assert e < 1e-2
    for x, y in zip(a, b):
        assert 3.5 < x / y < 4.5, (a, b)


def test_kittel_precession_fp32(N):
    e_phase, e_env = _kittel_errors(N, 1, 5.0e-4)
    assert e_phase < 1e-2 and e_env < 1e-2
