"""GPU parity of the learned-mass density trajectory with the float64 oracle."""
import numpy as np
import pytest

from gpu_common import chain_spec, coefficients32, mock, oracle_posterior, plain_mock, rel_l2, start_state
from oracle import hmc

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_1306_1821_amd.binding import Sampler  # noqa: E402

CASES = [("tiny8x2", 0.1, 8), ("small16", 0.08, 10), ("cfg1", 0.05, 12), (64, 0.04, 8)]


def case_mock(c):
    return mock(c) if isinstance(c, str) else plain_mock(c, 500.0, 20, nsub=2)


@pytest.mark.parametrize("case,eps,nsteps", CASES)
def test_learned_trajectory_matches_oracle(case, eps, nsteps):
    mk = case_mock(case)
    n = mk["cfg"].n
    rng = np.random.default_rng(n)
    logvar = (0.6 * rng.standard_normal((n, n, n)) - 2.0).astype(np.float32)
    a32, b32 = coefficients32(mk)
    s = Sampler([chain_spec(mk, eps=eps, nsteps=nsteps, seed=43)])
    s.set_coefficients(0, a32, b32)
    s.set_state(0, start_state(mk)[0])
    s.set_mass(0, logvar)
    post = oracle_posterior(mk, a32, b32, workers=4)
    sqrtD = hmc.mass_factor(logvar.astype(np.float64))
    for traj in range(2):
        before = s.state(0)
        dH, acc = s.trajectory(traj)
        st = s.state(0)
        ref = hmc.trajectory_learned(before["delta_k"].astype(np.complex128), post, sqrtD, eps,
                                     nsteps, 43, 0, traj)
        e_p = rel_l2(st["mom_k"], ref["p1"])
        print(f"N={n} traj {traj}: dH gpu {dH[0]:.6e} oracle {ref['dH']:.6e}; p rel-L2 {e_p:.2e}")
        assert e_p < 1e-4
        assert abs(dH[0] - ref["dH"]) < 2e-3 * max(1.0, abs(ref["dH"]))
        if abs(ref["log_u"] + ref["dH"]) > 1e-2:
            assert bool(acc[0]) == ref["accepted"]
        if acc[0]:
            assert rel_l2(st["delta_k"], ref["proposal"]) < 1e-4
            assert rel_l2(st["delta_r"], ref["delta1"]) < 1e-4
    # back to the plain mass: trajectories match the plain oracle again
    s.set_mass(0, None)
    before = s.state(0)
    dH, acc = s.trajectory(9)
    ref = hmc.trajectory(before["delta_k"].astype(np.complex128), post, eps, nsteps, 43, 0, 9)
    assert rel_l2(s.state(0)["mom_k"], ref["p1"]) < 1e-4
    s.close()
