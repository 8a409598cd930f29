"""Shared helpers for the GPU parity tests: inputs from synth, oracle posteriors
built from the same float32 arrays the GPU receives."""
import numpy as np

from oracle import grid, hmc, model
from synth import CONFIGS, MockConfig, make_mock

_MOCKS = {}


def mock(name):
    if name not in _MOCKS:
        _MOCKS[name] = make_mock(CONFIGS[name], dtype=np.float32)
    return _MOCKS[name]


def plain_mock(n, box, nb, nsub=1, seed=0):
    """A cap-masked single-R mock of any supported size (for sizes without a config)."""
    cfg = MockConfig(f"plain{n}", n, box, [1.0 + 0.2 * l for l in range(nsub)],
                     [3.0 / (l + 1) for l in range(nsub)], nb, cap_deg=60.0,
                     r_s=150.0 * 0.7 * box / 350.0, seed=seed)
    key = (n, box, nb, nsub, seed)
    if key not in _MOCKS:
        _MOCKS[key] = make_mock(cfg, dtype=np.float32)
    return _MOCKS[key]


def chain_spec(mk, **kw):
    cfg = mk["cfg"]
    spec = dict(n=cfg.n, box=cfg.box, nb=cfg.nb, R=mk["R"], counts=mk["counts"],
                bias=mk["bias"], nbar=mk["nbar"], pk=mk["pk_init"], fixed_mask=cfg.fixed_mask,
                nsteps=cfg.nsteps, eps=cfg.eps, rj=cfg.rj)
    spec.update(kw)
    return spec


def coefficients32(mk):
    """alpha, beta from the oracle, rounded to float32 (the arrays both sides then use)."""
    a, b, _ = model.coefficients(mk["R"].astype(np.float64), mk["counts"].astype(np.float64),
                                 mk["bias"], mk["nbar"])
    return a.astype(np.float32), b.astype(np.float32)


def oracle_posterior(mk, a32, b32, pk=None, workers=1):
    cfg = mk["cfg"]
    n, nb = cfg.n, cfg.nb
    shells = grid.half_shells(n, nb)
    alpha = a32.astype(np.float64)
    beta = b32.astype(np.float64)
    abar = float(alpha.mean())
    lam = model.lambdas(mk["pk_init"] if pk is None else pk, n, cfg.box)
    return hmc.Posterior(n, cfg.box, nb, shells, grid.half_weights(n), model.per_mode(lam, shells),
                         model.per_mode(model.mass_table(lam, abar), shells), alpha, beta, abar,
                         workers)


def rel_l2(a, b):
    a = np.asarray(a, dtype=np.complex128).ravel()
    b = np.asarray(b, dtype=np.complex128).ravel()
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def start_state(mk):
    """delta_hat of the truth field, float64 (k = 0 removed), from its float32 copy."""
    d32 = mk["delta"].astype(np.float32)
    dk = grid.fwd(d32.astype(np.float64))
    dk[0, 0, 0] = 0.0
    return d32, dk


def dh_tol(n):
    """Bound on |dH_gpu - dH_oracle| end to end for an N^3 chain.

    The state (delta_hat, p_hat) is float32 on the device and float64 in the
    oracle; the energies are float64 sums on both sides, and on identical arrays
    they agree to 1e-9 (the evaluation itself).  End to end, each of the N^3
    per-voxel energy terms carries the rounding its float32 state accumulated
    over the trajectory's transforms and updates, and these add up as a random
    walk: |dH_32 - dH_64| ~ c u sqrt(N^3), u = 2^-24.  Measured over 8^3 - 256^3
    (trajectories of 4 - 20 steps from the mocks' truth fields) the coefficient
    c u stays between 1.5e-7 and 5.7e-7 (about 3 - 10 u); the bound takes
    2e-6 sqrt(N^3), 3.5 times the largest (4.5e-5 at 8^3, 8.2e-3 at 256^3).
    """
    return 2e-6 * float(n) ** 1.5
