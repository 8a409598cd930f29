"""Mock galaxy surveys in the spirit of Sec. "Generating artificial observations".

The paper's own mock uses the SDSS DR7 completeness mask and an Eisenstein-Hu
spectrum, neither of which is available here; synthetic stand-ins keep the
structure:

* truth field: Gaussian, zero mean, P(k) = A k / (1 + (k / 0.02)^3) (k in h/Mpc),
  with A chosen so that the voxel variance of the field is exactly 0.25
  (sigma_delta = 0.5) under the unitary DFT convention;
* survey response R = C(angle) F(r), shared by all subsamples: an angular cap
  around +z seen from the box centre (optionally with 2-degree-wide rings at
  fixed polar angle and 0.5-degree circular holes) times the radial selection
  n(r) ~ r^2 exp(-(r / r_s)^1.5) normalised to a peak of 1;
* counts N^l = Nbar^l R (1 + b^l delta) + sqrt(Nbar^l R) eps, eps ~ N(0, 1),
  and N^l = 0 where R = 0 (the data model of eq. data_model with noise
  variance Nbar R, eq. cov_mat_noise).

Voxel centres sit at (i + 1/2) dx - L/2 from the observer at the box centre.
"""
from dataclasses import dataclass, field
from typing import List

import numpy as np


@dataclass
class MockConfig:
    name: str
    n: int
    box: float
    bias: List[float]
    nbar: List[float]
    nb: int
    cap_deg: float
    r_s: float
    rings_deg: List[float] = field(default_factory=list)
    n_holes: int = 0
    seed: int = 0
    mask_seed: int = 0
    fixed_mask: int = 1
    eps: float = 0.05
    nsteps: int = 20
    rj: bool = False

    @property
    def nsub(self):
        return len(self.bias)


def _survey(name, n, box, bias, nbar, nb, **kw):
    r_max = 0.7 * box
    return MockConfig(name, n, box, bias, nbar, nb, cap_deg=50.47, r_s=150.0 * r_max / 350.0,
                      rings_deg=[12.6, 25.2, 37.9], n_holes=200, **kw)


CONFIGS = {
    # 8^3 and 16^3: unit-test sizes (4 and 8 shells keep every shell populated)
    "tiny8": MockConfig("tiny8", 8, 500.0, [1.2], [2.0], 4, cap_deg=60.0, r_s=150.0),
    "tiny8x2": MockConfig("tiny8x2", 8, 500.0, [1.0, 1.4], [5.0, 1.0], 4, cap_deg=60.0,
                          r_s=150.0),
    "small16": MockConfig("small16", 16, 500.0, [1.0, 1.4], [5.0, 1.0], 8, cap_deg=60.0,
                          r_s=150.0),
    # plain method, CPU scale: 32^3, L = 500, one subsample (b = 1.2, Nbar = 2), 16 shells
    "cfg1": MockConfig("cfg1", 32, 500.0, [1.2], [2.0], 16, cap_deg=60.0, r_s=150.0,
                       eps=0.05, nsteps=20),
    # 128^3, L = 1000, four subsamples, 40 shells, 30 leapfrog steps, joint move on
    "cfg2": _survey("cfg2", 128, 1000.0, [1.0, 1.2, 1.4, 1.6], [5.0, 2.0, 1.0, 0.5], 40,
                    nsteps=30, eps=0.05, rj=True),
    # 256^3, L = 1500, six subsamples, 60 shells
    "cfg3": _survey("cfg3", 256, 1500.0, list(np.linspace(0.9, 2.0, 6)),
                    list(np.geomspace(8.0, 0.2, 6)), 60, nsteps=30, eps=0.05, rj=True),
    # batched-chain size groups (constant 7.8125 Mpc/h voxels)
    "grp64": _survey("grp64", 64, 500.0, [1.0, 1.2], [5.0, 2.0], 20, mask_seed=0, nsteps=30),
    "grp128": _survey("grp128", 128, 1000.0, [1.0, 1.2, 1.4, 1.6], [5.0, 2.0, 1.0, 0.5], 40,
                      mask_seed=1, nsteps=30),
    "grp192": _survey("grp192", 192, 1500.0, [1.0, 1.2, 1.4], [5.0, 2.0, 1.0], 60,
                      mask_seed=2, nsteps=30),
}


def fiducial_shape(k):
    """P(k) / A = k / (1 + (k / 0.02)^3), k in h/Mpc."""
    k = np.asarray(k, dtype=np.float64)
    return k / (1.0 + (k / 0.02) ** 3)


def _kmag(n, box):
    f = np.fft.fftfreq(n, d=1.0 / n)
    fz = np.arange(n // 2 + 1)
    q = f[:, None, None] ** 2 + f[None, :, None] ** 2 + fz[None, None, :] ** 2
    return 2.0 * np.pi / box * np.sqrt(q)


def amplitude(n, box, sigma2=0.25):
    """A such that (1/V) sum_{k != 0} P(k) over the full grid equals sigma2."""
    k = _kmag(n, box)
    w = np.full(k.shape, 2.0)
    w[:, :, 0] = 1.0
    w[:, :, n // 2] = 1.0
    s = fiducial_shape(k)
    s[0, 0, 0] = 0.0
    return sigma2 * box ** 3 / float(np.sum(w * s))


def shell_centres(n, box, nb):
    """k_m = (m + 1/2) k_corner / nb with k_corner = sqrt(3) (N/2) 2 pi / L."""
    kc = np.sqrt(3.0) * (n // 2) * 2.0 * np.pi / box
    return (np.arange(nb) + 0.5) * kc / nb


def gaussian_field(n, box, A, seed):
    """Truth delta: unitary transform of white noise scaled by sqrt(P N^3 / V)."""
    rng = np.random.default_rng(seed)
    w = rng.standard_normal((n, n, n))
    k = _kmag(n, box)
    lam = A * fiducial_shape(k) * n ** 3 / box ** 3
    lam[0, 0, 0] = 0.0
    wk = np.fft.rfftn(w, norm="ortho")
    return np.fft.irfftn(np.sqrt(lam) * wk, s=(n, n, n), axes=(0, 1, 2), norm="ortho")


def _directions(n, box):
    dx = box / n
    c = (np.arange(n) + 0.5) * dx - 0.5 * box
    x = c[:, None, None]
    y = c[None, :, None]
    z = c[None, None, :]
    r = np.sqrt(x * x + y * y + z * z)
    return x, y, z, r


def response(cfg):
    """R = C(angle) n(r), float64 [N][N][N]."""
    C, sel = mask_and_selection(cfg)
    return C * sel


def mask_and_selection(cfg):
    """Angular mask C and radial selection n(r) separately (float64 [N][N][N])."""
    n, box = cfg.n, cfg.box
    x, y, z, r = _directions(n, box)
    cos_t = z / r
    polar = np.degrees(np.arccos(np.clip(cos_t, -1.0, 1.0)))
    C = (polar <= cfg.cap_deg).astype(np.float64)
    for ring in cfg.rings_deg:
        C[np.abs(polar - ring) < 1.0] = 0.0
    if cfg.n_holes:
        rng = np.random.default_rng(1000 + cfg.mask_seed)
        ct = rng.uniform(np.cos(np.radians(cfg.cap_deg)), 1.0, cfg.n_holes)
        ph = rng.uniform(0.0, 2.0 * np.pi, cfg.n_holes)
        st = np.sqrt(1.0 - ct * ct)
        cen = np.stack([st * np.cos(ph), st * np.sin(ph), ct], axis=0)      # 3 x H
        u = np.stack(np.broadcast_arrays(x / r, y / r, z / r), axis=-1).reshape(-1, 3)
        flat = C.reshape(-1)
        cmin = np.cos(np.radians(0.5))
        chunk = 1 << 20
        for s in range(0, u.shape[0], chunk):
            dots = u[s:s + chunk] @ cen
            flat[s:s + chunk][dots.max(axis=1) > cmin] = 0.0
    rp = cfg.r_s * (4.0 / 3.0) ** (2.0 / 3.0)
    sel = (r / rp) ** 2 * np.exp(-((r / cfg.r_s) ** 1.5 - (rp / cfg.r_s) ** 1.5))
    return C, sel


def make_mock(cfg, dtype=np.float64, geometry=None):
    """Mock survey for `cfg`.  Returns a dict of arrays and scalars.

    R, counts: [c][N][N][N]; delta: truth field [N][N][N]; pk_init: prior
    spectrum at the shell centres, (Mpc/h)^3; A: spectrum amplitude; mask,
    sel: angular mask and radial selection.  geometry: (mask, sel) computed
    earlier by mask_and_selection for the same geometry (saves the mask).
    """
    n, box = cfg.n, cfg.box
    A = amplitude(n, box)
    delta = gaussian_field(n, box, A, cfg.seed)
    C, sel = mask_and_selection(cfg) if geometry is None else geometry
    R1 = C * sel
    obs = R1 > 0
    rng = np.random.default_rng(2000 + cfg.seed)
    c = cfg.nsub
    R = np.empty((c, n, n, n), dtype=dtype)
    counts = np.empty((c, n, n, n), dtype=dtype)
    for l in range(c):
        eps = rng.standard_normal((n, n, n))
        mu = cfg.nbar[l] * R1 * (1.0 + cfg.bias[l] * delta)
        counts[l] = np.where(obs, mu + np.sqrt(cfg.nbar[l] * R1) * eps, 0.0)
        R[l] = R1
    pk_init = A * fiducial_shape(shell_centres(n, box, cfg.nb))
    return dict(cfg=cfg, R=R, counts=counts, delta=delta, pk_init=pk_init, A=A,
                mask=C.astype(dtype), sel=sel.astype(dtype),
                bias=np.array(cfg.bias, dtype=np.float64),
                nbar=np.array(cfg.nbar, dtype=np.float64), n_obs=int(obs.sum()))
