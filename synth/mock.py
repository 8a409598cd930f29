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

Magnitude-binned surveys (MockConfig.lf, the paper's own test scenario of Sec.
"Generating artificial observations" with synthetic geometry): subsample l holds
the galaxies of absolute-magnitude bin [M_l, M_l+1] of [-23, -17]; its radial
selection f^l(r) is the fraction of the bin's Schechter luminosity function
(alpha = -1.05, M* - 5 log h = -20.44) visible within 14.5 < r_Petrosian < 17.77
at the voxel's luminosity distance (flat LCDM, Omega_m = 0.3, low-z Hubble flow
in h units), R^l = C f^l; the biases follow the luminosity-dependent relation
b^l = b* (a + b 10^(0.4 (M*_b - M^l)) + c (M^l - M*_b)) with a = 0.895,
b = 0.105, c = -0.040, M*_b = -20.83, b* = 1.2 at the bin centres M^l; Nbar^l is
the luminosity function integrated over the bin times the voxel volume, with
Phi* = 0.0149 h^3 Mpc^-3 (a stated normalisation; the paper leaves it free).
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
    lf: bool = False   # magnitude-binned subsamples from the Schechter luminosity function

    @property
    def nsub(self):
        return len(self.bias)


def _survey(name, n, box, bias, nbar, nb, **kw):
    r_max = 0.7 * box
    return MockConfig(name, n, box, bias, nbar, nb, cap_deg=50.47, r_s=150.0 * r_max / 350.0,
                      rings_deg=[12.6, 25.2, 37.9], n_holes=200, **kw)


# --------------------------------------------------------------------------- magnitude bins
LF_ALPHA, LF_MSTAR, LF_PHISTAR = -1.05, -20.44, 0.0149      # Schechter, r band, h units
BIAS_A, BIAS_B, BIAS_C, BIAS_MSTAR, BIAS_BSTAR = 0.895, 0.105, -0.040, -20.83, 1.2
M_BRIGHT, M_FAINT, R_BRIGHT, R_FAINT = -23.0, -17.0, 14.5, 17.77
OMEGA_M = 0.3


def schechter(M):
    """Phi(M) per unit magnitude (h^3 Mpc^-3) of the Schechter form (appendix)."""
    x = 10.0 ** (0.4 * (LF_MSTAR - np.asarray(M, dtype=np.float64)))
    return 0.4 * np.log(10.0) * LF_PHISTAR * x ** (LF_ALPHA + 1.0) * np.exp(-x)


def _lf_integral(lo, hi, pts=2001):
    """int_lo^hi Phi(M) dM (elementwise over arrays lo <= hi), composite Simpson."""
    lo, hi = np.broadcast_arrays(np.asarray(lo, np.float64), np.asarray(hi, np.float64))
    t = np.linspace(0.0, 1.0, pts)
    w = np.ones(pts)
    w[1:-1:2], w[2:-1:2] = 4.0, 2.0
    M = lo[..., None] + (hi - lo)[..., None] * t
    return (hi - lo) * (schechter(M) @ w) / (3.0 * (pts - 1))


def magnitude_bins(nsub):
    edges = np.linspace(M_BRIGHT, M_FAINT, nsub + 1)
    return edges, 0.5 * (edges[:-1] + edges[1:])


def lf_bias(M):
    """Luminosity-dependent bias at absolute magnitude M."""
    M = np.asarray(M, dtype=np.float64)
    return BIAS_BSTAR * (BIAS_A + BIAS_B * 10.0 ** (0.4 * (BIAS_MSTAR - M)) + BIAS_C * (M - BIAS_MSTAR))


def distance_modulus(r):
    """m - (M - 5 log h) at comoving distance r (Mpc/h): 5 log10 D_L + 25, D_L = (1 + z) r,
    z(r) from flat LCDM with Omega_m = OMEGA_M."""
    z = np.linspace(0.0, 1.0, 4001)
    ez = np.sqrt(OMEGA_M * (1.0 + z) ** 3 + 1.0 - OMEGA_M)
    chi = np.concatenate([[0.0], np.cumsum(0.5 * (1.0 / ez[1:] + 1.0 / ez[:-1]) * np.diff(z))])
    chi *= 299792.458 / 100.0
    zr = np.interp(np.asarray(r, np.float64), chi, z)
    return 5.0 * np.log10(np.maximum((1.0 + zr) * np.asarray(r, np.float64), 1e-6)) + 25.0


def lf_selection(r, nsub, table=8192):
    """f^l(r) for the nsub magnitude bins: [nsub] + r.shape (evaluated on a table of
    `table` radii up to max r, then linearly interpolated per voxel)."""
    edges, _ = magnitude_bins(nsub)
    r = np.asarray(r, np.float64)
    rt = np.linspace(0.0, float(r.max()) * 1.0001 + 1e-9, table)
    dm = distance_modulus(rt)
    m_lo, m_hi = R_BRIGHT - dm, R_FAINT - dm                 # visible absolute magnitudes
    out = np.empty((nsub,) + r.shape)
    for l in range(nsub):
        lo = np.clip(m_lo, edges[l], edges[l + 1])
        hi = np.clip(m_hi, edges[l], edges[l + 1])
        ft = _lf_integral(lo, hi, pts=401) / _lf_integral(edges[l], edges[l + 1])
        out[l] = np.interp(r, rt, ft)
    return out


def _lf_survey(name, n, box, nsub, nb, **kw):
    """The paper's magnitude-binned scenario on synthetic geometry."""
    _, mc = magnitude_bins(nsub)
    edges, _ = magnitude_bins(nsub)
    nbar = [float(_lf_integral(edges[l], edges[l + 1]) * (box / n) ** 3) for l in range(nsub)]
    cfg = _survey(name, n, box, [float(b) for b in lf_bias(mc)], nbar, nb, **kw)
    cfg.lf = True
    return cfg


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
    # the paper's scenario: 15 magnitude bins in [-23, -17], 128^3 at L = 750 Mpc/h
    "paper15": _lf_survey("paper15", 128, 750.0, 15, 40, nsteps=30, eps=0.05, rj=True,
                          mask_seed=3),
    # the same scenario at 64^3 (L = 375 Mpc/h, the same voxel size) for parity tests:
    # the smallest box whose survey cone reaches the brightest bin (r > ~250 Mpc/h)
    "paper15s": _lf_survey("paper15s", 64, 375.0, 15, 20, nsteps=20, eps=0.05, rj=True,
                           mask_seed=3),
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
    if cfg.lf:
        sel_l = lf_selection(_directions(n, box)[3], c)
    R = np.empty((c, n, n, n), dtype=dtype)
    counts = np.empty((c, n, n, n), dtype=dtype)
    for l in range(c):
        eps = rng.standard_normal((n, n, n))
        Rl = C * sel_l[l] if cfg.lf else R1
        ob = Rl > 0
        mu = cfg.nbar[l] * Rl * (1.0 + cfg.bias[l] * delta)
        counts[l] = np.where(ob, mu + np.sqrt(cfg.nbar[l] * Rl) * eps, 0.0)
        R[l] = Rl
        if cfg.lf:
            obs = obs | ob
    pk_init = A * fiducial_shape(shell_centres(n, box, cfg.nb))
    return dict(cfg=cfg, R=R, counts=counts, delta=delta, pk_init=pk_init, A=A,
                mask=C.astype(dtype), sel=sel.astype(dtype),
                bias=np.array(cfg.bias, dtype=np.float64),
                nbar=np.array(cfg.nbar, dtype=np.float64), n_obs=int(obs.sum()))
