"""Synthetic streamer-like fields on the workloads of the photoionization study.

Every array is drawn from ``numpy.random.default_rng(seed)`` or is fully
deterministic, so each side of a comparison rebuilds identical inputs.

Units: lengths in cm, quadrature weights in cm^3, the bare source I in
m^-3 s^-1 (the library and the oracle multiply by the quenching/efficiency
prefactor themselves), |E| in V/m.

Shapes follow the paper's workloads: single Gaussian emission sources
(Sec. 4.1, eq. (20); Sec. 4.2, eq. (21)) and a streamer head with a trailing
channel whose emission spans many decades (Sec. 5, where the field is
strongest ahead of the head and photoionization matters most there).
The Gaussian convention exp(-|x-x0|^2/sigma^2) is the one of eq. (20).
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Optional

import numpy as np

# Gas parameters (Sec. 4.1 and Sec. 5): p_q = 30 Torr, xi = 0.1, omega/alpha = 0.6,
# chi_min = 0.035 and chi_max = 2 cm^-1 Torr^-1 (Sec. 2.1, eq. (3)); p_O2 = 0.2 p.
GAS_760 = dict(p_torr=760.0, o2_fraction=0.2, pq_torr=30.0,
               xi_omega_over_alpha=0.06, chi_min=0.035, chi_max=2.0)
GAS_40 = dict(GAS_760, p_torr=40.0)

I_PEAK = 1e28          # peak emission, m^-3 s^-1
E_PEAK = 1.5e7         # V/m, field at the head
E_BG = 5e6             # V/m, background field
R0_FIELD = 0.05        # cm, radius inside which the head field is flat


@dataclass
class Workload:
    name: str
    xyz: np.ndarray                    # (n, 3) float64, cm, caller order
    I: np.ndarray                      # (n,) float64, bare source
    w: Optional[np.ndarray]            # (n,) float64 cm^3, None on a uniform grid
    h: float                           # grid spacing (cm), 0 for point clouds
    gas: dict
    thresholds: dict                   # src_rel, e_abs, e_applied, e_rel
    E: Optional[np.ndarray] = None     # (n,) float64 V/m, None when no field rule
    head: Optional[np.ndarray] = None  # (3,) cm
    domain: tuple = (0.0, 1.0)         # cube [lo, hi]^3, cm
    grid_n: int = 0                    # points per axis on a uniform grid
    meta: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.xyz.shape[0])

    def weights(self) -> np.ndarray:
        if self.w is not None:
            return self.w
        return np.full(self.n, self.h ** 3)


def grid_points(n_axis: int, lo: float, hi: float) -> tuple[np.ndarray, float]:
    """Cell centres of a uniform n^3 grid on [lo, hi]^3; index ((ix*n)+iy)*n+iz."""
    h = (hi - lo) / n_axis
    c = lo + (np.arange(n_axis) + 0.5) * h
    X, Y, Z = np.meshgrid(c, c, c, indexing="ij")
    xyz = np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1)
    return np.ascontiguousarray(xyz), h


def gaussian_ball(xyz: np.ndarray, centre, sigma: float) -> np.ndarray:
    d2 = ((xyz - np.asarray(centre)[None, :]) ** 2).sum(axis=1)
    return np.exp(-d2 / sigma ** 2)


def _streamer_I(xyz, head, sigma_h=0.02, r_channel=0.03, ell=0.3, amp_channel=1e-2,
                floor=1e-8, head_sigma_override=None):
    """Gaussian head plus a channel trailing along +z with axial decay ell."""
    sh = sigma_h if head_sigma_override is None else head_sigma_override
    d = xyz - head[None, :]
    head_part = np.exp(-(d ** 2).sum(axis=1) / sh ** 2)
    s = d[:, 2]                                   # distance behind the head along +z
    rho2 = d[:, 0] ** 2 + d[:, 1] ** 2
    chan = amp_channel * np.exp(-rho2 / r_channel ** 2) * np.exp(-np.clip(s, 0, None) / ell)
    chan = np.where(s >= 0.0, chan, 0.0)
    return I_PEAK * np.maximum(floor, head_part + chan)


def _head_field(xyz, head):
    r2 = ((xyz - head[None, :]) ** 2).sum(axis=1)
    with np.errstate(divide="ignore"):
        f = np.minimum(1.0, R0_FIELD ** 2 / np.maximum(r2, 1e-300))
    return E_BG + (E_PEAK - E_BG) * f


def config1() -> Workload:
    """24^3 cell-centred grid in a 2 mm cube, isotropic Gaussian blob plus background."""
    xyz, h = grid_points(24, 0.0, 0.2)
    x0 = np.array([0.1, 0.1, 0.1])
    I = I_PEAK * gaussian_ball(xyz, x0, 0.015) + 1e18
    return Workload("c1_gauss24", xyz, I, None, h, dict(GAS_760),
                    dict(src_rel=0.0, e_abs=-1.0, e_applied=0.0, e_rel=-1.0),
                    E=None, head=x0, domain=(0.0, 0.2), grid_n=24)


def config2(seed: int = 1000, n_axis: int = 128) -> Workload:
    """Streamer head + channel on a uniform grid in a 1 cm cube (default 128^3)."""
    rng = np.random.default_rng(seed)
    head = np.array([0.5 + rng.uniform(-0.1, 0.1), 0.5 + rng.uniform(-0.1, 0.1),
                     rng.uniform(0.3, 0.7)])
    xyz, h = grid_points(n_axis, 0.0, 1.0)
    I = _streamer_I(xyz, head)
    E = _head_field(xyz, head)
    return Workload(f"c2_streamer{n_axis}_s{seed}", xyz, I, None, h, dict(GAS_760),
                    dict(src_rel=1e-4, e_abs=3e6, e_applied=0.0, e_rel=-1.0),
                    E=E, head=head, domain=(0.0, 1.0), grid_n=n_axis)


def _lognormal_pdf(r, median, s):
    return np.exp(-((np.log(r) - np.log(median)) ** 2) / (2 * s * s)) / (r * s * np.sqrt(2 * np.pi))


def config3(seed: int = 2000, n: int = 4_000_000, gas: Optional[dict] = None,
            src_rel: float = 1e-4, clustered_frac: float = 0.7) -> Workload:
    """Nonuniform cloud in a 4 cm cube: log-normal radial cluster around the head plus uniform points.

    Quadrature weights are w_j = 1/(n rho(x_j)) with rho the known sampling density,
    so sum_j w_j f(x_j) is a Monte Carlo estimate of the volume integral.
    """
    rng = np.random.default_rng(seed)
    lo, hi = 0.0, 4.0
    head = np.array([2.0, 2.0, 2.0]) + rng.uniform(-0.2, 0.2, size=3)
    median, s_ln = 0.1, 1.0
    n_c = int(round(clustered_frac * n))
    n_u = n - n_c
    pts = []
    need = n_c
    while need > 0:
        m = int(need * 1.2) + 16
        r = np.exp(rng.normal(np.log(median), s_ln, size=m))
        u = rng.normal(size=(m, 3))
        u /= np.linalg.norm(u, axis=1, keepdims=True)
        p = head[None, :] + r[:, None] * u
        ok = np.all((p > lo) & (p < hi), axis=1)
        p = p[ok][:need]
        pts.append(p)
        need -= p.shape[0]
    clustered = np.concatenate(pts, axis=0)
    uniform = rng.uniform(lo, hi, size=(n_u, 3))
    xyz = np.ascontiguousarray(np.concatenate([clustered, uniform], axis=0))
    # in-cube mass of the cluster law (Monte Carlo, fixed seed)
    mc = np.random.default_rng(seed + 1)
    m = 400_000
    r = np.exp(mc.normal(np.log(median), s_ln, size=m))
    u = mc.normal(size=(m, 3))
    u /= np.linalg.norm(u, axis=1, keepdims=True)
    p = head[None, :] + r[:, None] * u
    Z = float(np.mean(np.all((p > lo) & (p < hi), axis=1)))
    rr = np.linalg.norm(xyz - head[None, :], axis=1)
    rho = clustered_frac * _lognormal_pdf(rr, median, s_ln) / (4 * np.pi * rr ** 2 * Z) \
        + (1 - clustered_frac) / (hi - lo) ** 3
    w = 1.0 / (n * rho)
    I = _streamer_I(xyz, head)
    E = _head_field(xyz, head)
    return Workload(f"c3_cloud{n}_s{seed}", xyz, I, w, 0.0, dict(gas or GAS_760),
                    dict(src_rel=src_rel, e_abs=3e6, e_applied=0.0, e_rel=-1.0),
                    E=E, head=head, domain=(lo, hi), grid_n=0, meta=dict(Z=Z))


def config5(seed: int = 3000, n_axis: int = 256) -> Workload:
    """Streamer head (sigma 0.15 mm) ahead of a Gaussian plasma cloud, 2 cm cube (default 256^3).

    The cloud (radius 2 mm) sits 5 mm ahead of the head, i.e. along -z; its
    surface layer emits at 1e-3 of the head peak.
    """
    rng = np.random.default_rng(seed)
    lo, hi = 0.0, 2.0
    head = np.array([1.0 + rng.uniform(-0.1, 0.1), 1.0 + rng.uniform(-0.1, 0.1),
                     rng.uniform(1.1, 1.3)])
    xyz, h = grid_points(n_axis, lo, hi)
    I = _streamer_I(xyz, head, head_sigma_override=0.015)
    cloud = head - np.array([0.0, 0.0, 0.5])
    d = np.linalg.norm(xyz - cloud[None, :], axis=1)
    I = I + 1e-3 * I_PEAK * np.exp(-((d - 0.2) ** 2) / 0.02 ** 2)
    E = _head_field(xyz, head)
    return Workload(f"c5_cloud{n_axis}_s{seed}", xyz, I, None, h, dict(GAS_760),
                    dict(src_rel=1e-4, e_abs=3e6, e_applied=0.0, e_rel=-1.0),
                    E=E, head=head, domain=(lo, hi), grid_n=n_axis, meta=dict(cloud=cloud))


def sample_targets(active_idx: np.ndarray, xyz: np.ndarray, head, k: int = 10_000,
                   seed: int = 12345, head_radius: float = 0.1, head_cap: int = 10_000) -> np.ndarray:
    """k targets drawn uniformly from ``active_idx`` plus the ones within head_radius of the head."""
    rng = np.random.default_rng(seed)
    active_idx = np.asarray(active_idx, dtype=np.int64)
    pick = active_idx if active_idx.size <= k else rng.choice(active_idx, size=k, replace=False)
    near = active_idx[np.linalg.norm(xyz[active_idx] - np.asarray(head)[None, :], axis=1) <= head_radius]
    if near.size > head_cap:
        near = rng.choice(near, size=head_cap, replace=False)
    return np.unique(np.concatenate([pick, near]))
