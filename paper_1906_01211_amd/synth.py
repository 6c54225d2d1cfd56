"""Seeded synthetic water boxes (input generation only; no force-field arithmetic).

The paper's benchmark systems (DHFR, the Puddle water box; Table of the
molecular systems) are not available, so liquid-density water boxes of the
same atom counts stand in for them.  This module only draws coordinates and
per-atom parameters; it serves both the GPU path and the CPU oracle and holds
none of the method's arithmetic.

Recipe (fixed; the draw order is part of it):
  * waters sit on a cubic lattice of n_side = ceil(n_w^(1/3)) sites per edge,
    spacing a = L / n_side, site centres at (i + 1/2) a; if n_w < n_side^3 a
    seeded subset of n_w sites is used (kept in lattice order);
  * oxygen = centre + U(-0.2, 0.2)^3 A (one draw per molecule);
  * orientation = rotation from a normalised 4-D Gaussian quaternion;
  * body-frame hydrogens at (+-0.9572 sin(52.26 deg), 0, 0.9572 cos(52.26 deg));
  * atom order O, H, H; molid = atom // 3; positions wrapped into [0, L);
  * RNG numpy.random.default_rng(seed), draws in the order
    sites -> jitter -> quaternions -> dipoles -> quadrupoles;
  * dipoles N(0, 0.05) per component (e*A); quadrupoles: six components
    N(0, 0.1) (xx, xy, xz, yy, yz, zz), symmetrised, trace/3 removed from the
    diagonal (e*A^2).
"""
from dataclasses import dataclass, field
from typing import Dict, Optional

import numpy as np

OH_BOND = 0.9572
HOH_ANGLE_DEG = 104.52


@dataclass
class WaterBox:
    xyz: np.ndarray        # [n,3] float64, A, in [0, L)
    box: float             # cubic edge, A
    molid: np.ndarray      # [n] int32
    mpole: np.ndarray      # [n,10] float64: q, mu(3), Txx Txy Txz Tyy Tyz Tzz
    polarity: np.ndarray   # [n] float64, A^3
    thole: np.ndarray      # [n] float64
    vdw_rad: np.ndarray    # [n] float64: HAL R (A) or LJ sigma (A)
    vdw_eps: np.ndarray    # [n] float64, kcal/mol
    params: Dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.xyz.shape[0])

    @property
    def charges(self) -> np.ndarray:
        return np.ascontiguousarray(self.mpole[:, 0])


def _rotations(q: np.ndarray) -> np.ndarray:
    q = q / np.linalg.norm(q, axis=1, keepdims=True)
    w, x, y, z = q[:, 0], q[:, 1], q[:, 2], q[:, 3]
    R = np.empty((q.shape[0], 3, 3))
    R[:, 0, 0] = 1 - 2 * (y * y + z * z)
    R[:, 0, 1] = 2 * (x * y - z * w)
    R[:, 0, 2] = 2 * (x * z + y * w)
    R[:, 1, 0] = 2 * (x * y + z * w)
    R[:, 1, 1] = 1 - 2 * (x * x + z * z)
    R[:, 1, 2] = 2 * (y * z - x * w)
    R[:, 2, 0] = 2 * (x * z - y * w)
    R[:, 2, 1] = 2 * (y * z + x * w)
    R[:, 2, 2] = 1 - 2 * (x * x + y * y)
    return R


def water_geometry(n_w: int, box: float, seed: int):
    """Returns (xyz[3 n_w, 3], molid, rng) after the site/jitter/quaternion draws."""
    rng = np.random.default_rng(seed)
    n_side = int(np.ceil(round(n_w ** (1.0 / 3.0), 9)))
    while n_side ** 3 < n_w:
        n_side += 1
    n_sites = n_side ** 3
    a = box / n_side
    if n_w == n_sites:
        sites = np.arange(n_sites)
    else:
        sites = np.sort(rng.choice(n_sites, size=n_w, replace=False))
    ix, iy, iz = np.unravel_index(sites, (n_side, n_side, n_side))
    centres = (np.stack([ix, iy, iz], axis=1) + 0.5) * a
    oxy = centres + rng.uniform(-0.2, 0.2, size=(n_w, 3))
    rot = _rotations(rng.standard_normal((n_w, 4)))
    half = np.deg2rad(HOH_ANGLE_DEG / 2.0)
    body = np.array([[0.0, 0.0, 0.0],
                     [OH_BOND * np.sin(half), 0.0, OH_BOND * np.cos(half)],
                     [-OH_BOND * np.sin(half), 0.0, OH_BOND * np.cos(half)]])
    xyz = oxy[:, None, :] + np.einsum("mab,kb->mka", rot, body)
    xyz = xyz.reshape(-1, 3)
    xyz = xyz - box * np.floor(xyz / box)
    xyz[xyz >= box] -= box  # guard the rounding edge of the wrap
    molid = (np.arange(3 * n_w) // 3).astype(np.int32)
    return np.ascontiguousarray(xyz), molid, rng


def amoeba_water_box(n_w: int, box: float, seed: int, *, dip_sigma: float = 0.05,
                     quad_sigma: float = 0.1) -> WaterBox:
    """AMOEBA-style water: charges O -0.52 / H +0.26, random lab-frame dipoles and
    traceless quadrupoles, polarizabilities O 0.837 / H 0.496 A^3, Thole 0.39,
    HAL O (3.405 A, 0.11) / H (2.655 A, 0.0135)."""
    xyz, molid, rng = water_geometry(n_w, box, seed)
    n = 3 * n_w
    is_o = (np.arange(n) % 3) == 0
    mpole = np.zeros((n, 10))
    mpole[:, 0] = np.where(is_o, -0.52, 0.26)
    mpole[:, 1:4] = rng.normal(0.0, dip_sigma, size=(n, 3))
    raw = rng.normal(0.0, quad_sigma, size=(n, 6))
    T = np.zeros((n, 3, 3))
    T[:, 0, 0], T[:, 0, 1], T[:, 0, 2] = raw[:, 0], raw[:, 1], raw[:, 2]
    T[:, 1, 1], T[:, 1, 2], T[:, 2, 2] = raw[:, 3], raw[:, 4], raw[:, 5]
    T = T + np.transpose(T, (0, 2, 1)) - T * np.eye(3)[None]  # symmetrise (keep diagonal)
    tr = np.trace(T, axis1=1, axis2=2) / 3.0
    T = T - tr[:, None, None] * np.eye(3)[None]
    mpole[:, 4] = T[:, 0, 0]
    mpole[:, 5] = T[:, 0, 1]
    mpole[:, 6] = T[:, 0, 2]
    mpole[:, 7] = T[:, 1, 1]
    mpole[:, 8] = T[:, 1, 2]
    mpole[:, 9] = T[:, 2, 2]
    return WaterBox(
        xyz=xyz, box=float(box), molid=molid, mpole=np.ascontiguousarray(mpole),
        polarity=np.where(is_o, 0.837, 0.496).astype(np.float64),
        thole=np.full(n, 0.39),
        vdw_rad=np.where(is_o, 3.405, 2.655).astype(np.float64),
        vdw_eps=np.where(is_o, 0.11, 0.0135).astype(np.float64),
        params=dict(kind="amoeba", n_w=n_w, seed=seed))


def charge_lj_water_box(n_w: int, box: float, seed: int) -> WaterBox:
    """Three-site point-charge water: O -0.834 / H +0.417, LJ on O only
    (sigma 3.15 A, eps 0.152 kcal/mol), no dipoles or quadrupoles."""
    xyz, molid, _ = water_geometry(n_w, box, seed)
    n = 3 * n_w
    is_o = (np.arange(n) % 3) == 0
    mpole = np.zeros((n, 10))
    mpole[:, 0] = np.where(is_o, -0.834, 0.417)
    return WaterBox(
        xyz=xyz, box=float(box), molid=molid, mpole=mpole,
        polarity=np.zeros(n), thole=np.zeros(n),
        vdw_rad=np.where(is_o, 3.15, 0.0).astype(np.float64),
        vdw_eps=np.where(is_o, 0.152, 0.0).astype(np.float64),
        params=dict(kind="charge_lj", n_w=n_w, seed=seed))


FRAME_NONE, FRAME_Z_THEN_X, FRAME_BISECTOR = 0, 1, 2
FRAME_Z_ONLY, FRAME_Z_BISECTOR, FRAME_3FOLD = 3, 4, 5


def water_frames(n_w: int):
    """Local-frame topology of n_w waters (atoms O, H1, H2 per molecule): O
    bisector (z atom H1, x atom H2); each H Z-then-X (z atom O, x atom the
    other H).  Returns (frame_type[n] int32, frame_atoms[n, 3] int32: z, x, y
    atoms, -1 where a type takes none)."""
    n = 3 * n_w
    base = 3 * np.arange(n_w)
    ftype = np.zeros(n, np.int32)
    fat = np.full((n, 3), -1, np.int32)
    ftype[base] = FRAME_BISECTOR
    fat[base, 0], fat[base, 1] = base + 1, base + 2
    for h, other in ((1, 2), (2, 1)):
        ftype[base + h] = FRAME_Z_THEN_X
        fat[base + h, 0], fat[base + h, 1] = base, base + other
    return ftype, fat


def mixed_frames(n_w: int):
    """Every frame type on n_w >= 2 waters (a test topology, not a water
    model): the O of molecule k is bisector, Z-bisector or 3-fold (k mod 3;
    z atom H1, x atom H2, y atom the O of molecule k + 1); its H1 is
    Z-then-X or Z-only and its H2 the other (k mod 2; z atom O, x atom the
    other H).  Returns (frame_type[n], frame_atoms[n, 3]) as water_frames."""
    n = 3 * n_w
    ftype = np.zeros(n, np.int32)
    fat = np.full((n, 3), -1, np.int32)
    for k in range(n_w):
        o, h1, h2 = 3 * k, 3 * k + 1, 3 * k + 2
        ftype[o] = (FRAME_BISECTOR, FRAME_Z_BISECTOR, FRAME_3FOLD)[k % 3]
        fat[o, :2] = h1, h2
        if ftype[o] != FRAME_BISECTOR:
            fat[o, 2] = 3 * ((k + 1) % n_w)
        for h, other, t in ((h1, h2, k % 2), (h2, h1, 1 - k % 2)):
            fat[h, 0] = o
            if t == 0:
                ftype[h] = FRAME_Z_THEN_X
                fat[h, 1] = other
            else:
                ftype[h] = FRAME_Z_ONLY
    return ftype, fat


def water_vdw_reduction(n_w: int, red_h: float = 0.91):
    """vdW reduction topology of n_w waters: each H's parent is its O, with
    reduction factor red_h (AMOEBA water's value, 0.91); O has none.  Returns
    (parent[n] int32, -1 for none; red[n] float64)."""
    n = 3 * n_w
    parent = np.full(n, -1, np.int32)
    red = np.ones(n)
    base = 3 * np.arange(n_w)
    for h in (1, 2):
        parent[base + h] = base
        red[base + h] = red_h
    return parent, red


def water_local_multipoles(n_w: int, seed: int) -> np.ndarray:
    """Multipoles in the local frames of water_frames: O -0.52 / H +0.26,
    dipoles along the local z axis (O 0.15, H -0.06 e A) with a small
    in-plane component, traceless quadrupoles (diagonal plus a small xz
    term), every value jittered by a few per cent (seeded)."""
    rng = np.random.default_rng(seed)
    n = 3 * n_w
    is_o = (np.arange(n) % 3) == 0
    m = np.zeros((n, 10))
    m[:, 0] = np.where(is_o, -0.52, 0.26)
    m[:, 1] = np.where(is_o, 0.0, 0.02)
    m[:, 3] = np.where(is_o, 0.15, -0.06)
    m[:, 4] = np.where(is_o, 0.30, 0.03)
    m[:, 7] = np.where(is_o, -0.45, -0.02)
    m[:, 6] = np.where(is_o, 0.0, 0.01)
    m[:, 1:] *= 1.0 + 0.05 * rng.standard_normal((n, 9))
    m[:, 9] = -(m[:, 4] + m[:, 7])
    return m


# Workload settings (readings: Ewald beta with erfc(beta rc) ~ 1e-8 at 7 A,
# list cutoffs = kernel cutoffs + 1e-3 A skin, taper on [0.9 rc, rc]).
AMOEBA_SETTINGS = dict(rc_ewald=7.0, rc_vdw=9.0, skin=1e-3, beta=0.5446, tol_debye=1e-5,
                       maxiter=100, taper_frac=0.9, dhal=0.07, ghal=0.12)
CHARGE_SETTINGS = dict(rc_ewald=12.0, rc_vdw=12.0, skin=1e-3, beta=0.34, taper_frac=0.9)

CONFIGS = {
    # 216 waters, 648 atoms, 18.64 A box
    "water216": dict(builder=amoeba_water_box, n_w=216, box=18.64, seed=1000,
                     settings=AMOEBA_SETTINGS),
    # 7,853 waters, 23,559 atoms, 62.23 A box (DHFR-sized stand-in)
    "water7853": dict(builder=amoeba_water_box, n_w=7853, box=62.23, seed=1001,
                      settings=AMOEBA_SETTINGS),
    # 32,000 three-site waters, 96,000 atoms, 98.5 A box (Puddle-sized stand-in)
    "water32000_charge_lj": dict(builder=charge_lj_water_box, n_w=32000, box=98.5,
                                 seed=1003, settings=CHARGE_SETTINGS),
}


def make(name: str) -> WaterBox:
    c = CONFIGS[name]
    wb = c["builder"](c["n_w"], c["box"], c["seed"])
    wb.params.update(c["settings"])
    wb.params["name"] = name
    return wb


def serving_requests(count: int = 512, seed: int = 1004, lo: int = 300, hi: int = 30000,
                     density: float = 0.03335, rate: Optional[float] = None):
    """Request stream for the serving form: sizes log-uniform in [lo, hi] atoms,
    n_w = round(n/3), box L = (n_w/density)^(1/3) (water-box density), per-request
    seed 20000 + k.  With a rate (requests/s), Poisson arrival offsets are drawn
    from the same generator."""
    rng = np.random.default_rng(seed)
    n_atoms = np.exp(rng.uniform(np.log(lo), np.log(hi), size=count))
    n_w = np.maximum(1, np.rint(n_atoms / 3.0)).astype(int)
    boxes = (n_w / density) ** (1.0 / 3.0)
    arrivals = None
    if rate is not None:
        arrivals = np.cumsum(rng.exponential(1.0 / rate, size=count))
    return [dict(k=k, n_w=int(n_w[k]), box=float(boxes[k]), seed=20000 + k,
                 arrival=None if arrivals is None else float(arrivals[k]))
            for k in range(count)]
