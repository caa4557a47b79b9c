"""Seeded synthetic inputs shared by the oracle and the GPU library.

This module holds data only -- geometry planes, material constants, run
configuration values and seeded primary generators.  It contains none of the
transport arithmetic, so both sides of every parity test can take their
inputs from here without sharing any of the method.

The calorimeter is the paper's validation set-up (section 2.2, "Physics
integration and validation": 50 layers, each an absorber slab of 2.3 mm and a
liquid-argon slab of 5.7 mm), with lead as the absorber instead of lead
tungstate, 40 x 40 cm transverse.  Primaries use numpy's Philox bit generator
so every workload is reproducible from its seed.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

# Species codes (gamma, electron, positron), shared by both C interfaces.
GAMMA, ELECTRON, POSITRON = 0, 1, 2

# Process-mask bits (same meaning on both sides).
P_COMPTON, P_PHOT, P_CONV, P_EIONI, P_EBREM, P_ANNIH, P_CONT = (1 << i for i in range(7))
P_ALL = 0x7F
# Optional along-step processes of e-/e+ (outside P_ALL): multiple
# scattering and fluctuations of the restricted loss.
P_MSC, P_FLUCT = 1 << 7, 1 << 8

# Materials: (Z, A [g/mol], density [g/cm3], mean excitation energy I [eV]).
# Z and density of lead and liquid argon as in the workload definition;
# A and I are the PDG values.
LEAD = (82.0, 207.2, 11.35, 823.0)
LIQUID_ARGON = (18.0, 39.948, 1.396, 188.0)


def compound(density_g_cm3: float, I_eV: float, elements) -> tuple:
    """A compound: (Z, A, rho, I, ((Z_i, A_i, atoms_i), ...)) with 1..4
    elements; the leading Z and A are the atom-averaged values (informative
    only, the elements define the material)."""
    els = tuple((float(z), float(a), float(n)) for z, a, n in elements)
    n = sum(e[2] for e in els)
    return (sum(e[0] * e[2] for e in els) / n, sum(e[1] * e[2] for e in els) / n,
            float(density_g_cm3), float(I_eV), els)


# Lead tungstate PbWO4, the absorber of the paper's validation calorimeter:
# PDG density and mean excitation energy, standard atomic weights.
LEAD_TUNGSTATE = compound(8.300, 600.7, ((82, 207.2, 1), (74, 183.84, 1), (8, 15.999, 4)))

# One primary record: 64 bytes, the layout both C interfaces declare.
PRIMARY_DTYPE = np.dtype(
    [("event", "<u4"), ("species", "<u4"), ("ekin", "<f8"), ("pos", "<f8", (3,)), ("dir", "<f8", (3,))],
    align=True,
)
assert PRIMARY_DTYPE.itemsize == 64


@dataclasses.dataclass
class Geometry:
    z_mm: np.ndarray          # n_slabs + 1 planes
    material: np.ndarray      # n_slabs indices (uint32)
    materials: list           # list of (Z, A, rho, I)
    half_xy_mm: float

    @property
    def n_slabs(self) -> int:
        return int(self.material.shape[0])

    @property
    def n_cols(self) -> int:
        """deposit columns: one per slab"""
        return self.n_slabs


@dataclasses.dataclass
class BoxGeometry:
    """Non-overlapping axis-aligned boxes inside a world box whose remaining
    volume is world_material; deposits per box, the world last."""
    lo: np.ndarray            # (n_boxes, 3) mm
    hi: np.ndarray            # (n_boxes, 3) mm
    material: np.ndarray      # n_boxes indices (uint32)
    materials: list
    world_lo: tuple
    world_hi: tuple
    world_material: int

    @property
    def n_boxes(self) -> int:
        return int(self.material.shape[0])

    @property
    def n_cols(self) -> int:
        return self.n_boxes + 1


def calorimeter(n_layers: int = 50, absorber_mm: float = 2.3, gap_mm: float = 5.7,
                half_xy_mm: float = 200.0, absorber=LEAD, gap=LIQUID_ARGON) -> Geometry:
    """Layered sampling calorimeter: slab 2l is absorber, slab 2l+1 is gap."""
    widths = np.tile(np.array([absorber_mm, gap_mm]), n_layers)
    z = np.concatenate([[0.0], np.cumsum(widths)])
    mat = np.tile(np.array([0, 1], dtype=np.uint32), n_layers)
    return Geometry(z_mm=z.astype(np.float64), material=mat, materials=[absorber, gap],
                    half_xy_mm=float(half_xy_mm))


def boxes_from_slabs(geo: Geometry) -> BoxGeometry:
    """The slab stack written as boxes: box k is slab k over the whole
    transverse extent, the world box is the stack itself."""
    n = geo.n_slabs
    h = geo.half_xy_mm
    lo = np.empty((n, 3))
    hi = np.empty((n, 3))
    lo[:, 0], lo[:, 1], lo[:, 2] = -h, -h, geo.z_mm[:-1]
    hi[:, 0], hi[:, 1], hi[:, 2] = h, h, geo.z_mm[1:]
    return BoxGeometry(lo=lo, hi=hi, material=geo.material.astype(np.uint32).copy(), materials=list(geo.materials),
                       world_lo=(-h, -h, float(geo.z_mm[0])), world_hi=(h, h, float(geo.z_mm[-1])),
                       world_material=int(geo.material[0]))


def towers(cells: int = 9, pitch_mm: float = 40.0, crack_mm: float = 1.0, n_layers: int = 50,
           absorber_mm: float = 2.3, gap_mm: float = 5.7, absorber=LEAD, gap=LIQUID_ARGON,
           margin_mm: float = 20.0) -> BoxGeometry:
    """A cells x cells array of sampling towers (the 50-layer absorber / gap
    sequence, each layer one box per tower) with cracks of crack_mm between
    towers; cracks and the surroundings are the world, of the gap material.
    Tower (i, j) is centred at ((i - c) pitch, (j - c) pitch), c = (cells - 1)/2;
    an odd count keeps the beam axis inside the central tower."""
    widths = np.tile(np.array([absorber_mm, gap_mm]), n_layers)
    z = np.concatenate([[0.0], np.cumsum(widths)])
    half = 0.5 * (pitch_mm - crack_mm)
    centres = (np.arange(cells) - 0.5 * (cells - 1)) * pitch_mm
    lo, hi, mat = [], [], []
    for i in range(cells):
        for j in range(cells):
            for k in range(2 * n_layers):
                lo.append((centres[i] - half, centres[j] - half, z[k]))
                hi.append((centres[i] + half, centres[j] + half, z[k + 1]))
                mat.append(k % 2)
    w = centres[-1] + half + margin_mm
    return BoxGeometry(lo=np.array(lo), hi=np.array(hi), material=np.array(mat, dtype=np.uint32),
                       materials=[absorber, gap], world_lo=(-w, -w, float(z[0])), world_hi=(w, w, float(z[-1])),
                       world_material=1)


def single_slab(thickness_mm: float, material=LEAD, half_xy_mm: float = 200.0) -> Geometry:
    return Geometry(z_mm=np.array([0.0, thickness_mm]), material=np.zeros(1, np.uint32),
                    materials=[material], half_xy_mm=float(half_xy_mm))


@dataclasses.dataclass
class RunConfig:
    """Physics and stepping configuration (values only)."""
    bz_tesla: float = 0.0
    gamma_cut_MeV: float = 0.1
    electron_cut_MeV: float = 0.2
    n_bins: int = 200
    emin_MeV: float = 1e-3
    emax_MeV: float = 1e8
    dr_over_range: float = 0.2
    final_range_mm: float = 1.0
    lin_loss_limit: float = 0.01
    process_mask: int = P_ALL
    max_steps_per_track: int = 100000
    seed: int = 1


def primaries(n: int) -> np.ndarray:
    return np.zeros(n, dtype=PRIMARY_DTYPE)


def beam(n_events: int, species: int, ekin_MeV: float, smear_rad: float = 0.0,
         seed: int = 0) -> np.ndarray:
    """One primary per event at the origin along +z, optional Gaussian
    angular smear of the x and y slopes (independent, sigma = smear_rad)."""
    p = primaries(n_events)
    p["event"] = np.arange(n_events, dtype=np.uint32)
    p["species"] = species
    p["ekin"] = ekin_MeV
    d = np.zeros((n_events, 3))
    d[:, 2] = 1.0
    if smear_rad > 0.0:
        rng = np.random.Generator(np.random.Philox(seed))
        tx = rng.normal(0.0, smear_rad, n_events)
        ty = rng.normal(0.0, smear_rad, n_events)
        d[:, 0] = np.tan(tx)
        d[:, 1] = np.tan(ty)
        d /= np.linalg.norm(d, axis=1)[:, None]
    p["dir"] = d
    return p


def mixed_species(n_events: int, e_lo_MeV: float = 1e3, e_hi_MeV: float = 1e5,
                  seed: int = 3) -> np.ndarray:
    """Species (e-, e+, gamma) by event index mod 3; energy log-uniform."""
    rng = np.random.Generator(np.random.Philox(seed))
    p = primaries(n_events)
    p["event"] = np.arange(n_events, dtype=np.uint32)
    order = np.array([ELECTRON, POSITRON, GAMMA], dtype=np.uint32)
    p["species"] = order[np.arange(n_events) % 3]
    p["ekin"] = np.exp(rng.uniform(math.log(e_lo_MeV), math.log(e_hi_MeV), n_events))
    p["dir"] = np.array([0.0, 0.0, 1.0])
    return p


def workload(name: str):
    """(geometry, config, primaries) of a named workload."""
    geo = calorimeter()
    if name == "cal_1GeV_e-_x32":
        return geo, RunConfig(seed=1), beam(32, ELECTRON, 1000.0)
    if name == "cal_10GeV_e-_x10k":
        return geo, RunConfig(seed=2), beam(10_000, ELECTRON, 10_000.0, smear_rad=1e-3, seed=2)
    if name == "cal_mixed_1-100GeV_bz3.8_x10k":
        return geo, RunConfig(seed=3, bz_tesla=3.8), mixed_species(10_000, seed=3)
    if name == "cal_10GeV_e-_x100k":
        return geo, RunConfig(seed=4), beam(100_000, ELECTRON, 10_000.0, smear_rad=1e-3, seed=4)
    if name == "cal_10GeV_e-_x10k_msc_fluct":
        # the benchmark beam with multiple scattering and loss fluctuations
        return geo, RunConfig(seed=7, process_mask=P_ALL | P_MSC | P_FLUCT), \
            beam(10_000, ELECTRON, 10_000.0, smear_rad=1e-3, seed=7)
    if name in ("towers_1GeV_e-_x32", "towers_10GeV_e-_x10k"):
        # 9 x 9 towers of the 50-layer sequence (8100 boxes, 1 mm cracks):
        # impact points uniform over the central 3 x 3 towers and their cracks
        n, e, seed = (32, 1000.0, 9) if name == "towers_1GeV_e-_x32" else (10_000, 10_000.0, 8)
        p = beam(n, ELECTRON, e, smear_rad=1e-3, seed=seed)
        rng = np.random.Generator(np.random.Philox(seed + 100))
        p["pos"][:, 0] = rng.uniform(-60.0, 60.0, n)
        p["pos"][:, 1] = rng.uniform(-60.0, 60.0, n)
        return towers(), RunConfig(seed=seed), p
    # the same stack with the paper's lead tungstate absorber
    pbwo4 = calorimeter(absorber=LEAD_TUNGSTATE)
    if name == "calPbWO4_1GeV_e-_x32":
        return pbwo4, RunConfig(seed=5), beam(32, ELECTRON, 1000.0)
    if name == "calPbWO4_10GeV_e-_x10k":
        return pbwo4, RunConfig(seed=6), beam(10_000, ELECTRON, 10_000.0, smear_rad=1e-3, seed=6)
    raise KeyError(name)


def random_tracks(n: int, n_events: int, geo: Geometry, e_lo: float, e_hi: float,
                  seed: int, species=None) -> np.ndarray:
    """Isotropic tracks at random points inside the stack (for edge cases)."""
    rng = np.random.Generator(np.random.Philox(seed))
    p = primaries(n)
    p["event"] = rng.integers(0, n_events, n).astype(np.uint32)
    p["species"] = rng.integers(0, 3, n) if species is None else species
    p["ekin"] = np.exp(rng.uniform(math.log(e_lo), math.log(e_hi), n))
    pos = np.empty((n, 3))
    pos[:, 0] = rng.uniform(-0.9, 0.9, n) * geo.half_xy_mm
    pos[:, 1] = rng.uniform(-0.9, 0.9, n) * geo.half_xy_mm
    pos[:, 2] = rng.uniform(geo.z_mm[0], geo.z_mm[-1], n)
    p["pos"] = pos
    d = rng.normal(size=(n, 3))
    d /= np.linalg.norm(d, axis=1)[:, None]
    p["dir"] = d
    return p


def serving_request(rng, e_median_MeV: float = 5000.0, sigma: float = 1.0, max_tracks: int = 200,
                    half_xy_mm: float = 200.0) -> np.ndarray:
    """One offload request: n ~ U{1..max_tracks} EM tracks of uniformly drawn
    species; total energy lognormal(ln e_median, sigma) clamped to
    [10 MeV, 2 TeV], split by a flat Dirichlet with every track >= 1 MeV;
    positions (N(0, 10 mm), N(0, 10 mm), 0) on the front face; directions +z
    with independent 1 mrad Gaussian slope smears.  `rng` is a
    numpy Generator."""
    etot = float(np.clip(rng.lognormal(math.log(e_median_MeV), sigma), 10.0, 2e6))
    n = int(rng.integers(1, max_tracks + 1))
    n = max(1, min(n, int(etot)))
    w = rng.dirichlet(np.ones(n))
    p = primaries(n)
    p["species"] = rng.integers(0, 3, n)
    p["ekin"] = 1.0 + (etot - n) * w
    pos = np.zeros((n, 3))
    pos[:, 0] = np.clip(rng.normal(0.0, 10.0, n), -0.9 * half_xy_mm, 0.9 * half_xy_mm)
    pos[:, 1] = np.clip(rng.normal(0.0, 10.0, n), -0.9 * half_xy_mm, 0.9 * half_xy_mm)
    p["pos"] = pos
    d = np.zeros((n, 3))
    d[:, 0] = np.tan(rng.normal(0.0, 1e-3, n))
    d[:, 1] = np.tan(rng.normal(0.0, 1e-3, n))
    d[:, 2] = 1.0
    p["dir"] = d / np.linalg.norm(d, axis=1)[:, None]
    return p
