"""Seeded synthetic workloads: voxel label images, parameter sets, arrival streams.

This module is shared by the HIP path, the oracle-based tests and the benchmark.
It holds none of the cell model's arithmetic (no fluxes, no kinetics, no open-
circuit potentials, no initial state): it only draws microstructures and
parameter tuples and converts a C-rate into an applied current.

Microstructure stand-in (the paper's stochastic generator, Sec. 2.1, needs
fitted parameters that the paper does not print): overlapping random spheres
per electrode slab, the separator all pore.  The paper's particle system is
fully connected by construction (Sec. 2.1, connectivity graph of the
tessellation), so solid voxels that are not face-connected to their own
current collector plane are returned to the pore phase, and pore voxels that
are not face-connected to the separator (closed porosity) are filled with the
surrounding electrode's solid.

Random numbers come from a counter-based generator, SplitMix64 (Steele,
Lea and Flood, "Fast splittable pseudorandom number generators", OOPSLA 2014):
the k-th draw of stream s is mix(s + (k+1) * golden_gamma), mix being the
SplitMix64 finaliser.  Uniform doubles take the top 53 bits.

Label convention: uint8 array of shape (nz, ny, nx) in C order, so the flat
index of voxel (i, j, k) is i + nx*(j + ny*k); k = 0 touches the anode current
collector, k = nz-1 the cathode current collector.  0 = pore (electrolyte),
1 = anode active material, 2 = cathode active material, 3 = Li-metal foil (the
counter electrode of a half cell, Sec. 2.2; a cell holds 2 or 3, not both).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field, asdict

import numpy as np

PORE, ANODE, CATHODE, FOIL = 0, 1, 2, 3

_GOLDEN = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def _mix64(z: np.ndarray) -> np.ndarray:
    z = z.astype(np.uint64)
    with np.errstate(over="ignore"):
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
    return z ^ (z >> np.uint64(31))


class Stream:
    """Counter-based SplitMix64 stream keyed by (seed, stream id)."""

    def __init__(self, seed: int, stream_id: int = 0):
        key = _mix64(np.array([(int(seed) * 0x100000001B3 + int(stream_id) * 0xD6E8FEB86659FD93)
                               & 0xFFFFFFFFFFFFFFFF], dtype=np.uint64))[0]
        self.key = np.uint64(key)
        self.counter = 0

    def u64(self, n: int) -> np.ndarray:
        k = np.arange(self.counter + 1, self.counter + 1 + n, dtype=np.uint64)
        self.counter += n
        with np.errstate(over="ignore"):
            z = self.key + k * _GOLDEN
        return _mix64(z)

    def uniform(self, n: int, lo: float = 0.0, hi: float = 1.0) -> np.ndarray:
        u = (self.u64(n) >> np.uint64(11)).astype(np.float64) * (1.0 / 9007199254740992.0)
        return lo + (hi - lo) * u


def _face_components(mask: np.ndarray):
    """6-connected components of a boolean volume (union-find free: scipy.ndimage)."""
    import scipy.ndimage as ndi
    struct = ndi.generate_binary_structure(3, 1)
    return ndi.label(mask, structure=struct)


def _fill_slab(lab: np.ndarray, z0: int, z1: int, phase: int, porosity: float,
               r_min: float, r_max: float, rng: Stream) -> None:
    nz, ny, nx = lab.shape
    target = int(math.ceil((1.0 - porosity) * nx * ny * (z1 - z0)))
    slab = lab[z0:z1]
    solid = int(np.count_nonzero(slab == phase))
    while solid < target:
        cx, cy, cz, r = rng.uniform(4)
        cx *= nx
        cy *= ny
        cz = z0 + cz * (z1 - z0)
        r = r_min + (r_max - r_min) * r
        i0, i1 = max(0, int(math.floor(cx - r))), min(nx, int(math.ceil(cx + r)) + 1)
        j0, j1 = max(0, int(math.floor(cy - r))), min(ny, int(math.ceil(cy + r)) + 1)
        k0, k1 = max(z0, int(math.floor(cz - r))), min(z1, int(math.ceil(cz + r)) + 1)
        if i0 >= i1 or j0 >= j1 or k0 >= k1:
            continue
        zz, yy, xx = np.meshgrid(np.arange(k0, k1) + 0.5, np.arange(j0, j1) + 0.5,
                                 np.arange(i0, i1) + 0.5, indexing="ij")
        inside = (xx - cx) ** 2 + (yy - cy) ** 2 + (zz - cz) ** 2 <= r * r
        box = lab[k0:k1, j0:j1, i0:i1]
        new = inside & (box != phase)
        solid += int(np.count_nonzero(new))
        box[new] = phase


def _clean_connectivity(lab: np.ndarray, z_an: int, z_sep: int) -> None:
    """Solid clusters that do not span their electrode -> pore; pore not connected
    to the separator -> solid of the electrode it sits in.

    A cluster spans its electrode when it is face-connected both to its collector
    plane and to the electrode's face on the separator.  Every other cluster is
    removed, as well as the isolated ones: a cluster that touches only the
    cathode collector would take its share of the applied current, which is spread
    evenly over the solid voxels of that plane, with no path to the rest of the
    electrode.  It would then use up its lithium within seconds, after which an
    implicit Euler step has no admissible solution.
    """
    nz = lab.shape[0]
    for phase, plane, sep_face in ((ANODE, 0, z_an - 1), (CATHODE, nz - 1, z_sep)):
        comp, n = _face_components(lab == phase)
        if n == 0:
            continue
        keep = np.intersect1d(np.unique(comp[plane][comp[plane] > 0]),
                              np.unique(comp[sep_face][comp[sep_face] > 0]))
        drop = (comp > 0) & ~np.isin(comp, keep)
        lab[drop] = PORE
    comp, n = _face_components(lab == PORE)
    sep_ids = np.unique(comp[z_an:z_sep][comp[z_an:z_sep] > 0])
    closed = (comp > 0) & ~np.isin(comp, sep_ids)
    if np.any(closed):
        kk = np.nonzero(closed)[0]
        lab[closed] = np.where(kk < z_an, ANODE, CATHODE).astype(np.uint8)


def sphere_cell(nx: int, ny: int, nz: int, seed: int, r_min: float, r_max: float,
                porosity_an: float, porosity_ca: float,
                layers: tuple[int, int, int] | None = None) -> np.ndarray:
    """Full-cell label image: anode slab | all-pore separator | cathode slab.

    `layers` = (anode, separator, cathode) thicknesses in voxels; default is the
    0.4 / 0.2 / 0.4 split of nz.  Redraws (new stream ids) until each collector
    plane holds solid of its electrode.
    """
    if layers is None:
        a = int(round(0.4 * nz))
        s = int(round(0.2 * nz))
        layers = (a, s, nz - a - s)
    if sum(layers) != nz or min(layers) < 1:
        raise ValueError(f"layers {layers} do not split nz={nz}")
    z_an, z_sep = layers[0], layers[0] + layers[1]
    for attempt in range(64):
        lab = np.zeros((nz, ny, nx), dtype=np.uint8)
        _fill_slab(lab, 0, z_an, ANODE, porosity_an, r_min, r_max, Stream(seed, 2 * attempt + 1))
        _fill_slab(lab, z_sep, nz, CATHODE, porosity_ca, r_min, r_max, Stream(seed, 2 * attempt + 2))
        _clean_connectivity(lab, z_an, z_sep)
        if np.any(lab[0] == ANODE) and np.any(lab[nz - 1] == CATHODE):
            return lab
    raise RuntimeError("could not draw a cell with solid on both collector planes")


def half_cell(nx: int, ny: int, nz: int, seed: int, r_min: float, r_max: float, porosity: float,
              layers: tuple[int, int, int]) -> np.ndarray:
    """Half-cell label image (Sec. 2.2): graphite slab | all-pore separator |
    Li-foil slab, `layers` = (graphite, separator, foil) thicknesses in voxels.
    The graphite is drawn and cleaned like a full cell's anode; the foil fills
    its slab."""
    if sum(layers) != nz or min(layers) < 1:
        raise ValueError(f"layers {layers} do not split nz={nz}")
    z_an, z_sep = layers[0], layers[0] + layers[1]
    for attempt in range(64):
        lab = np.zeros((nz, ny, nx), dtype=np.uint8)
        _fill_slab(lab, 0, z_an, ANODE, porosity, r_min, r_max, Stream(seed, 2 * attempt + 1))
        _clean_connectivity(lab, z_an, z_sep)
        lab[z_sep:] = FOIL
        if np.any(lab[0] == ANODE):
            return lab
    raise RuntimeError("could not draw a graphite slab with solid on its collector plane")


def anode_faces(labels: np.ndarray):
    """Anode/pore faces in canonical order (anode voxel index, then direction
    0:-x 1:+x 2:-y 3:+y 4:-z 5:+z): (voxel index, direction, face centre in
    voxel units (x, y, z))."""
    nz, ny, nx = labels.shape
    lab = labels.ravel()
    vox, dirs, cen = [], [], []
    steps = ((-1, 0, 0), (1, 0, 0), (0, -1, 0), (0, 1, 0), (0, 0, -1), (0, 0, 1))
    idx = np.nonzero(lab == ANODE)[0]
    k, r = np.divmod(idx, nx * ny)
    j, i = np.divmod(r, nx)
    for d, (dx, dy, dz) in enumerate(steps):
        ii, jj, kk = i + dx, j + dy, k + dz
        inside = (ii >= 0) & (ii < nx) & (jj >= 0) & (jj < ny) & (kk >= 0) & (kk < nz)
        nb = np.where(inside, ii + nx * (jj + ny * kk), 0)
        face = inside & (lab[nb] == PORE)
        vox.append(idx[face])
        dirs.append(np.full(int(face.sum()), d))
        cen.append(np.stack([i[face] + 0.5 + 0.5 * dx, j[face] + 0.5 + 0.5 * dy, k[face] + 0.5 + 0.5 * dz], axis=1))
    vox, dirs, cen = np.concatenate(vox), np.concatenate(dirs), np.concatenate(cen)
    order = np.lexsort((dirs, vox))
    return vox[order], dirs[order], cen[order]


def germ_grain_plating(labels: np.ndarray, z_sep_face: int, h: float, seed: int, lam_per_m2: float = 0.01e12,
                       r_s: float = 2.2e-6, molar_volume: float = 1.30e-5):
    """Initial plated Li by the germ-grain model of Sec. 2.3: germs are a
    Poisson process of intensity lam on the separator/graphite plane
    z = z_sep_face; each germ's line towards the graphite collector meets the
    structure at p* (the top face of the first graphite voxel below it); every
    graphite/pore face whose centre lies within r_s of p* is plated one voxel
    thick (h / molar_volume mol/m^2).  Returns (mask over the anode faces in
    canonical order, plated amount, germ positions in voxel units)."""
    nz, ny, nx = labels.shape
    rng = Stream(seed, 7777)
    area = nx * ny * h * h
    # Poisson count by inversion of uniforms (product of uniforms below exp(-mean))
    mean = lam_per_m2 * area
    count, prod, lim = 0, 1.0, math.exp(-mean)
    while True:
        prod *= float(rng.uniform(1)[0])
        if prod <= lim:
            break
        count += 1
    xy = rng.uniform(2 * count).reshape(count, 2) * np.array([nx, ny]) if count else np.zeros((0, 2))
    _, _, cen = anode_faces(labels)
    mask = np.zeros(cen.shape[0], dtype=bool)
    r_vox = r_s / h
    germs = []
    for gx, gy in xy:
        i, j = min(int(gx), nx - 1), min(int(gy), ny - 1)
        col = labels[:z_sep_face, j, i]
        hit = np.nonzero(col == ANODE)[0]
        if hit.size == 0:
            continue
        k = int(hit[-1])
        p = np.array([gx, gy, k + 1.0])
        germs.append(p)
        mask |= np.sum((cen - p) ** 2, axis=1) <= r_vox * r_vox
    return mask, h / molar_volume, np.array(germs).reshape(-1, 3)


def paper_half_cell(seed: int = 3, current_density: float = -250.0, scale: int = 1) -> Workload:
    """The paper's case study (Sec. 3.2): a 100 x 100 x 149 half cell at
    h = 0.44 um (44 x 44 x 65.6 um), graphite 100 / separator 40 / foil 9
    layers, spheres r in [4, 8] voxels, porosity 0.3, initial graphite
    stoichiometry 0.9 with germ-grain plated Li, delithiated at a constant
    current density in [2.5, 250] A/m^2 (negative: delithiation) for 60 s.
    The graphite's solid diffusivity is 1e-13 m^2/s (the paper does not
    print its material constants; with 1e-14 the particle surfaces near the
    separator empty before 60 s at 250 A/m^2).  `scale` divides the grid
    and radii for oracle-sized copies."""
    nx, nz = 100 // scale, 149 // scale
    layers = (100 // scale, 40 // scale, nz - 100 // scale - 40 // scale)
    lab = half_cell(nx, nx, nz, seed, 4.0 / scale, 8.0 / scale, 0.30, layers)
    p = CellParams(x0=0.9, Ds_an=1e-13)
    p.I_app = current_density * nx * nx * p.h * p.h
    w = Workload(f"half cell {nx}x{nx}x{nz}, {current_density:g} A/m^2 for 60 s", lab, p, 1.0, 60)
    w.meta["z_sep_face"] = layers[0]
    w.meta["current_density"] = current_density
    return w


# ---------------------------------------------------------------------------
# parameter sets (SI units).  The paper prints no material table; these are the
# synthetic defaults, shared as *inputs* by every solver.
# ---------------------------------------------------------------------------
FARADAY_FOR_CRATE = 96485.33212  # C/mol, used only to turn a C-rate into amperes


@dataclass
class CellParams:
    T: float = 298.15            # K
    I_app: float = 0.0           # A, > 0 charges the cell (anode lithiates)
    h: float = 0.44e-6           # voxel edge, m (44 um / 100 voxels)
    c0: float = 1000.0           # electrolyte salt concentration, mol/m^3
    x0: float = 0.05             # initial anode stoichiometry
    y0: float = 0.95             # initial cathode stoichiometry
    De: float = 2e-10            # electrolyte diffusivity, m^2/s
    kappa: float = 1.0           # electrolyte conductivity, S/m
    tplus: float = 0.38          # transference number
    thermo: float = 1.0          # thermodynamic factor 1 + dln f/dln c
    Ds_an: float = 1e-14
    Ds_ca: float = 1e-14
    sigma_an: float = 100.0
    sigma_ca: float = 10.0
    cmax_an: float = 31000.0
    cmax_ca: float = 31000.0
    i00_an: float = 1e-4         # A m / mol  (i = 2 i00 sqrt(cs ce) sinh(...))
    i00_ca: float = 1e-4
    i00_pl: float = 1e-2         # A m^-1/2 mol^-1/2
    i00_ce: float = 10.0         # A/m^2, Li-foil counter electrode of a half cell (i = 2 i00_ce sinh(...))
    n_c: float = 0.48e-9 / 1.30e-5   # mol/m^2: 0.48 nm of Li metal
    U_an: tuple = (0.12, 0.03)   # U = a0 + a1 ln((1-x)/x)   [V]
    U_ca: tuple = (3.95, 0.06)
    plating: int = 1

    def as_dict(self) -> dict:
        d = asdict(self)
        d["U_an"] = tuple(self.U_an)
        d["U_ca"] = tuple(self.U_ca)
        return d


def one_c_current(labels: np.ndarray, p: CellParams) -> float:
    """1C in amperes: the smaller electrode capacity (F c_max V_solid) per hour
    (a half cell's Li foil is a reservoir: the graphite capacity)."""
    v = p.h ** 3
    cap_an = FARADAY_FOR_CRATE * p.cmax_an * v * np.count_nonzero(labels == ANODE)
    if not np.any(labels == CATHODE):
        return float(cap_an / 3600.0)
    cap_ca = FARADAY_FOR_CRATE * p.cmax_ca * v * np.count_nonzero(labels == CATHODE)
    return float(min(cap_an, cap_ca) / 3600.0)


@dataclass
class Workload:
    name: str
    labels: np.ndarray
    params: CellParams
    dt: float
    steps: int
    precision: str = "fp64"      # "fp64" | "mixed"
    meta: dict = field(default_factory=dict)

    @property
    def shape(self):
        nz, ny, nx = self.labels.shape
        return nx, ny, nz


def config0(seed: int = 0) -> Workload:
    """12x12x40 full cell (16/8/16), spheres r in [2,3], porosity 0.35, 1C charge,
    20 steps of 10 s, plating on, FP64."""
    lab = sphere_cell(12, 12, 40, seed, 2.0, 3.0, 0.35, 0.35, layers=(16, 8, 16))
    p = CellParams()
    p.I_app = one_c_current(lab, p)
    return Workload("full cell 12x12x40, 1C charge, 20 x 10 s", lab, p, 10.0, 20)


def config1(seed: int = 1, scale: int = 1) -> Workload:
    """64x64x160 full cell (64/32/64), spheres r in [3,6], porosity U[0.30,0.40]
    per electrode, 2C charge, 200 steps of 5 s.  `scale` divides the grid (and
    the radii) for oracle-sized parity copies."""
    s = Stream(seed, 1000)
    pa, pc = s.uniform(2, 0.30, 0.40)
    nx, nz = 64 // scale, 160 // scale
    lab = sphere_cell(nx, nx, nz, seed, 3.0 / scale ** 0.5, 6.0 / scale ** 0.5, pa, pc)
    p = CellParams()
    p.I_app = 2.0 * one_c_current(lab, p)
    return Workload(f"full cell {nx}x{nx}x{nz}, 2C charge, 200 x 5 s", lab, p, 5.0, 200,
                    meta={"porosity": (float(pa), float(pc))})


def config2(seed: int = 2, scale: int = 1) -> Workload:
    """128x128x320 full cell, 3C fast charge at 268 K, 500 steps of 2 s to 4.2 V."""
    s = Stream(seed, 1000)
    pa, pc = s.uniform(2, 0.30, 0.40)
    nx, nz = 128 // scale, 320 // scale
    lab = sphere_cell(nx, nx, nz, seed, 3.0, 6.0, pa, pc)
    p = CellParams(T=268.0)
    p.I_app = 3.0 * one_c_current(lab, p)
    return Workload(f"full cell {nx}x{nx}x{nz}, 3C charge at 268 K, 2 s steps", lab, p, 2.0, 500,
                    precision="mixed", meta={"porosity": (float(pa), float(pc)), "cutoff_V": 4.2})


def sampled_query(seed: int, n_choices, dt: float = 5.0, steps: int = 12,
                  scale: int = 1) -> Workload:
    """One parameter query as in the batched and served workloads: grid
    Nx in n_choices (Ny = Nx, Nz = 2.5 Nx), C-rate U[0.5,4], T U[268,308] K,
    plating rate constant log-uniform over [1e-2, 1e2] x default."""
    s = Stream(seed, 2000)
    u = s.uniform(5)
    nx = int(n_choices[min(int(u[0] * len(n_choices)), len(n_choices) - 1)]) // scale
    nz = int(round(2.5 * nx))
    pa, pc = 0.30 + 0.10 * u[3], 0.30 + 0.10 * u[4]
    lab = sphere_cell(nx, nx, nz, seed, 3.0, 6.0, pa, pc)
    crate = 0.5 + 3.5 * u[1]
    p = CellParams(T=268.0 + 40.0 * u[2])
    p.i00_pl = CellParams().i00_pl * 10.0 ** (-2.0 + 4.0 * s.uniform(1)[0])
    p.I_app = crate * one_c_current(lab, p)
    return Workload(f"query {nx}x{nx}x{nz}, {crate:.2f}C at {p.T:.1f} K", lab, p, dt, steps,
                    precision="mixed", meta={"crate": crate})


def config3(n_cells: int = 32, base_seed: int = 1000, scale: int = 1) -> list[Workload]:
    """32 cells, grids 32x32x80 .. 96x96x240 (Nx step 8), distinct seeds."""
    return [sampled_query(base_seed + k, list(range(32, 97, 8)), scale=scale) for k in range(n_cells)]


def poisson_arrivals(rate_hz: float, n: int, seed: int = 2000) -> np.ndarray:
    """Arrival times (s) of a Poisson stream: exponential inter-arrival gaps."""
    u = Stream(seed, 3000).uniform(n)
    return np.cumsum(-np.log1p(-u) / rate_hz)


def config4_requests(n: int, base_seed: int = 2001, scale: int = 1) -> list[Workload]:
    """Served parameter queries, grids 48x48x120 .. 128x128x320 (Nx step 8)."""
    return [sampled_query(base_seed + k, list(range(48, 129, 8)), scale=scale) for k in range(n)]
