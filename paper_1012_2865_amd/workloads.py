"""Seeded synthetic workloads for the adaptive ray tracer.

Every input either side of the parity tests sees is built here: density and
neutral-fraction fields, point-source lists, spectra and trace parameters, for
the five workload classes the benchmark and the tests use. The module holds no
step of the ray-tracing method itself; the oracle and the GPU path both receive
the arrays it returns and nothing else.

Conventions shared by every consumer:

* A field is a float32 array of shape (nz, ny, nx) in C order, so the linear
  cell index is ``i + nx*(j + ny*k)`` (x fastest).
* Source positions are in cells of the root grid, measured from the root
  grid's lower corner. They are general float64 values drawn uniformly (no
  lattice): the library accepts any position inside the root grid, and the
  inputs exercise that.
* Energies are in eV, cross-sections in cm^2, photon rates in photons/s,
  lengths in cm.

The workload shapes follow the paper's test problems: a single source in a
uniform medium (Test 1 geometry, section 4.1), a 128^3 grid with 16 sources
(the shape of Test 4, section 4.4, whose cosmological density field is not
available, so a seeded lognormal field stands in for it), the four hydrogen
groups of the spectrum tests, and a two-level nested grid (section 3.1, the
AMR hierarchy the tracer walks).
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Sequence, Tuple

import numpy as np

PC_CM = 3.0856775814913673e18      # parsec in cm (IAU 2015 exact value)
KPC_CM = 1.0e3 * PC_CM
EV_ERG = 1.602176634e-12           # electron-volt in erg (SI exact value)
SIGMA_HI_13P6 = 6.3e-18            # HI photo-ionisation cross-section at threshold, cm^2
E_ION_HI_EV = 13.6                 # hydrogen ionisation energy, eV


@dataclass
class Grid:
    """One uniform grid patch (root or a 2x-refined child of the root)."""
    n_h: np.ndarray          # float32 (nz, ny, nx), hydrogen number density, cm^-3
    x_hi: np.ndarray         # float32 (nz, ny, nx), neutral fraction in [0, 1]
    dx_cm: float             # cell width, cm
    parent: int = -1         # -1 for the root grid, 0 for a child of the root
    offset: Tuple[int, int, int] = (0, 0, 0)   # lower corner in parent cells (x, y, z)

    @property
    def shape_xyz(self) -> Tuple[int, int, int]:
        nz, ny, nx = self.n_h.shape
        return nx, ny, nz

    @property
    def n_cells(self) -> int:
        return int(self.n_h.size)


@dataclass
class Spectrum:
    energy_ev: np.ndarray            # float64 (G,)
    sigma_cm2: np.ndarray            # float64 (G,)
    frac: np.ndarray                 # float64 (G,), photon-number fraction per group
    e_ion_ev: float = E_ION_HI_EV

    @property
    def n_groups(self) -> int:
        return int(len(self.energy_ev))


@dataclass
class Params:
    phi_c: float = 5.1          # minimum rays per cell face before a split
    level_init: int = 1         # HEALPix level of the seed rays
    level_max: int = 14         # rays at this level never split
    p_min_frac: float = 1e-8    # a ray ends when P < p_min_frac * P0
    covering: bool = False      # scale k_ph and heating by the covering factor (section 2.3)
    tau_thin: float = 0.0       # > 0: optically-thin approximation below this optical depth (section 2.4)


@dataclass
class Problem:
    grids: List[Grid]
    sources: np.ndarray              # float64 (S, 4): x, y, z (root cells), ndot (ph/s)
    spectrum: Spectrum
    params: Params = field(default_factory=Params)
    name: str = ""

    @property
    def n_sources(self) -> int:
        return int(self.sources.shape[0])

    @property
    def n_cells(self) -> int:
        return sum(g.n_cells for g in self.grids)


def rng_for(cfg: int, item: int, stream: int) -> np.random.Generator:
    """Independent, reproducible stream for (workload class, item, purpose)."""
    return np.random.default_rng(np.random.SeedSequence([cfg, item, stream]))


def _below(hi) -> np.ndarray:
    """The largest float64 below each upper bound (positions stay inside a
    half-open interval)."""
    return np.nextafter(np.asarray(hi, dtype=np.float64), -np.inf)


def hydrogen_spectrum(energies_ev: Sequence[float], frac: Sequence[float] | None = None) -> Spectrum:
    """Monochromatic hydrogen-ionising groups with sigma(E) = 6.3e-18 (E/13.6)^-3.

    Photon-number fractions default to equal shares.
    """
    e = np.asarray(energies_ev, dtype=np.float64)
    sig = SIGMA_HI_13P6 * (e / E_ION_HI_EV) ** -3
    if frac is None:
        f = np.full(len(e), 1.0 / len(e))
    else:
        f = np.asarray(frac, dtype=np.float64)
    return Spectrum(energy_ev=e, sigma_cm2=sig, frac=f)


FOUR_GROUPS_EV = (13.6, 20.0, 30.0, 60.0)


def uniform_grid(n: int | Tuple[int, int, int], dx_cm: float, n_h: float, x_hi: float) -> Grid:
    nx, ny, nz = (n, n, n) if np.isscalar(n) else n
    return Grid(n_h=np.full((nz, ny, nx), n_h, dtype=np.float32),
                x_hi=np.full((nz, ny, nx), x_hi, dtype=np.float32), dx_cm=float(dx_cm))


def lognormal_density(n: int, sigma_ln: float, mean: float, rng: np.random.Generator) -> np.ndarray:
    """Lognormal density on an n^3 grid from a Gaussian random field with P(k) ~ k^-2.

    White Gaussian noise is filtered by |k|^-1 in Fourier space (k = 0 mode
    removed), normalised to unit variance g, and mapped to
    mean * exp(sigma_ln g) / <exp(sigma_ln g)>, so the sample mean is `mean`
    before the final rounding to float32.
    """
    white = rng.standard_normal((n, n, n))
    fk = np.fft.rfftn(white)
    k1 = np.fft.fftfreq(n)
    kr = np.fft.rfftfreq(n)
    kk = np.sqrt(k1[:, None, None] ** 2 + k1[None, :, None] ** 2 + kr[None, None, :] ** 2)
    filt = np.zeros_like(kk)
    nz = kk > 0
    filt[nz] = 1.0 / kk[nz]
    g = np.fft.irfftn(fk * filt, s=(n, n, n), axes=(0, 1, 2))
    g = (g - g.mean()) / g.std()
    f = np.exp(sigma_ln * g)
    return (mean * f / f.mean()).astype(np.float32)


def random_sources(rng: np.random.Generator, n_src: int, box: Tuple[float, float, float],
                   log_ndot: Tuple[float, float], lo: Tuple[float, float, float] = (0.0, 0.0, 0.0)) -> np.ndarray:
    """Uniform positions inside [lo, lo+box) (root cells), log-uniform photon rates."""
    pos = np.empty((n_src, 3))
    for a in range(3):
        pos[:, a] = lo[a] + rng.uniform(0.0, box[a], n_src)
    for a in range(3):
        pos[:, a] = np.clip(pos[:, a], lo[a], _below(lo[a] + box[a]))
    ndot = 10.0 ** rng.uniform(log_ndot[0], log_ndot[1], n_src)
    return np.column_stack([pos, ndot])


# ---------------------------------------------------------------------------
# The five workload classes
# ---------------------------------------------------------------------------

DX_C1 = 2.0 * KPC_CM / 128.0       # 15.625 pc


def config0(level_init: int = 1) -> Problem:
    """32^3 uniform grid, 8 kpc box, n_H = 2e-3, x_HI = 1; one 1e49 ph/s 13.6 eV
    source at the box centre (a cell vertex); 48 seed rays, Phi_c = 5.1."""
    g = uniform_grid(32, 8.0 * KPC_CM / 32.0, 2e-3, 1.0)
    src = np.array([[16.0, 16.0, 16.0, 1e49]])
    return Problem([g], src, hydrogen_spectrum([13.6]),
                   Params(phi_c=5.1, level_init=level_init, level_max=14, p_min_frac=1e-8), name="uniform32")


def lognormal_problem(cfg: int, item: int, n: int, n_src: int, log_ndot=(48.0, 50.0),
                      dx_cm: float = DX_C1, energies=FOUR_GROUPS_EV, sigma_ln: float = 1.0,
                      mean: float = 1e-2, params: Params | None = None) -> Problem:
    """Lognormal n_H (sigma_ln, mean), x_HI ~ U(0.5, 1), uniformly placed sources."""
    n_h = lognormal_density(n, sigma_ln, mean, rng_for(cfg, item, 0))
    x_hi = rng_for(cfg, item, 1).uniform(0.5, 1.0, (n, n, n)).astype(np.float32)
    src = random_sources(rng_for(cfg, item, 2), n_src, (n, n, n), log_ndot)
    return Problem([Grid(n_h, x_hi, dx_cm)], src, hydrogen_spectrum(energies),
                   params or Params(), name=f"lognormal{n}_s{n_src}")


def config1() -> Problem:
    """128^3 lognormal grid (2 kpc box), 16 sources, 4 groups (13.6/20/30/60 eV)."""
    return lognormal_problem(1, 0, 128, 16)


def config1_ionised(tau_thin: float = 0.0) -> Problem:
    """config1 with every neutral fraction scaled by 1e-3: ionised gas around
    the sources, optically thin for tens of cells (the regime the optically-thin
    approximation of section 2.4 is for); tau_thin as given."""
    p = config1()
    g = p.grids[0]
    p.grids[0] = Grid(g.n_h, (g.x_hi * np.float32(1e-3)).astype(np.float32), g.dx_cm)
    p.params = Params(**{**p.params.__dict__, "tau_thin": tau_thin})
    p.name = "ionised_lognormal128_16src_4grp"
    return p


def thin_box(n: int = 128, tau_thin: float = 0.0) -> Problem:
    """The optically thin medium of the angular-resolution test (section 7.2):
    a 6.6 kpc box of n^3 cells, n_H = 1e-3, x_HI = 1e-4, one 5e48 ph/s 13.6 eV
    source at the corner (as in Test 1), phi_c = 5.1; tau_thin as given."""
    g = uniform_grid(n, 6.6 * KPC_CM / n, 1e-3, 1e-4)
    return Problem([g], np.array([[0.0, 0.0, 0.0, 5e48]]), hydrogen_spectrum([13.6]),
                   Params(phi_c=5.1, level_init=1, tau_thin=tau_thin), name=f"thin_box{n}_corner_source")


def angular_box(n: int, phi_c: float, covering: bool = True) -> Problem:
    """The angular-resolution test (section 7.2): Test 1's 6.6 kpc box of n^3
    cells in optically thin gas (n_H = 1e-3, x_HI = 1e-4) with its 5e48 ph/s
    13.6 eV source on the box's corner, traced once at the given phi_c, with
    the covering-factor correction (section 2.3) on unless asked otherwise."""
    g = uniform_grid(n, 6.6 * KPC_CM / n, 1e-3, 1e-4)
    return Problem([g], np.array([[0.0, 0.0, 0.0, 5e48]]), hydrogen_spectrum([13.6]),
                   Params(phi_c=phi_c, level_init=1, level_max=14, p_min_frac=1e-8, covering=covering),
                   name=f"angular_box{n}_phi{phi_c}")


C2_EDGES = (32, 48, 64, 96)


def config2(n_problems: int = 64) -> List[Problem]:
    """Independent lognormal grids with edges from {32,48,64,96} and 1-8 sources."""
    rng = rng_for(2, 10_000, 0)
    edges = rng.choice(C2_EDGES, n_problems)
    nsrc = rng.integers(1, 9, n_problems)
    return [lognormal_problem(2, i, int(edges[i]), int(nsrc[i])) for i in range(n_problems)]


C3_EDGES = (32, 64, 128, 256)


@dataclass
class Request:
    arrival_s: float
    problem: Problem


def config3(rate_hz: float, n_requests: int = 2000, horizon_s: float = 60.0, seed_item: int = 0,
            edges: Sequence[int] = C3_EDGES) -> List[Request]:
    """Poisson request stream: edge in `edges`, 1-32 sources, Ndot log-U[1e47, 1e51]."""
    rng = rng_for(3, seed_item, int(rate_hz))
    out: List[Request] = []
    t = 0.0
    for i in range(n_requests):
        t += rng.exponential(1.0 / rate_hz)
        if t > horizon_s:
            break
        n = int(rng.choice(edges))
        s = int(rng.integers(1, 33))
        out.append(Request(t, lognormal_problem(3, seed_item * 100_000 + i, n, s, log_ndot=(47.0, 51.0))))
    return out


@dataclass
class PooledRequest:
    """A serving request whose fields come from a shared pool (one of
    `pool[edge]`), with its own sources."""
    arrival_s: float
    edge: int
    pool_index: int
    sources: np.ndarray              # float64 (S, 4)


def config3_pool(rate_hz: float, n_requests: int = 2000, horizon_s: float = 60.0, pool_per_edge: int = 2,
                 seed_item: int = 0, edges: Sequence[int] = C3_EDGES):
    """The serving stream with device-resident fields: `pool_per_edge`
    lognormal field sets per grid edge (as config 1 otherwise), and Poisson
    arrivals each naming an edge, a pool entry, 1-32 sources and Ndot
    log-U[1e47, 1e51]. Returns (pool, requests): pool maps an edge to a list
    of Grid, requests is a list of PooledRequest."""
    pool = {}
    for e in edges:
        pool[int(e)] = [Grid(lognormal_density(int(e), 1.0, 1e-2, rng_for(3, 900_000 + 10 * int(e) + k, 0)),
                             rng_for(3, 900_000 + 10 * int(e) + k, 1).uniform(0.5, 1.0, (int(e),) * 3).astype(np.float32),
                             DX_C1)
                        for k in range(pool_per_edge)]
    rng = rng_for(3, seed_item, int(rate_hz * 1000))
    out: List[PooledRequest] = []
    t = 0.0
    for i in range(n_requests):
        t += rng.exponential(1.0 / rate_hz)
        if t > horizon_s:
            break
        e = int(rng.choice(edges))
        k = int(rng.integers(0, pool_per_edge))
        s = int(rng.integers(1, 33))
        out.append(PooledRequest(t, e, k, random_sources(rng, s, (e, e, e), (47.0, 51.0))))
    return pool, out


def pooled_problem(pool, req: PooledRequest, energies=FOUR_GROUPS_EV) -> Problem:
    return Problem([pool[req.edge][req.pool_index]], req.sources, hydrogen_spectrum(energies), Params(),
                   name=f"serve{req.edge}_s{len(req.sources)}")


def config4(n_clusters: int = 10, per_cluster: int = 100, root_n: int = 256, sub_root_cells: int = 64,
            sigma_root_cells: float = 8.0) -> Problem:
    """Two-level nested grid: root_n^3 root plus a 2x-refined child of
    (2*sub_root_cells)^3 fine cells centred on a Gaussian overdensity
    (peak 100x the mean n_H = 1e-2); sources in Gaussian clusters inside the child."""
    c = root_n / 2.0
    lo = int(root_n // 2 - sub_root_cells // 2)

    def density(xc, yc, zc):
        r2 = (xc - c) ** 2 + (yc - c) ** 2 + (zc - c) ** 2
        return (1e-2 * (1.0 + 99.0 * np.exp(-r2 / (2.0 * sigma_root_cells ** 2)))).astype(np.float32)

    ax = np.arange(root_n) + 0.5
    root_nh = density(ax[None, None, :], ax[None, :, None], ax[:, None, None])
    nf = 2 * sub_root_cells
    fx = lo + (np.arange(nf) + 0.5) / 2.0
    sub_nh = density(fx[None, None, :], fx[None, :, None], fx[:, None, None])
    root_x = rng_for(4, 0, 1).uniform(0.5, 1.0, root_nh.shape).astype(np.float32)
    sub_x = rng_for(4, 1, 1).uniform(0.5, 1.0, sub_nh.shape).astype(np.float32)
    root = Grid(root_nh, root_x, DX_C1)
    sub = Grid(sub_nh, sub_x, DX_C1 / 2.0, parent=0, offset=(lo, lo, lo))
    rng = rng_for(4, 2, 2)
    inner_lo = lo + sub_root_cells / 4.0
    centres = inner_lo + rng.uniform(0.0, sub_root_cells / 2.0, (n_clusters, 3))
    pos = np.repeat(centres, per_cluster, axis=0) + rng.normal(0.0, 2.0, (n_clusters * per_cluster, 3))
    pos = np.clip(pos, lo, _below(lo + sub_root_cells))
    ndot = 10.0 ** rng.uniform(48.0, 50.0, n_clusters * per_cluster)
    return Problem([root, sub], np.column_stack([pos, ndot]), hydrogen_spectrum(FOUR_GROUPS_EV),
                   Params(level_max=14), name="nested256+128")


def subset_sources(p: Problem, idx) -> Problem:
    """Same grids and spectrum, a subset of the sources (for linearity checks)."""
    return Problem(p.grids, p.sources[np.asarray(idx)], p.spectrum, p.params, name=p.name + "_subset")
