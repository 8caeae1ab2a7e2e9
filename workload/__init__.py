"""Seeded synthetic workloads for the scan-resolved Ti-6Al-4V phase update.

This module only *describes inputs*: grids of material points, laser scan
paths (as tables of straight tracks), layer schedules, active-point masks and
seeded sample indices.  It contains none of the method's arithmetic (no
temperature model, no phase kinetics); the CPU oracle and the HIP library each
evaluate the method on these inputs independently.

Scan table layout (one row per straight laser track, float64, sorted by t_on):

    x0, y0, z0   start point of the track [m]; z0 is the surface height of
                 the layer being scanned (the body lies at z <= z0)
    ux, uy       unit direction of motion in the xy-plane
    t_on         switch-on time [s]
    dur          duration the source stays on [s]
    q            absorbed power [W]
    v            scan speed [m/s]

Grid convention: point (i, j, k) sits at (ox + i*h, oy + j*h, oz - k*h); the
linear index is i + nx*(j + ny*k), so x varies fastest and k counts downward
from the top surface.  A point is *active* during a layer when its z is at or
below that layer's surface (z <= z_top + 1e-3*h); inactive points are left
untouched.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Tuple

import numpy as np

TRACK_COLS = ("x0", "y0", "z0", "ux", "uy", "t_on", "dur", "q", "v")
N_TRACK_COLS = len(TRACK_COLS)

# Initial phase state used by every workload: alpha_s = 0.9, beta = 0.1,
# alpha_m = 0.
INIT_ALPHA_S = 0.9
INIT_ALPHA_M = 0.0
INIT_BETA = 0.1

MASK64 = (1 << 64) - 1


def splitmix64(x):
    """SplitMix64 finaliser (Steele, Lea, Flood 2014), vectorised over uint64."""
    z = np.asarray(x, dtype=np.uint64).copy()
    with np.errstate(over="ignore"):
        z = z + np.uint64(0x9E3779B97F4A7C15)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        z = z ^ (z >> np.uint64(31))
    return z


def sample_indices(n: int, p: float, seed: int, chunk: int = 1 << 24) -> np.ndarray:
    """Indices i in [0, n) with splitmix64(i ^ seed) < p * 2**64 (order-free)."""
    thr = np.uint64(min(int(p * 2.0 ** 64), MASK64))
    out = []
    s = np.uint64(seed & MASK64)
    for b in range(0, n, chunk):
        i = np.arange(b, min(n, b + chunk), dtype=np.uint64)
        out.append(np.nonzero(splitmix64(i ^ s) < thr)[0].astype(np.int64) + b)
    return np.concatenate(out) if out else np.zeros(0, np.int64)


@dataclasses.dataclass
class Grid:
    nx: int
    ny: int
    nz: int
    h: float
    ox: float = 0.0
    oy: float = 0.0
    oz: float = 0.0
    index: Optional[np.ndarray] = None  # int32 distinct box linear indices, or None = full box

    @property
    def n_box(self) -> int:
        return self.nx * self.ny * self.nz

    @property
    def n(self) -> int:
        return self.n_box if self.index is None else int(self.index.size)

    def box_index(self, local: np.ndarray) -> np.ndarray:
        """Map local point numbers (0..n-1) to box linear indices."""
        local = np.asarray(local, dtype=np.int64)
        return local if self.index is None else self.index[local].astype(np.int64)

    def coords(self, local: np.ndarray) -> np.ndarray:
        """(m, 3) float64 coordinates of the given local point numbers."""
        lin = self.box_index(local)
        i = lin % self.nx
        j = (lin // self.nx) % self.ny
        k = lin // (self.nx * self.ny)
        return np.stack([self.ox + i * self.h, self.oy + j * self.h, self.oz - k * self.h], axis=1)

    def first_active_k(self, z_top: float) -> int:
        """Smallest k whose plane satisfies oz - k*h <= z_top + 1e-3*h (nz if none)."""
        for k in range(self.nz):
            if self.oz - k * self.h <= z_top + 1e-3 * self.h:
                return k
        return self.nz


@dataclasses.dataclass
class Layer:
    step_begin: int
    step_end: int
    z_top: float


@dataclasses.dataclass
class Scan:
    tracks: np.ndarray          # (n_tracks, 9) float64
    conductivity: float         # k [W/(m K)]
    diffusivity: float          # alpha [m^2/s]
    T0: float                   # initial / far-field temperature [K]
    T_clamp: float              # temperature clamp [K]
    window: int                 # number of most recent tracks superposed


@dataclasses.dataclass
class Workload:
    name: str
    grid: Grid
    scan: Scan
    layers: List[Layer]
    dt: float
    seed: int

    @property
    def n_steps(self) -> int:
        return self.layers[-1].step_end if self.layers else 0

    def t0(self, layer: Layer) -> float:
        # simulated time of the first step of a layer (same expression on both sides)
        return float(layer.step_begin) * self.dt

    def point_updates(self) -> int:
        tot = 0
        for L in self.layers:
            tot += self.active_count(L.z_top) * (L.step_end - L.step_begin)
        return tot

    def active_count(self, z_top: float) -> int:
        g = self.grid
        k0 = g.first_active_k(z_top)
        if g.index is None:
            return (g.nz - k0) * g.nx * g.ny
        return int(np.count_nonzero(g.index >= k0 * g.nx * g.ny))



def initial_state(n: int, dtype=np.float64):
    """(beta, alpha_s, alpha_m) arrays of the common initial state."""
    return (np.full(n, INIT_BETA, dtype), np.full(n, INIT_ALPHA_S, dtype),
            np.full(n, INIT_ALPHA_M, dtype))


# ----------------------------------------------------------------------------
# scan-path builders
# ----------------------------------------------------------------------------

def _track(x0, y0, z0, ux, uy, t_on, dur, q, v):
    return [x0, y0, z0, ux, uy, t_on, dur, q, v]


def serpentine_layer(t_begin, t_end, z0, lines, q, v):
    """Tracks for a layer that runs consecutively along `lines` (list of
    (xs, ys, xe, ye)) from t_begin, cut at t_end."""
    rows = []
    t = t_begin
    for (xs, ys, xe, ye) in lines:
        if t >= t_end:
            break
        L = math.hypot(xe - xs, ye - ys)
        if L <= 0.0:
            continue
        dur = min(L / v, t_end - t)
        rows.append(_track(xs, ys, z0, (xe - xs) / L, (ye - ys) / L, t, dur, q, v))
        t += L / v
    return rows


def hatch_lines_x(x_lo, x_hi, y_first, hatch, n_lines, first):
    """Bidirectional lines along x at y = y_first + j*hatch, starting at line
    `first`; even lines run +x, odd lines -x."""
    out = []
    for j in range(first, n_lines):
        y = y_first + j * hatch
        out.append((x_lo, y, x_hi, y) if j % 2 == 0 else (x_hi, y, x_lo, y))
    return out


def island_lines(x_lo, y_lo, size, hatch, theta):
    """Serpentine hatch lines at angle theta clipped to the square island
    [x_lo, x_lo+size] x [y_lo, y_lo+size]."""
    c, s = math.cos(theta), math.sin(theta)
    cx, cy = x_lo + 0.5 * size, y_lo + 0.5 * size
    half = 0.5 * size * math.sqrt(2.0)
    n = int(math.floor(2 * half / hatch))
    out = []
    for j in range(n + 1):
        off = -half + (j + 0.5) * hatch
        # line: p(u) = centre + off * n_hat + u * d_hat, n_hat = (-s, c), d_hat = (c, s)
        px, py = cx - off * s, cy + off * c
        u_lo, u_hi = -1e9, 1e9
        ok = True
        for (p, d, lo, hi) in ((px, c, x_lo, x_lo + size), (py, s, y_lo, y_lo + size)):
            if abs(d) < 1e-12:
                if p < lo or p > hi:
                    ok = False
                continue
            a, b = (lo - p) / d, (hi - p) / d
            u_lo, u_hi = max(u_lo, min(a, b)), min(u_hi, max(a, b))
        if not ok or u_hi - u_lo <= 1e-9:
            continue
        a = (px + u_lo * c, py + u_lo * s)
        b = (px + u_hi * c, py + u_hi * s)
        out.append((a[0], a[1], b[0], b[1]) if len(out) % 2 == 0 else (b[0], b[1], a[0], a[1]))
    return out


# ----------------------------------------------------------------------------
# the configurations
# ----------------------------------------------------------------------------

K_W = 7.0            # conductivity [W/(m K)]
ALPHA = 3e-6         # diffusivity [m^2/s]
T0 = 300.0           # preheat / far field [K]
T_CLAMP = 1928.0     # clamp at liquidus [K]
Q_ABS = 0.35 * 200.0  # absorbed power [W]
V_SCAN = 1.0         # [m/s]


def single_track(nx=64, ny=32, nz=16, n_steps=2000, dt=1e-6, seed=1001) -> Workload:
    """64x32x16 grid at 10 um, one 0.6 mm line at 1 m/s (y = 155 um, between
    rows), 2000 steps of 1 us; the source switches off after 600 us."""
    h = 10e-6
    grid = Grid(nx, ny, nz, h)
    tracks = np.array([_track(20e-6, 155e-6, 0.0, 1.0, 0.0, 0.0, 600e-6, Q_ABS, V_SCAN)])
    scan = Scan(tracks, K_W, ALPHA, T0, T_CLAMP, window=1)
    return Workload("single_track", grid, scan, [Layer(0, n_steps, 0.0)], dt, seed)


def multilayer_block(nx=256, ny=256, nz=128, n_layers=10, layer_thick=30e-6,
                     steps_per_layer=2000, dt=2e-6, hatch=100e-6, seed=1002,
                     window=2) -> Workload:
    """256x256x128 block at 10 um; n_layers layers of 30 um, each scanned for
    steps_per_layer steps with bidirectional x-lines at 100 um hatch starting
    from a seeded line; superposition of the last `window` tracks."""
    h = 10e-6
    grid = Grid(nx, ny, nz, h)
    rng = np.random.default_rng(seed)
    width = nx * h
    n_lines = int(round(ny * h / hatch))
    rows, layers = [], []
    for ell in range(n_layers):
        z_top = -(n_layers - 1 - ell) * layer_thick
        first = int(rng.integers(0, max(1, n_lines - 1)))
        sb, se = ell * steps_per_layer, (ell + 1) * steps_per_layer
        lines = hatch_lines_x(0.0, width, 0.5 * hatch, hatch, n_lines, first)
        rows += serpentine_layer(sb * dt, se * dt, z_top, lines, Q_ABS, V_SCAN)
        layers.append(Layer(sb, se, z_top))
    scan = Scan(np.array(rows, dtype=np.float64), K_W, ALPHA, T0, T_CLAMP, window)
    return Workload("multilayer_block", grid, scan, layers, dt, seed)


@dataclasses.dataclass
class Phase:
    """n_steps steps of dt from simulated time t0 with one scheme
    ("explicit" or "implicit"); points above z_top are inactive."""
    t0: float
    dt: float
    n_steps: int
    z_top: float
    scheme: str


@dataclasses.dataclass
class PhasedWorkload:
    name: str
    grid: Grid
    scan: Scan
    phases: List[Phase]
    seed: int

    def point_updates(self) -> int:
        g = self.grid
        return sum((g.nz - g.first_active_k(p.z_top)) * g.nx * g.ny * p.n_steps for p in self.phases)


def cooldown_schedule(t_start, duration, dt_first, n_first=2000, double_every=10, dt_max=0.1):
    """Time steps of a cool-down phase as in the paper's cube example
    (Sec. 4.2): n_first steps of dt_first, then the step doubled after every
    `double_every` steps up to dt_max, until t_start + duration (the last step
    shortened to end there).  Returns [(t0, dt, n_steps)] segments."""
    segs = []
    t, t_end = t_start, t_start + duration
    dt, n = dt_first, n_first
    while t_end - t > 1e-12:
        fit = int(math.floor((t_end - t) / dt * (1.0 + 1e-12)))
        k = min(n, fit)
        if k > 0:
            segs.append((t, dt, k))
            t = t + k * dt
        if k < n:
            if t_end - t > 1e-12:
                segs.append((t, t_end - t, 1))
            break
        dt, n = min(2.0 * dt, dt_max), double_every
    return segs


def multilayer_cooldown(nx=256, ny=256, nz=128, n_layers=10, layer_thick=30e-6, steps_per_layer=2000,
                        dt=2e-6, hatch=100e-6, cooldown=1.0, final_cooldown=100.0, seed=1002,
                        window=2) -> PhasedWorkload:
    """The multi-layer block with the paper's inter-layer cool-down: each layer
    is scanned for steps_per_layer steps of dt (explicit scheme), then cools
    for `cooldown` seconds on the schedule of cooldown_schedule (implicit
    scheme, substeps of at most 0.01 s).  After the last layer's cool-down
    the part cools for `final_cooldown` more seconds in steps of 0.1 s, as
    the paper's examples end (Sec. 4.2).  Same seeded scan lines as
    multilayer_block, each layer starting after the previous cool-down."""
    h = 10e-6
    grid = Grid(nx, ny, nz, h)
    rng = np.random.default_rng(seed)
    width = nx * h
    n_lines = int(round(ny * h / hatch))
    active = steps_per_layer * dt
    rows, phases = [], []
    for ell in range(n_layers):
        z_top = -(n_layers - 1 - ell) * layer_thick
        first = int(rng.integers(0, max(1, n_lines - 1)))
        t_layer = ell * (active + cooldown)
        lines = hatch_lines_x(0.0, width, 0.5 * hatch, hatch, n_lines, first)
        rows += serpentine_layer(t_layer, t_layer + active, z_top, lines, Q_ABS, V_SCAN)
        phases.append(Phase(t_layer, dt, steps_per_layer, z_top, "explicit"))
        for (t0, d, k) in cooldown_schedule(t_layer + steps_per_layer * dt, cooldown, dt):
            phases.append(Phase(t0, d, k, z_top, "implicit"))
    if final_cooldown > 0:
        for (t0, d, k) in cooldown_schedule(n_layers * (active + cooldown), final_cooldown, 0.1, n_first=1 << 40):
            phases.append(Phase(t0, d, k, phases[-1].z_top, "implicit"))
    scan = Scan(np.array(rows, dtype=np.float64), K_W, ALPHA, T0, T_CLAMP, window)
    return PhasedWorkload("multilayer_cooldown", grid, scan, phases, seed)


def island_scan(nx, ny, nz, n_layers, layer_thick, steps_per_layer, dt, seed,
                island=5e-3, hatch=100e-6, window=2, index=None, name="island_scan"):
    """Island scan: square islands of `island` size tiled over the box top,
    serpentine inside each, per-layer seeded rotation in [0, pi) and seeded
    island order."""
    h = 10e-6
    grid = Grid(nx, ny, nz, h, index=index)
    rng = np.random.default_rng(seed)
    W, H = nx * h, ny * h
    nix, niy = int(math.ceil(W / island)), int(math.ceil(H / island))
    rows, layers = [], []
    for ell in range(n_layers):
        z_top = -(n_layers - 1 - ell) * layer_thick
        theta = float(rng.uniform(0.0, math.pi))
        order = rng.permutation(nix * niy)
        lines = []
        for o in order:
            ix, iy = int(o) % nix, int(o) // nix
            lines += island_lines(ix * island, iy * island, island, hatch, theta)
        sb, se = ell * steps_per_layer, (ell + 1) * steps_per_layer
        rows += serpentine_layer(sb * dt, se * dt, z_top, lines, Q_ABS, V_SCAN)
        layers.append(Layer(sb, se, z_top))
    scan = Scan(np.array(rows, dtype=np.float64), K_W, ALPHA, T0, T_CLAMP, window)
    return Workload(name, grid, scan, layers, dt, seed)


def cantilever_mask(nx, ny, nz, seed, top=32, base=24, leg_frac=0.08):
    """Sorted int32 box indices of a seeded cantilever-like body: a top slab of
    `top` planes, a base of `base` planes, and seeded rectangular legs joining
    them covering about `leg_frac` of the xy-area."""
    rng = np.random.default_rng(seed)
    legs = np.zeros((ny, nx), dtype=bool)
    target = leg_frac * nx * ny
    while legs.sum() < target:
        w, d = int(rng.integers(nx // 32, nx // 8)), int(rng.integers(ny // 32, ny // 8))
        x, y = int(rng.integers(0, nx - w)), int(rng.integers(0, ny - d))
        legs[y:y + d, x:x + w] = True
    plane = nx * ny
    leg_idx = np.nonzero(legs.ravel())[0].astype(np.int64)
    parts = []
    for k in range(nz):
        if k < top or k >= nz - base:
            parts.append(np.arange(k * plane, (k + 1) * plane, dtype=np.int64))
        else:
            parts.append(leg_idx + k * plane)
    idx = np.concatenate(parts)
    assert idx.max() < 2 ** 31
    return idx.astype(np.int32)


def tile_order(index: np.ndarray, nx: int, ny: int, a: int = 8) -> np.ndarray:
    """The same box indices, each plane's points through its a x a tiles row
    by row (within a tile row by row): 64 consecutive entries of a full
    plane are then one 8 x 8 patch instead of part of a row."""
    lin = index.astype(np.int64)
    plane = nx * ny
    k, r = lin // plane, lin % plane
    j, i = r // nx, r % nx
    tx, ty = (nx + a - 1) // a, (ny + a - 1) // a
    key = ((k * ty + j // a) * tx + i // a) * (a * a) + (j % a) * a + i % a
    return index[np.argsort(key, kind="stable")]


def cantilever_islands(nx=1024, ny=512, nz=128, n_layers=10, steps_per_layer=5000,
                       dt=2e-6, seed=1003, order="tiles") -> Workload:
    """Masked cantilever-like body (about 32M points) with 5x5 mm island scan;
    the point list in 8 x 8 tile order per plane (order="tiles") or sorted
    ("sorted")."""
    idx = cantilever_mask(nx, ny, nz, seed)
    if order == "tiles":
        idx = tile_order(idx, nx, ny)
    return island_scan(nx, ny, nz, n_layers, 30e-6, steps_per_layer, dt, seed,
                       index=idx, name="cantilever_islands")


def island_block(nx=512, ny=512, nz=256, n_layers=100, steps_per_layer=2000,
                 dt=2e-6, seed=1005) -> Workload:
    """512x512x256 box, 100 layers of 20 um, 5x5 mm island scan."""
    return island_scan(nx, ny, nz, n_layers, 20e-6, steps_per_layer, dt, seed,
                       name="island_block")


def truncated(wl: Workload, n_layers: int = None, steps_per_layer: int = None) -> Workload:
    """Same grid and scan, keeping the first layers and/or fewer steps each
    (layer start times unchanged, so the scan is the same)."""
    layers = wl.layers[: (n_layers or len(wl.layers))]
    if steps_per_layer is not None:
        layers = [Layer(L.step_begin, min(L.step_end, L.step_begin + steps_per_layer), L.z_top)
                  for L in layers]
    return dataclasses.replace(wl, layers=layers)


def mlp_init_params(seed=0) -> np.ndarray:
    """Seeded He-style random parameters of the 6-64-64-3 network (float32),
    layout W1[64][6], b1[64], W2[64][64], b2[64], W3[3][64], b3[3]."""
    rng = np.random.default_rng(seed)
    parts = [rng.normal(0, math.sqrt(2 / 7), 64 * 6), np.zeros(64), rng.normal(0, math.sqrt(2 / 64), 64 * 64),
             np.zeros(64), rng.normal(0, math.sqrt(1 / 64), 3 * 64), np.zeros(3)]
    return np.concatenate(parts).astype(np.float32)
