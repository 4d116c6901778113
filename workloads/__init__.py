"""Seeded synthetic inputs for the capacitance -> B_z path.

This module holds input generation only: loop polygons, field-point grids,
capacitance batches, frequency lists and target fields.  It contains none of
the method's arithmetic (no Biot-Savart, no inductance, no circuit solve), so
both the FP64 oracle and the HIP library can consume what it produces.

The structures stand in for the paper's three resonant structures (Sec. III-B):
a single copper loop, an 8x1 line and an 8x8 array of coupled unit cells.  The
paper's full-wave exports are not available, so the geometry is synthetic with
the shapes and sizes of the five workload configurations listed in the design doc.

Conventions
-----------
* Units are SI: metres, farads, ohms, hertz, tesla.
* A loop is a closed polygon given by its vertices in counter-clockwise order
  seen from +z; segment s of loop k joins vertex s to vertex s+1 (the last
  vertex joins back to the first).  ``seg_off`` is the CSR offset array: loop k
  owns vertices ``verts[seg_off[k]:seg_off[k+1]]``.
* Loop k of an nx-by-ny array is ``k = iy*nx + ix`` and is centred at
  ``((ix-(nx-1)/2)*pitch, (iy-(ny-1)/2)*pitch, 0)``.
* Field points are ordered plane, then y, then x; each plane is an inclusive
  ``linspace(-L/2, L/2, N)`` grid in x and y.
"""
from __future__ import annotations

import dataclasses
from typing import List, Optional, Sequence

import numpy as np

SEED_BASE = 18479


def rng_for(config_id: int, stream: int = 0) -> np.random.Generator:
    """Seeded generator for configuration ``config_id`` (1..5)."""
    return np.random.default_rng([SEED_BASE, int(config_id), int(stream)])


# --------------------------------------------------------------------------
# geometry
# --------------------------------------------------------------------------

def regular_polygon(radius: float, n_seg: int, center=(0.0, 0.0, 0.0)) -> np.ndarray:
    """Vertices of a regular n_seg-gon inscribed in a circle, vertex 0 at angle 0, CCW."""
    ang = 2.0 * np.pi * np.arange(n_seg) / n_seg
    v = np.zeros((n_seg, 3))
    v[:, 0] = center[0] + radius * np.cos(ang)
    v[:, 1] = center[1] + radius * np.sin(ang)
    v[:, 2] = center[2]
    return v


def square_loop(side: float, n_seg: int, center=(0.0, 0.0, 0.0)) -> np.ndarray:
    """Square of the given side, corner (-s/2,-s/2) first, CCW, each side cut
    into n_seg/4 equal segments."""
    if n_seg % 4:
        raise ValueError("square loops need a multiple of 4 segments")
    m = n_seg // 4
    h = side / 2.0
    corners = np.array([[-h, -h], [h, -h], [h, h], [-h, h]])
    pts = []
    for c in range(4):
        a, b = corners[c], corners[(c + 1) % 4]
        for i in range(m):
            t = i / m
            pts.append(a + (b - a) * t)
    v = np.zeros((n_seg, 3))
    v[:, :2] = np.asarray(pts)
    v[:, 0] += center[0]
    v[:, 1] += center[1]
    v[:, 2] += center[2]
    return v


@dataclasses.dataclass
class Geometry:
    """A set of closed wire loops (one tunable capacitor per loop)."""
    verts: np.ndarray      # [V,3] float64
    seg_off: np.ndarray    # [n+1] int32
    wire_a: np.ndarray     # [n] float64 wire radius
    R: np.ndarray          # [n] float64 series resistance
    nx: int = 1
    ny: int = 1
    pitch: float = 0.0

    @property
    def n(self) -> int:
        return int(self.seg_off.shape[0] - 1)

    def loop(self, k: int) -> np.ndarray:
        return self.verts[self.seg_off[k]:self.seg_off[k + 1]]


def square_array(nx: int, ny: int, side: float, pitch: float, n_seg: int,
                 wire_a: float = 1e-3, R: float = 0.3) -> Geometry:
    loops = []
    for iy in range(ny):
        for ix in range(nx):
            c = ((ix - (nx - 1) / 2.0) * pitch, (iy - (ny - 1) / 2.0) * pitch, 0.0)
            loops.append(square_loop(side, n_seg, c))
    return _pack(loops, wire_a, R, nx, ny, pitch)


def single_circle(radius: float = 0.05, n_seg: int = 64, wire_a: float = 1e-3,
                  R: float = 0.5) -> Geometry:
    return _pack([regular_polygon(radius, n_seg)], wire_a, R, 1, 1, 0.0)


def _pack(loops: Sequence[np.ndarray], wire_a, R, nx, ny, pitch) -> Geometry:
    n = len(loops)
    seg_off = np.zeros(n + 1, dtype=np.int32)
    seg_off[1:] = np.cumsum([len(l) for l in loops])
    verts = np.ascontiguousarray(np.concatenate(loops, axis=0), dtype=np.float64)
    wa = np.broadcast_to(np.asarray(wire_a, dtype=np.float64), (n,)).copy()
    rr = np.broadcast_to(np.asarray(R, dtype=np.float64), (n,)).copy()
    return Geometry(verts, seg_off, wa, rr, nx, ny, pitch)


def grid_points(n_side: int, extent: float, z_planes: Sequence[float]) -> np.ndarray:
    """[P,3] grid, plane-major then y then x, inclusive linspace over extent."""
    xs = np.linspace(-extent / 2.0, extent / 2.0, n_side)
    out = []
    for z in z_planes:
        yy, xx = np.meshgrid(xs, xs, indexing="ij")
        p = np.zeros((n_side * n_side, 3))
        p[:, 0] = xx.ravel()
        p[:, 1] = yy.ravel()
        p[:, 2] = z
        out.append(p)
    return np.ascontiguousarray(np.concatenate(out, axis=0))


# --------------------------------------------------------------------------
# targets (synthetic magnitudes; none is derived from the field model)
# --------------------------------------------------------------------------

def gaussian_hotspot(pts: np.ndarray, center_xy, sigma: float, peak: float) -> np.ndarray:
    d2 = (pts[:, 0] - center_xy[0]) ** 2 + (pts[:, 1] - center_xy[1]) ** 2
    return peak * np.exp(-d2 / (2.0 * sigma * sigma))


def smooth_noise_target(rng: np.random.Generator, n_side: int, extent: float,
                        sigma: float, peak: float, n_planes: int = 1) -> np.ndarray:
    """White N(0,1) noise on the grid, Gaussian-filtered (sigma in metres,
    reflect boundary), absolute value, scaled to the given peak."""
    from scipy.ndimage import gaussian_filter
    dx = extent / (n_side - 1)
    planes = []
    for _ in range(n_planes):
        w = rng.standard_normal((n_side, n_side))
        f = np.abs(gaussian_filter(w, sigma / dx, mode="reflect"))
        planes.append((peak * f / f.max()).ravel())
    return np.concatenate(planes)


# --------------------------------------------------------------------------
# workload configurations
# --------------------------------------------------------------------------

@dataclasses.dataclass
class Workload:
    name: str
    geom: Geometry
    pts: np.ndarray        # [P,3]
    C: np.ndarray          # [B,n] farads
    freqs: np.ndarray      # [F] hertz
    target: np.ndarray     # [P] tesla (non-negative magnitudes)
    bext_z: float = 1e-6

    @property
    def omega(self) -> np.ndarray:
        return 2.0 * np.pi * self.freqs

    @property
    def B(self) -> int:
        return int(self.C.shape[0])

    @property
    def F(self) -> int:
        return int(self.freqs.shape[0])

    @property
    def P(self) -> int:
        return int(self.pts.shape[0])

    def summary(self) -> dict:
        return {"workload": self.name, "loops": self.geom.n,
                "segments": int(self.geom.verts.shape[0]), "points": self.P,
                "freqs": self.F, "batch": self.B}


def config1_single_loop(batch: int = 64, grid: int = 32) -> Workload:
    """Single circular copper loop r=5 cm, 64 segments, R=0.5 ohm, wire 1 mm,
    capacitor swept over [10,200] pF at 128 MHz; B_z on a grid over 12x12 cm
    at z=2 cm."""
    rng = rng_for(1)
    g = single_circle(0.05, 64, 1e-3, 0.5)
    pts = grid_points(grid, 0.12, [0.02])
    C = np.linspace(10e-12, 200e-12, batch).reshape(batch, 1)
    c = rng.uniform(-0.03, 0.03, size=2)
    T = gaussian_hotspot(pts, c, 0.03, 0.2e-6)
    return Workload("single_loop_64seg", g, pts, C, np.array([128e6]), T)


def config2_line8(batch: int = 1024, grid: int = 64) -> Workload:
    """8x1 line of 4 cm squares at 5 cm pitch, 32 segments per loop,
    C uniform in [20,150] pF, R=0.3 ohm, 128 MHz, B_z on 64x64 at z=1.5 cm."""
    rng = rng_for(2)
    g = square_array(8, 1, 0.04, 0.05, 32, 1e-3, 0.3)
    pts = grid_points(grid, 8 * 0.05, [0.015])
    C = rng.uniform(20e-12, 150e-12, size=(batch, 8))
    c = np.array([rng.uniform(-0.175, 0.175), 0.0])
    T = gaussian_hotspot(pts, c, 0.03, 0.5e-6)
    return Workload("array_8x1", g, pts, C, np.array([128e6]), T)


def config3_array8x8(batch: int = 4096, grid: int = 256, two_planes: bool = False,
                     n_freq: int = 21) -> Workload:
    """8x8 array of 3 cm squares at 3.5 cm pitch, 32 segments per loop,
    C uniform in [20,150] pF, 21 frequencies 118..138 MHz, B_z on 256x256
    points over 28 cm at z=1 cm (and z=3 cm when two_planes), Gaussian
    hotspot target sigma=3 cm, 2 uT, seeded centre."""
    rng = rng_for(3)
    g = square_array(8, 8, 0.03, 0.035, 32, 1e-3, 0.3)
    planes = [0.01, 0.03] if two_planes else [0.01]
    pts = grid_points(grid, 8 * 0.035, planes)
    C = rng.uniform(20e-12, 150e-12, size=(batch, 64))
    c = rng.uniform(-0.14, 0.14, size=2)
    T = gaussian_hotspot(pts, c, 0.03, 2e-6)
    freqs = np.linspace(118e6, 138e6, n_freq)
    return Workload("array_8x8", g, pts, C, freqs, T)


def config4_instances(count: int = 2048, grid_range=(128, 256), stream: int = 0) -> list:
    """Ragged configuration: `count` independent instances, each its own
    square array (n_side uniform in {4, 6, 8, 12, 16}: 16 to 256 loops, 3 cm
    squares at 3.5 cm pitch, 32 segments), its own g x g grid at z = 1 cm over
    the array footprint (g uniform integer in grid_range), its own F uniform in
    1..8 frequencies drawn uniformly in [118, 138] MHz (sorted), one
    configuration with C log-uniform in [10, 300] pF, and a Gaussian hotspot
    target (sigma 3 cm, 1 uT, seeded centre)."""
    rng = rng_for(4, stream)
    out = []
    for i in range(count):
        ns = int(rng.choice([4, 6, 8, 12, 16]))
        gsz = int(rng.integers(grid_range[0], grid_range[1] + 1))
        nf = int(rng.integers(1, 9))
        g = square_array(ns, ns, 0.03, 0.035, 32, 1e-3, 0.3)
        ext = ns * 0.035
        pts = grid_points(gsz, ext, [0.01])
        freqs = np.sort(rng.uniform(118e6, 138e6, size=nf))
        C = np.exp(rng.uniform(np.log(10e-12), np.log(300e-12), size=(1, ns * ns)))
        c = rng.uniform(-ext / 2, ext / 2, size=2)
        T = gaussian_hotspot(pts, c, 0.03, 1e-6)
        out.append(Workload(f"ragged_{i}", g, pts, C, freqs, T))
    return out


def config5_array32x32(batch: int = 256, grid: int = 512) -> Workload:
    """32x32 array (1024 loops), 512x512 points at z=2 cm, batch 256, F=1,
    smooth random target (Gaussian-filtered noise, sigma=4 cm, peak 2 uT)."""
    rng = rng_for(5)
    g = square_array(32, 32, 0.03, 0.035, 32, 1e-3, 0.3)
    ext = 32 * 0.035
    pts = grid_points(grid, ext, [0.02])
    C = rng.uniform(20e-12, 150e-12, size=(batch, 1024))
    T = smooth_noise_target(rng, grid, ext, 0.04, 2e-6)
    return Workload("array_32x32", g, pts, C, np.array([128e6]), T)


def small_array(nx: int, ny: int, batch: int, grid: int, n_freq: int = 3,
                n_seg: int = 32, seed: int = 0, side: float = 0.03,
                pitch: float = 0.035, z: Sequence[float] = (0.01,),
                c_range=(20e-12, 150e-12)) -> Workload:
    """Reduced-size square array for parity tests (same recipe as the 8x8)."""
    rng = np.random.default_rng([SEED_BASE, 100, seed])
    g = square_array(nx, ny, side, pitch, n_seg, 1e-3, 0.3)
    ext = max(nx, ny) * pitch
    pts = grid_points(grid, ext, list(z))
    C = rng.uniform(c_range[0], c_range[1], size=(batch, nx * ny))
    c = rng.uniform(-ext / 2, ext / 2, size=2)
    T = gaussian_hotspot(pts, c, 0.03, 2e-7)
    freqs = np.linspace(118e6, 138e6, n_freq) if n_freq > 1 else np.array([128e6])
    return Workload(f"array_{nx}x{ny}_small", g, pts, C, freqs, T)


def with_drive_coil(g: Geometry, radius: float = 0.0445, z: float = 0.02, n_seg: int = 64,
                    wire_a: float = 0.5e-3, square: bool = False) -> Geometry:
    """g plus one coaxial excitation coil, appended as the last loop (a
    perfect conductor: R = 0; its port is described separately).  The
    default is a circular 1 mm wire on a 45 mm outer radius, as in the
    single-cell setup of Sec. IV-A, at an axial offset z (the paper gives
    none); `square` makes it a square of side 2 radius instead."""
    coil = (square_loop(2.0 * radius, n_seg, (0.0, 0.0, z)) if square
            else regular_polygon(radius, n_seg, (0.0, 0.0, z)))
    loops = [g.loop(k) for k in range(g.n)] + [coil]
    wa = np.concatenate([g.wire_a, [wire_a]])
    rr = np.concatenate([g.R, [0.0]])
    return _pack(loops, wa, rr, g.nx, g.ny, g.pitch)


def random_points(rng: np.random.Generator, P: int, extent: float, zmin: float,
                  zmax: float) -> np.ndarray:
    p = np.zeros((P, 3))
    p[:, 0] = rng.uniform(-extent / 2, extent / 2, P)
    p[:, 1] = rng.uniform(-extent / 2, extent / 2, P)
    p[:, 2] = rng.uniform(zmin, zmax, P)
    return p


CONFIGS = {
    1: config1_single_loop,
    2: config2_line8,
    3: config3_array8x8,
    5: config5_array32x32,
}
