"""Seeded synthetic terrestrial-LiDAR scans (input generator only).

This module produces the int32 millimetre point clouds that both the HIP path
and the CPU oracle consume.  It holds none of the decimation arithmetic: it
casts rays from a tripod-mounted station against a box scene and quantises the
hit points.

Scan model (the paper's workloads are stationary LiDAR scans of buildings,
taken from a tripod about 1.5 m above the ground, merged from 2-38 stations,
with an equal number of samples per elevation row so that density peaks at
the poles; Introduction, Sec. 6):

* station at height 1500 mm;
* row i of R: elevation -60 deg + 150 deg * i / (R - 1);
* column j of C: azimuth 360 deg * j / C;
* range noise N(0, sigma) mm added along the ray, sigma = 2 mm;
* xyz rounded to the nearest millimetre (numpy ``rint``) and stored as int32.

Every ray must hit so that the point count equals R * C: the scene is closed
by an axis-aligned box whose floor is the ground plane z = 0.

All randomness comes from ``numpy.random.Generator(PCG64(seed))``.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

DEG = math.pi / 180.0


@dataclass(frozen=True)
class Scene:
    """Solid axis-aligned boxes (mm) inside a closing box (mm)."""

    box_lo: np.ndarray  # [nb, 3] float64
    box_hi: np.ndarray  # [nb, 3] float64
    close_lo: np.ndarray  # [3]
    close_hi: np.ndarray  # [3]


def _ray_dirs(rows: int, cols: int) -> tuple[np.ndarray, np.ndarray]:
    el = (-60.0 + 150.0 * np.arange(rows, dtype=np.float64) / max(rows - 1, 1)) * DEG
    az = (360.0 * np.arange(cols, dtype=np.float64) / cols) * DEG
    return el, az


def wall_scene(rng: np.random.Generator, nboxes: int, rmin_m: float, rmax_m: float,
               close_half_m: float, close_height_m: float,
               centres_xy_mm: np.ndarray | None = None) -> Scene:
    """Random wall-like boxes: 0.2-0.5 m thick, 2-20 m long, 2-10 m high.

    Each box is placed at a distance drawn from U[rmin, rmax] metres (and a
    uniform bearing) from a random anchor in ``centres_xy_mm`` (the station
    positions; the origin if None), resting on the ground.  Boxes that would
    contain any station (with a 1 m margin) are redrawn.
    """
    if centres_xy_mm is None:
        centres_xy_mm = np.zeros((1, 2))
    lo = np.zeros((nboxes, 3))
    hi = np.zeros((nboxes, 3))
    b = 0
    while b < nboxes:
        thick = rng.uniform(200.0, 500.0)
        length = rng.uniform(2000.0, 20000.0)
        height = rng.uniform(2000.0, 10000.0)
        dist = rng.uniform(rmin_m, rmax_m) * 1000.0
        bearing = rng.uniform(0.0, 2.0 * math.pi)
        along_x = rng.uniform() < 0.5
        anchor = centres_xy_mm[rng.integers(0, len(centres_xy_mm))]
        cx = anchor[0] + dist * math.cos(bearing)
        cy = anchor[1] + dist * math.sin(bearing)
        sx, sy = (length, thick) if along_x else (thick, length)
        blo = np.array([cx - sx / 2, cy - sy / 2, 0.0])
        bhi = np.array([cx + sx / 2, cy + sy / 2, height])
        # keep every station outside every box, with a margin
        inside = ((centres_xy_mm[:, 0] > blo[0] - 1000) & (centres_xy_mm[:, 0] < bhi[0] + 1000) &
                  (centres_xy_mm[:, 1] > blo[1] - 1000) & (centres_xy_mm[:, 1] < bhi[1] + 1000))
        if inside.any():
            continue
        lo[b], hi[b] = blo, bhi
        b += 1
    ch = close_half_m * 1000.0
    cmin = centres_xy_mm.min(axis=0)
    cmax = centres_xy_mm.max(axis=0)
    close_lo = np.array([cmin[0] - ch, cmin[1] - ch, 0.0])
    close_hi = np.array([cmax[0] + ch, cmax[1] + ch, close_height_m * 1000.0])
    return Scene(lo, hi, close_lo, close_hi)


def _slab(o, lo, hi, dx, dy, dz):
    """Entry distance of rays o + t (dx, dy, dz) into the box [lo, hi]
    (inf where the ray misses it or starts past it)."""
    with np.errstate(divide="ignore", invalid="ignore"):
        tn = np.full(dx.shape, -np.inf)
        tf = np.full(dx.shape, np.inf)
        for a, d in enumerate((dx, dy, dz)):
            inv = 1.0 / d
            t1 = (lo[a] - o[a]) * inv
            t2 = (hi[a] - o[a]) * inv
            a_min = np.where(np.isnan(t1), -np.inf, np.minimum(t1, t2))
            a_max = np.where(np.isnan(t1), np.inf, np.maximum(t1, t2))
            tn = np.maximum(tn, a_min)
            tf = np.minimum(tf, a_max)
        return np.where((tn <= tf) & (tn > 0.0), tn, np.inf)


def _exit(o, lo, hi, dx, dy, dz):
    """Exit distance of rays starting inside the box [lo, hi]."""
    with np.errstate(divide="ignore", invalid="ignore"):
        t = np.full(dx.shape, np.inf)
        for a, d in enumerate((dx, dy, dz)):
            bound = np.where(d > 0, hi[a], lo[a])
            ta = (bound - o[a]) / d
            t = np.minimum(t, np.where(d == 0, np.inf, ta))
        return t


def _window(o, lo, hi, rows, cols):
    """Row range and column indices of the rays that can reach box [lo, hi]
    from station o (conservative: footprint corners bound the azimuth; the
    nearest and farthest horizontal distances bound the elevation)."""
    cx = np.array([lo[0], hi[0], lo[0], hi[0]]) - o[0]
    cy = np.array([lo[1], lo[1], hi[1], hi[1]]) - o[1]
    mid = math.atan2((lo[1] + hi[1]) / 2 - o[1], (lo[0] + hi[0]) / 2 - o[0])
    diff = (np.arctan2(cy, cx) - mid + math.pi) % (2 * math.pi) - math.pi
    a0, a1 = mid + diff.min(), mid + diff.max()
    step = 2 * math.pi / cols
    j0 = int(math.floor((a0 % (2 * math.pi)) / step)) - 1
    nj = int(math.ceil((a1 - a0) / step)) + 3
    jcols = np.arange(j0, j0 + min(nj, cols)) % cols
    hx = max(lo[0] - o[0], 0.0, o[0] - hi[0])
    hy = max(lo[1] - o[1], 0.0, o[1] - hi[1])
    dmin = max(math.hypot(hx, hy), 1e-9)
    dmax = float(np.sqrt(cx ** 2 + cy ** 2).max())
    el_hi = math.atan2(hi[2] - o[2], dmin if hi[2] > o[2] else dmax)
    el_lo = math.atan2(lo[2] - o[2], dmin if lo[2] < o[2] else dmax)
    to_row = lambda e: (math.degrees(e) + 60.0) / 150.0 * (rows - 1)  # noqa: E731
    i0 = max(0, int(math.floor(to_row(el_lo))) - 1)
    i1 = min(rows, int(math.ceil(to_row(el_hi))) + 2)
    return i0, i1, jcols


def scan_station(rows: int, cols: int, station_xy_mm: tuple[float, float], scene: Scene,
                 rng: np.random.Generator, sigma_mm: float = 2.0, height_mm: float = 1500.0) -> np.ndarray:
    """One station's R x C scan as int32 [R*C, 3], row-major (row, column)."""
    el, az = _ray_dirs(rows, cols)
    o = np.array([station_xy_mm[0], station_xy_mm[1], height_mm], dtype=np.float64)
    ce, se = np.cos(el)[:, None], np.sin(el)[:, None]
    ca, sa = np.cos(az)[None, :], np.sin(az)[None, :]
    dx, dy, dz = ce * ca, ce * sa, np.broadcast_to(se, (rows, cols))
    t = _exit(o, scene.close_lo, scene.close_hi, dx, dy, dz)
    for b in range(scene.box_lo.shape[0]):
        lo, hi = scene.box_lo[b], scene.box_hi[b]
        i0, i1, jc = _window(o, lo, hi, rows, cols)
        if i0 >= i1:
            continue
        sub = np.ix_(np.arange(i0, i1), jc)
        tb = _slab(o, lo, hi, dx[sub], dy[sub], dz[sub])
        t[sub] = np.minimum(t[sub], tb)
    t = t + rng.normal(0.0, sigma_mm, size=t.shape)
    out = np.empty((rows, cols, 3), dtype=np.int32)
    out[..., 0] = np.rint(o[0] + t * dx)
    out[..., 1] = np.rint(o[1] + t * dy)
    out[..., 2] = np.rint(o[2] + t * dz)
    return out.reshape(-1, 3)


# ----------------------------------------------------------------------------
# the five workload configurations
# ----------------------------------------------------------------------------

@dataclass(frozen=True)
class Workload:
    name: str
    xyz: np.ndarray          # int32 [n, 3]
    k: int
    keep: int
    offsets: np.ndarray | None = None   # int64 [nscan+1] for batches
    keeps: np.ndarray | None = None     # int64 [nscan] for batches


def single_scan(rows: int, cols: int, nboxes: int, rmin_m: float, rmax_m: float,
                close_half_m: float, seed: int, close_height_m: float | None = None,
                sigma_mm: float = 2.0) -> np.ndarray:
    rng = np.random.Generator(np.random.PCG64(seed))
    if close_height_m is None:
        close_height_m = max(20.0, close_half_m / 2.0)
    scene = wall_scene(rng, nboxes, rmin_m, rmax_m, close_half_m, close_height_m)
    return scan_station(rows, cols, (0.0, 0.0), scene, rng, sigma_mm)


def place_stations(rng: np.random.Generator, count: int, square_m: float,
                   dmin_m: float = 30.0, dmax_m: float = 80.0) -> np.ndarray:
    """Stations by rejection: each 30-80 m from its nearest earlier station,
    at least 30 m from all of them, inside a square of side ``square_m``."""
    half = square_m * 500.0
    st = [np.zeros(2)]
    tries = 0
    while len(st) < count:
        tries += 1
        if tries > 1_000_000:
            raise RuntimeError("station placement failed")
        c = rng.uniform(-half, half, size=2)
        dist = np.sqrt(((np.array(st) - c) ** 2).sum(axis=1))
        if dist.min() >= dmin_m * 1000 and dist.min() <= dmax_m * 1000:
            st.append(c)
    return np.array(st)


_M64 = (1 << 64) - 1


def _mix64(x: np.ndarray) -> np.ndarray:
    """splitmix64 output function on uint64 arrays (wrapping arithmetic)."""
    x = x + np.uint64(0x9E3779B97F4A7C15)
    x = (x ^ (x >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
    x = (x ^ (x >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
    return x ^ (x >> np.uint64(31))


def ray_noise(seed: int, station: int, ray: np.ndarray, sigma_mm: float) -> np.ndarray:
    """Range noise N(0, sigma) of rays ``ray`` (row * cols + column) of one
    station of a merged cloud.  Counter-based: two uniforms from the
    splitmix64 hash of (seed, station, ray), then Box-Muller, so that any
    subset of a scan's rays gets the values the whole scan has."""
    key = np.array([(seed * 0x100000001B3 + station * 0x9E3779B1) & _M64], dtype=np.uint64)
    key = _mix64(key)
    c = ray.astype(np.uint64) << np.uint64(1)
    u1 = (_mix64(key ^ c) >> np.uint64(11)).astype(np.float64) * (1.0 / 9007199254740992.0)
    u2 = (_mix64(key ^ (c | np.uint64(1))) >> np.uint64(11)).astype(np.float64) * (1.0 / 9007199254740992.0)
    return sigma_mm * np.sqrt(-2.0 * np.log1p(-u1)) * np.cos(2.0 * math.pi * u2)


def station_rays(rows: int, cols: int, o: np.ndarray, scene: Scene, i0: int, i1: int, jcols: np.ndarray,
                 seed: int, station: int, sigma_mm: float) -> np.ndarray:
    """Hit points (int32 [.., 3]) of the rays of rows [i0, i1) x columns
    ``jcols`` (ascending) of one station of a merged cloud, row-major."""
    el, az = _ray_dirs(rows, cols)
    el, az = el[i0:i1], az[jcols]
    nr, nc = i1 - i0, len(jcols)
    ce, se = np.cos(el)[:, None], np.sin(el)[:, None]
    dx, dy, dz = ce * np.cos(az)[None, :], ce * np.sin(az)[None, :], np.broadcast_to(se, (nr, nc))
    t = _exit(o, scene.close_lo, scene.close_hi, dx, dy, dz)
    col_pos = np.full(cols, -1, dtype=np.int64)
    col_pos[jcols] = np.arange(nc)
    for b in range(scene.box_lo.shape[0]):
        lo, hi = scene.box_lo[b], scene.box_hi[b]
        b0, b1, jc = _window(o, lo, hi, rows, cols)
        r0, r1 = max(b0, i0), min(b1, i1)
        sel = col_pos[jc]
        sel = sel[sel >= 0]
        if r0 >= r1 or len(sel) == 0:
            continue
        sub = np.ix_(np.arange(r0 - i0, r1 - i0), sel)
        t[sub] = np.minimum(t[sub], _slab(o, lo, hi, dx[sub], dy[sub], dz[sub]))
    ray = np.arange(i0, i1, dtype=np.int64)[:, None] * cols + jcols[None, :].astype(np.int64)
    t = t + ray_noise(seed, station, ray, sigma_mm)
    out = np.empty((nr, nc, 3), dtype=np.int32)
    out[..., 0] = np.rint(o[0] + t * dx)
    out[..., 1] = np.rint(o[1] + t * dy)
    out[..., 2] = np.rint(o[2] + t * dz)
    return out.reshape(-1, 3)


def multi_station(stations: int, rows: int, cols: int, nboxes: int, square_m: float,
                  seed: int, sigma_mm: float = 2.0, crop: tuple | None = None) -> np.ndarray:
    """Scans of ``stations`` stations (placed by place_stations) of one
    scene, concatenated station by station, each row-major.  With ``crop`` =
    (lo, hi) (mm, xyz) only the points inside that box, in the same order:
    each station casts just the rays that can reach the box."""
    rng = np.random.Generator(np.random.PCG64(seed))
    st = place_stations(rng, stations, square_m)
    scene = wall_scene(rng, nboxes, 2.0, 50.0, 60.0, 40.0, centres_xy_mm=st)
    parts = []
    for s, c in enumerate(st):
        o = np.array([c[0], c[1], 1500.0])
        i0, i1, jcols = 0, rows, np.arange(cols)
        if crop is not None:
            lo, hi = np.asarray(crop[0], dtype=np.float64), np.asarray(crop[1], dtype=np.float64)
            if not (lo[0] <= o[0] <= hi[0] and lo[1] <= o[1] <= hi[1]):
                i0, i1, jcols = _window(o, lo, hi, rows, cols)
                jcols = np.unique(jcols)
        p = station_rays(rows, cols, o, scene, i0, i1, jcols, seed, s, sigma_mm)
        if crop is not None:
            m = ((p >= np.asarray(crop[0])) & (p <= np.asarray(crop[1]))).all(axis=1)
            p = p[m]
        parts.append(p)
    return np.concatenate(parts, axis=0)


# Half-width (mm) of the crop of the merged clouds: the box from -3 m to
# +3 m around the first station in x and y, -1 m to 12 m in z, which holds
# about 20M points of either merged cloud (the ground around the tripod,
# densest near its foot, plus the sparse hits of the other stations).
CROP_HALF_MM = 3000


def crop_box(half_mm: int = CROP_HALF_MM) -> tuple:
    return ((-half_mm, -half_mm, -1000), (half_mm, half_mm, 12000))


def config(idx: int, scale: float = 1.0, seed: int | None = None, crop: bool = False) -> Workload:
    """Workload ``idx`` (1-5).  ``scale`` < 1 shrinks the ray grid (rows and
    columns by sqrt(scale)) for quick tests; 1.0 is the stated size.  For the
    merged clouds (3, 5), ``crop`` gives only the points inside crop_box(),
    re-indexed from 0 in their order in the whole cloud, with the keep ratio
    of the whole."""
    def grid(r, c):
        f = math.sqrt(scale)
        return max(2, int(round(r * f))), max(2, int(round(c * f)))

    if idx == 1:
        r, c = grid(500, 400)
        xyz = single_scan(r, c, 6, 2.0, 50.0, 50.0, 1 if seed is None else seed)
        n = xyz.shape[0]
        keep = n // 4
        return Workload("scan-200k-k8-keep25", xyz, 8, keep)
    if idx == 2:
        r, c = grid(5000, 4000)
        xyz = single_scan(r, c, 40, 2.0, 120.0, 120.0, 2 if seed is None else seed)
        n = xyz.shape[0]
        return Workload("scan-20M-k16-keep10", xyz, 16, n // 10)
    if idx == 3:
        r, c = grid(10000, 5000)
        xyz = multi_station(10, r, c, 60, 400.0, 3 if seed is None else seed, crop=crop_box() if crop else None)
        n = xyz.shape[0]
        return Workload("merged-10st-500M-k8-keep5" + ("/crop3m" if crop else ""), xyz, 8, n // 20)
    if idx == 4:
        return batch_config(4096 if scale >= 1.0 else max(2, int(4096 * scale)),
                            scale=1.0 if scale >= 1.0 else scale, base_seed=10000 if seed is None else seed)
    if idx == 5:
        r, c = grid(10000, 5000)
        xyz = multi_station(40, r, c, 200, 1000.0, 5 if seed is None else seed, crop=crop_box() if crop else None)
        n = xyz.shape[0]
        return Workload("merged-40st-2B-k8-keep2" + ("/crop3m" if crop else ""), xyz, 8, n // 50)
    raise ValueError(idx)


def batch_scan_shape(seed: int, size_scale: float = 1.0) -> tuple[int, int, float]:
    """(rows, cols, keep_ratio) of batch scan ``seed``: n log-uniform in
    [1e4, 2e6], aspect log-uniform in [1/2, 2], keep ratio U[0.1, 0.5]."""
    rng = np.random.Generator(np.random.PCG64(seed))
    n = math.exp(rng.uniform(math.log(1e4), math.log(2e6))) * size_scale
    aspect = math.exp(rng.uniform(math.log(0.5), math.log(2.0)))
    rows = max(2, int(round(math.sqrt(n * aspect))))
    cols = max(2, int(round(n / rows)))
    ratio = rng.uniform(0.1, 0.5)
    return rows, cols, ratio


def batch_scan(seed: int, size_scale: float = 1.0) -> tuple[np.ndarray, int]:
    rows, cols, ratio = batch_scan_shape(seed, size_scale)
    xyz = single_scan(rows, cols, 6, 2.0, 50.0, 50.0, seed + 7_000_000)
    n = xyz.shape[0]
    return xyz, max(1, int(math.floor(ratio * n)))


def batch_config(nscan: int, scale: float = 1.0, base_seed: int = 10000) -> Workload:
    parts, keeps = [], []
    for s in range(nscan):
        xyz, keep = batch_scan(base_seed + s, scale)
        parts.append(xyz)
        keeps.append(keep)
    offs = np.zeros(nscan + 1, dtype=np.int64)
    offs[1:] = np.cumsum([p.shape[0] for p in parts])
    return Workload(f"batch-{nscan}scans-k8", np.concatenate(parts), 8, int(sum(keeps)),
                    offsets=offs, keeps=np.array(keeps, dtype=np.int64))


def random_cloud(n: int, box_mm: int, seed: int) -> np.ndarray:
    """Uniform integer points in [0, box_mm)^3: small boxes give many
    duplicates and distance ties."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.integers(0, box_mm, size=(n, 3), dtype=np.int64).astype(np.int32)
