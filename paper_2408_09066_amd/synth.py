"""Seeded synthetic lidar-like workloads (inputs only; none of the method's arithmetic).

The paper's datasets (ToySim, Intel Map, EviLOG; Sec. IV, dataset summary table) are not
available, so every workload here is generated: a square world with axis-aligned rectangles and
circles, one or more sensor poses, beams at evenly spaced angles, ranges ray-cast exactly and
perturbed by Gaussian noise.  Beam end points are labelled occupied (psi = 1) and points drawn
uniformly along each beam are labelled empty (psi = 0), the labelling heuristic of Sec. III-B
(data format and preprocessing).

The phase basis Theta is also drawn here: it is the one random draw the method makes
(initialisation of the axis vectors, Sec. III-B), so it is passed to both the oracle and the GPU
library as an input.  Theta[k] = theta_k / l with theta_k ~ U[-pi, pi] per axis for
k = 1..D/2-1, mirrored as Theta[D-k] = -Theta[k], and Theta[0] = Theta[D/2] = 0 so that every
fractional power of the axis spectra is the spectrum of a real vector.

Every array comes from ``numpy.random.default_rng(SeedSequence([2408, config_id, stream]))``
with streams 0: Theta, 1: world, 2: poses, 3: range noise, 4: empty samples, 5: request stream.
"""
from __future__ import annotations

import dataclasses
import hashlib
import math
from typing import Dict, List, Optional, Tuple

import numpy as np

STREAM_THETA, STREAM_WORLD, STREAM_POSES, STREAM_NOISE, STREAM_EMPTY, STREAM_REQUESTS = range(6)


def rng_for(config_id: int, stream: int) -> np.random.Generator:
    return np.random.default_rng(np.random.SeedSequence([2408, int(config_id), int(stream)]))


def make_theta(D: int, ell: float, rng: np.random.Generator) -> np.ndarray:
    """Conjugate-symmetric phase basis, float64 [D][2] in rad/m (already divided by l)."""
    if D < 4 or D % 2:
        raise ValueError("D must be even and >= 4")
    h = D // 2
    th = np.zeros((D, 2), dtype=np.float64)
    ph = rng.uniform(-np.pi, np.pi, size=(h - 1, 2))
    th[1:h] = ph
    th[h + 1:] = -ph[::-1]
    return th / float(ell)


@dataclasses.dataclass
class World:
    half: float                      # world is [-half, half]^2, its boundary is a wall
    rects: np.ndarray                # [nr][4] xmin, ymin, xmax, ymax
    circles: np.ndarray              # [nc][3] cx, cy, radius


def _dist_to_obstacles(p: np.ndarray, w: World) -> float:
    d = math.inf
    for xmn, ymn, xmx, ymx in w.rects:
        dx = max(xmn - p[0], 0.0, p[0] - xmx)
        dy = max(ymn - p[1], 0.0, p[1] - ymx)
        d = min(d, math.hypot(dx, dy))
    for cx, cy, r in w.circles:
        d = min(d, math.hypot(p[0] - cx, p[1] - cy) - r)
    return d


def make_world(half: float, n_rect: int, n_circ: int, rect_side: Tuple[float, float],
               circ_radius: Tuple[float, float], keep_clear: np.ndarray, clearance: float,
               rng: np.random.Generator) -> World:
    rects: List[List[float]] = []
    circles: List[List[float]] = []
    tries = 0
    while len(rects) < n_rect:
        tries += 1
        if tries > 100000:
            raise RuntimeError("could not place rectangles")
        sx, sy = rng.uniform(rect_side[0], rect_side[1], size=2)
        cx, cy = rng.uniform(-half + sx / 2, half - sx / 2), rng.uniform(-half + sy / 2, half - sy / 2)
        r = [cx - sx / 2, cy - sy / 2, cx + sx / 2, cy + sy / 2]
        ok = True
        for p in keep_clear:
            dx = max(r[0] - p[0], 0.0, p[0] - r[2])
            dy = max(r[1] - p[1], 0.0, p[1] - r[3])
            if math.hypot(dx, dy) < clearance:
                ok = False
                break
        if ok:
            rects.append(r)
    tries = 0
    while len(circles) < n_circ:
        tries += 1
        if tries > 100000:
            raise RuntimeError("could not place circles")
        rad = rng.uniform(circ_radius[0], circ_radius[1])
        cx, cy = rng.uniform(-half + rad, half - rad, size=2)
        if all(math.hypot(cx - p[0], cy - p[1]) - rad >= clearance for p in keep_clear):
            circles.append([cx, cy, rad])
    return World(half, np.array(rects, dtype=np.float64).reshape(-1, 4),
                 np.array(circles, dtype=np.float64).reshape(-1, 3))


def random_walk(world: World, n: int, start: np.ndarray, rng: np.random.Generator,
                step=(0.5, 1.5), margin: float = 0.5) -> np.ndarray:
    poses = [np.asarray(start, dtype=np.float64)]
    heading = rng.uniform(-np.pi, np.pi)
    tries = 0
    while len(poses) < n:
        tries += 1
        if tries > 200000:
            raise RuntimeError("random walk got stuck")
        heading += rng.normal(0.0, 0.6)
        s = rng.uniform(*step)
        q = poses[-1] + s * np.array([math.cos(heading), math.sin(heading)])
        if np.any(np.abs(q) > world.half - 1.0) or _dist_to_obstacles(q, world) < margin:
            heading += rng.uniform(-np.pi, np.pi)
            continue
        poses.append(q)
    return np.stack(poses)


def raycast(world: World, pose: np.ndarray, angles: np.ndarray) -> np.ndarray:
    """Exact range from pose along each angle to the first wall, rectangle or circle."""
    dx, dy = np.cos(angles), np.sin(angles)
    px, py = float(pose[0]), float(pose[1])
    with np.errstate(divide="ignore", invalid="ignore"):
        # world boundary (ray starts inside): exit distance
        tx = np.where(dx > 0, (world.half - px) / dx, np.where(dx < 0, (-world.half - px) / dx, np.inf))
        ty = np.where(dy > 0, (world.half - py) / dy, np.where(dy < 0, (-world.half - py) / dy, np.inf))
        t = np.minimum(tx, ty)
        if len(world.rects):
            # slab test, obstacles x beams at once
            xmn, ymn, xmx, ymx = (world.rects[:, i:i + 1] for i in range(4))
            DX, DY = dx[None, :], dy[None, :]
            t1x = np.where(DX != 0, (xmn - px) / DX, np.where(px >= xmn, -np.inf, np.inf))
            t2x = np.where(DX != 0, (xmx - px) / DX, np.where(px <= xmx, np.inf, -np.inf))
            t1y = np.where(DY != 0, (ymn - py) / DY, np.where(py >= ymn, -np.inf, np.inf))
            t2y = np.where(DY != 0, (ymx - py) / DY, np.where(py <= ymx, np.inf, -np.inf))
            tmin = np.maximum(np.minimum(t1x, t2x), np.minimum(t1y, t2y))
            tmax = np.minimum(np.maximum(t1x, t2x), np.maximum(t1y, t2y))
            hit = (tmax >= tmin) & (tmin > 0)
            t = np.minimum(t, np.where(hit, tmin, np.inf).min(axis=0))
        if len(world.circles):
            ox, oy = px - world.circles[:, 0:1], py - world.circles[:, 1:2]
            b = ox * dx[None, :] + oy * dy[None, :]
            c = ox * ox + oy * oy - world.circles[:, 2:3] ** 2
            disc = b * b - c
            tc = -b - np.sqrt(np.maximum(disc, 0.0))
            hit = (disc >= 0) & (tc > 0)
            t = np.minimum(t, np.where(hit, tc, np.inf).min(axis=0))
    return t


def scan_points(world: World, poses: np.ndarray, beams: int, empties_per_beam: int,
                sigma: float, rng_noise: np.random.Generator,
                rng_empty: np.random.Generator) -> Tuple[np.ndarray, np.ndarray]:
    """Occupied beam end points then empty samples along the beams, pose by pose."""
    ang = 2.0 * np.pi * np.arange(beams) / beams
    dirs = np.stack([np.cos(ang), np.sin(ang)], axis=1)
    xs, ls = [], []
    for p in poses:
        r = raycast(world, p, ang) + rng_noise.normal(0.0, sigma, size=beams)
        r = np.maximum(r, 0.0)
        hits = p[None, :] + r[:, None] * dirs
        u = rng_empty.uniform(0.0, 1.0, size=(beams, empties_per_beam))
        emp = p[None, None, :] + (u * r[:, None])[:, :, None] * dirs[:, None, :]
        xs.append(hits)
        ls.append(np.ones(beams, dtype=np.uint8))
        xs.append(emp.reshape(-1, 2))
        ls.append(np.zeros(beams * empties_per_beam, dtype=np.uint8))
    return (np.concatenate(xs).astype(np.float32), np.concatenate(ls))


@dataclasses.dataclass
class Workload:
    name: str
    D: int
    ell: float
    theta: np.ndarray            # float64 [D][2], rad/m
    layout: Tuple[float, float, float, float]   # x0, y0, x1, y1 of the tile layout
    tiles: Tuple[int, int]
    grid: Tuple[float, float, float]            # x0, y0, res
    nx: int
    ny: int
    xy: np.ndarray               # float32 [n][2], world metres
    label: np.ndarray            # uint8 [n], 1 = occupied
    r_occ: int
    r_emp: int
    rho: float = 0.0
    poses: Optional[np.ndarray] = None

    @property
    def n(self) -> int:
        return int(self.xy.shape[0])

    def digest(self) -> Dict[str, str]:
        return {k: hashlib.sha256(np.ascontiguousarray(v).tobytes()).hexdigest()
                for k, v in (("theta", self.theta), ("xy", self.xy), ("label", self.label))}


@dataclasses.dataclass
class ScanRecipe:
    config_id: int
    name: str
    half: float
    n_rect: int
    n_circ: int
    rect_side: Tuple[float, float]
    circ_radius: Tuple[float, float]
    n_poses: int
    beams: int
    empties: int
    D: int
    ell: float
    tiles: Tuple[int, int]
    res: float
    nx: int
    ny: int
    r: int
    sigma: float = 0.02
    grid_origin: Optional[Tuple[float, float]] = None


# Workload recipes.  "toy_room" and "world40" are the plain-method configurations (a single
# 360-beam scan in a 12.8 m room; 50 scans of 1080 beams in a 40 m world at D = 8192);
# the small ones are multi-tile and ragged variants sized for the oracle.
RECIPES: Dict[str, ScanRecipe] = {
    "toy_room": ScanRecipe(1, "toy_room", 6.4, 6, 0, (0.5, 2.5), (0.25, 1.5), 1, 360, 5,
                           1024, 0.2, (1, 1), 0.1, 128, 128, 2),
    "world40": ScanRecipe(2, "world40", 20.0, 20, 20, (0.5, 4.0), (0.25, 1.5), 50, 1080, 10,
                          8192, 0.1, (4, 4), 0.05, 800, 800, 3),
    "world40_d1": ScanRecipe(2, "world40_d1", 20.0, 20, 20, (0.5, 4.0), (0.25, 1.5), 50, 1080, 10,
                             8192, 0.1, (1, 1), 0.05, 800, 800, 3),
    "mini4x4": ScanRecipe(11, "mini4x4", 8.0, 8, 6, (0.5, 2.0), (0.25, 1.0), 8, 360, 5,
                          2048, 0.2, (4, 4), 0.1, 160, 160, 3),
    "ragged3x3": ScanRecipe(12, "ragged3x3", 7.5, 6, 4, (0.5, 2.0), (0.25, 1.0), 5, 300, 4,
                            1000, 0.2, (3, 3), 0.1, 150, 130, 2, grid_origin=(-7.5, -6.5)),
}


def build(recipe: ScanRecipe) -> Workload:
    rt = rng_for(recipe.config_id, STREAM_THETA)
    theta = make_theta(recipe.D, recipe.ell, rt)
    rw = rng_for(recipe.config_id, STREAM_WORLD)
    start = np.zeros(2)
    world = make_world(recipe.half, recipe.n_rect, recipe.n_circ, recipe.rect_side,
                       recipe.circ_radius, start[None, :], 1.0, rw)
    if recipe.n_poses == 1:
        poses = start[None, :]
    else:
        poses = random_walk(world, recipe.n_poses, start, rng_for(recipe.config_id, STREAM_POSES))
    xy, label = scan_points(world, poses, recipe.beams, recipe.empties, recipe.sigma,
                            rng_for(recipe.config_id, STREAM_NOISE),
                            rng_for(recipe.config_id, STREAM_EMPTY))
    if recipe.grid_origin is None:
        gx0 = gy0 = -recipe.half
    else:
        gx0, gy0 = recipe.grid_origin
    layout = (gx0, gy0, gx0 + recipe.nx * recipe.res, gy0 + recipe.ny * recipe.res)
    return Workload(recipe.name, recipe.D, recipe.ell, theta, layout, recipe.tiles,
                    (gx0, gy0, recipe.res), recipe.nx, recipe.ny, xy, label,
                    recipe.r, recipe.r, 0.0, poses)


def workload(name: str) -> Workload:
    return build(RECIPES[name])


@dataclasses.dataclass
class MapSpec:
    D: int
    ell: float
    theta: np.ndarray
    tiles: Tuple[int, int]
    side: int                  # grid cells per axis
    res: float
    layout: Tuple[float, float, float, float]
    grid: Tuple[float, float, float]
    world: World


@dataclasses.dataclass
class UpdateRequest:
    map_id: int
    xy: np.ndarray
    label: np.ndarray
    arrival_s: float           # Poisson arrival offset (seconds) at unit rate


def serving_stream(n_maps: int = 16, n_requests: int = 256, config_id: int = 4,
                   beams=(360, 4320), empties: int = 10, grid_side=(64, 1024), res: float = 0.05,
                   dims=(2048, 4096, 8192), ell: float = 0.1, max_tiles: int = 4):
    """Maps of uneven size and a Poisson stream of lidar updates to random maps.

    Each map draws D from dims, tiles per axis from 1..max_tiles (1..max_tiles^2 regions) and a
    grid side log-uniform in grid_side rounded to a multiple of the tiles, at res m.  Its world
    is the grid's square with 2 + side/40 rectangles and circles.  Each request picks a map
    uniformly, a pose by a short random walk, a beam count log-uniform in beams and `empties`
    samples per beam; arrivals are exponential gaps of mean 1 (scale by 1/QPS)."""
    rr = rng_for(config_id, STREAM_REQUESTS)
    maps: List[MapSpec] = []
    for m in range(n_maps):
        D = int(rr.choice(dims))
        t = int(rr.integers(1, max_tiles + 1))
        side = int(round(math.exp(rr.uniform(math.log(grid_side[0]), math.log(grid_side[1])))))
        side = max(t, side - side % t)
        half = side * res / 2.0
        theta = make_theta(D, ell, rng_for(1000 + 16 * config_id + m, STREAM_THETA))
        nob = 2 + side // 40
        world = make_world(half, nob // 2 + 1, nob // 2, (0.3, min(4.0, half / 2)), (0.2, min(1.5, half / 4)),
                           np.zeros((1, 2)), min(1.0, half / 4), rr)
        maps.append(MapSpec(D, ell, theta, (t, t), side, res, (-half, -half, half, half),
                            (-half, -half, res), world))
    reqs: List[UpdateRequest] = []
    tnow = 0.0
    poses = [np.zeros(2) for _ in range(n_maps)]
    for _ in range(n_requests):
        m = int(rr.integers(0, n_maps))
        spec = maps[m]
        B = int(round(math.exp(rr.uniform(math.log(beams[0]), math.log(beams[1])))))
        step = rr.normal(0.0, 0.3 * spec.world.half / 4, size=2)
        p = np.clip(poses[m] + step, -0.8 * spec.world.half, 0.8 * spec.world.half)
        if _dist_to_obstacles(p, spec.world) > 0.2:
            poses[m] = p
        xy, lab = scan_points(spec.world, poses[m][None, :], B, empties, 0.02, rr, rr)
        tnow += float(rr.exponential(1.0))
        reqs.append(UpdateRequest(m, xy, lab, tnow))
    return maps, reqs


@dataclasses.dataclass
class StressScenario:
    """A large map updated in scan groups: one long random walk, an update every few poses."""
    name: str
    D: int
    ell: float
    theta: np.ndarray
    layout: Tuple[float, float, float, float]
    tiles: Tuple[int, int]
    grid: Tuple[float, float, float]
    nx: int
    ny: int
    r: int
    world: World
    poses: np.ndarray
    beams: int
    empties: int
    poses_per_update: int
    config_id: int
    sigma: float = 0.02

    @property
    def n_updates(self) -> int:
        return -(-len(self.poses) // self.poses_per_update)

    @property
    def points_per_update(self) -> int:
        return self.poses_per_update * self.beams * (1 + self.empties)

    def update(self, u: int) -> Tuple[np.ndarray, np.ndarray]:
        """(xy float32 [n][2], label uint8 [n]) of update u (its own noise and empty streams)."""
        ps = self.poses[u * self.poses_per_update:(u + 1) * self.poses_per_update]
        rn = np.random.default_rng(np.random.SeedSequence([2408, self.config_id, STREAM_NOISE, u]))
        re = np.random.default_rng(np.random.SeedSequence([2408, self.config_id, STREAM_EMPTY, u]))
        return scan_points(self.world, ps, self.beams, self.empties, self.sigma, rn, re)

    def updates(self, limit: Optional[int] = None, workers: int = 1) -> List[Tuple[np.ndarray, np.ndarray]]:
        """The first `limit` updates in walk order, generated by `workers` processes."""
        n = self.n_updates if limit is None else min(limit, self.n_updates)
        if workers <= 1 or n <= 1:
            return [self.update(u) for u in range(n)]
        import multiprocessing as mp
        with mp.get_context("fork").Pool(min(workers, n)) as pool:
            return pool.map(self.update, range(n), chunksize=1)


def stress_scenario(n_poses: int = 2000, config_id: int = 5) -> StressScenario:
    """200 m square world, 200 rectangles + 200 circles, 1080 beams and 10 empties per beam,
    D = 16384, l = 0.1 m, 16 x 16 tiles, a 4000 x 4000 grid at 0.05 m, r = 3, and one update per
    10 poses (118 800 points)."""
    half, D, ell = 100.0, 16384, 0.1
    theta = make_theta(D, ell, rng_for(config_id, STREAM_THETA))
    start = np.zeros(2)
    world = make_world(half, 200, 200, (0.5, 4.0), (0.25, 1.5), start[None, :], 1.0,
                       rng_for(config_id, STREAM_WORLD))
    poses = random_walk(world, n_poses, start, rng_for(config_id, STREAM_POSES))
    return StressScenario("stress200", D, ell, theta, (-half, -half, half, half), (16, 16),
                          (-half, -half, 0.05), 4000, 4000, 3, world, poses, 1080, 10, 10, config_id)


# ---- three dimensions -------------------------------------------------------------------

def make_theta3(D: int, ell: float, rng: np.random.Generator) -> np.ndarray:
    """Conjugate-symmetric phase basis for three axes, float64 [D][3] in rad/m."""
    if D < 4 or D % 2:
        raise ValueError("D must be even and >= 4")
    h = D // 2
    th = np.zeros((D, 3), dtype=np.float64)
    ph = rng.uniform(-np.pi, np.pi, size=(h - 1, 3))
    th[1:h] = ph
    th[h + 1:] = -ph[::-1]
    return th / float(ell)


@dataclasses.dataclass
class World3:
    half: Tuple[float, float, float]   # the room is [-hx, hx] x [-hy, hy] x [0, 2 hz]; walls, floor, ceiling
    boxes: np.ndarray                  # [nb][6] xmin, ymin, zmin, xmax, ymax, zmax


def raycast3(world: World3, pose: np.ndarray, dirs: np.ndarray) -> np.ndarray:
    """Exact range from pose along each unit direction to the first wall, floor, ceiling or box."""
    lo = np.array([-world.half[0], -world.half[1], 0.0])
    hi = np.array([world.half[0], world.half[1], 2.0 * world.half[2]])
    with np.errstate(divide="ignore", invalid="ignore"):
        tb = np.where(dirs > 0, (hi - pose) / dirs, np.where(dirs < 0, (lo - pose) / dirs, np.inf))
        t = tb.min(axis=1)
        for b in world.boxes:
            t1 = np.where(dirs != 0, (b[:3] - pose) / dirs, np.where(pose >= b[:3], -np.inf, np.inf))
            t2 = np.where(dirs != 0, (b[3:] - pose) / dirs, np.where(pose <= b[3:], np.inf, -np.inf))
            tmin = np.minimum(t1, t2).max(axis=1)
            tmax = np.maximum(t1, t2).min(axis=1)
            hit = (tmax >= tmin) & (tmin > 0)
            t = np.where(hit & (tmin < t), tmin, t)
    return t


def sphere_directions(n: int) -> np.ndarray:
    """n near-uniform unit directions (Fibonacci sphere)."""
    i = np.arange(n) + 0.5
    z = 1.0 - 2.0 * i / n
    r = np.sqrt(np.maximum(0.0, 1.0 - z * z))
    a = np.pi * (3.0 - np.sqrt(5.0)) * i
    return np.stack([r * np.cos(a), r * np.sin(a), z], axis=1)


@dataclasses.dataclass
class Volume:
    name: str
    D: int
    ell: float
    theta: np.ndarray                                # float64 [D][3]
    layout: Tuple[float, float, float, float, float, float]
    tiles: Tuple[int, int, int]
    grid: Tuple[float, float, float, float]          # x0, y0, z0, res
    nx: int
    ny: int
    nz: int
    xyz: np.ndarray                                  # float32 [n][3]
    label: np.ndarray                                # uint8 [n]
    r_occ: int
    r_emp: int
    rho: float = 0.0

    @property
    def n(self) -> int:
        return int(self.xyz.shape[0])


@dataclasses.dataclass
class VolumeRecipe:
    config_id: int
    name: str
    half: Tuple[float, float, float]
    n_boxes: int
    box_side: Tuple[float, float]
    n_poses: int
    beams: int
    empties: int
    D: int
    ell: float
    tiles: Tuple[int, int, int]
    res: float
    r: int
    sigma: float = 0.02


# "room3d" is small enough for the FP64 oracle over every voxel; "hall3d" is the 3-D benchmark.
VOLUME_RECIPES: Dict[str, VolumeRecipe] = {
    "room3d": VolumeRecipe(31, "room3d", (3.2, 3.2, 1.6), 5, (0.4, 1.2), 3, 600, 3, 512, 0.3,
                           (2, 2, 1), 0.2, 1),
    "hall3d": VolumeRecipe(32, "hall3d", (6.4, 6.4, 1.6), 24, (0.4, 1.6), 20, 4000, 5, 4096, 0.2,
                           (2, 2, 1), 0.1, 2),
}


def volume(name: str, **changes) -> Volume:
    """A recipe's volume; keyword arguments replace recipe fields (e.g. D, ell, tiles)."""
    rc = dataclasses.replace(VOLUME_RECIPES[name], **changes)
    theta = make_theta3(rc.D, rc.ell, rng_for(rc.config_id, STREAM_THETA))
    rw = rng_for(rc.config_id, STREAM_WORLD)
    hx, hy, hz = rc.half
    boxes = []
    while len(boxes) < rc.n_boxes:
        s = rw.uniform(rc.box_side[0], rc.box_side[1], size=3)
        c = np.array([rw.uniform(-hx + s[0] / 2, hx - s[0] / 2), rw.uniform(-hy + s[1] / 2, hy - s[1] / 2),
                      s[2] / 2])  # standing on the floor
        b = np.r_[c - s / 2, c + s / 2]
        if np.all(np.abs(c[:2]) > 0.0) and not (b[0] < 0.8 and b[3] > -0.8 and b[1] < 0.8 and b[4] > -0.8):
            boxes.append(b)   # keeps the centre column clear for the sensor
    world = World3((hx, hy, hz), np.array(boxes, dtype=np.float64).reshape(-1, 6))
    rp = rng_for(rc.config_id, STREAM_POSES)
    poses = []
    for _ in range(rc.n_poses):
        while True:
            q = np.array([rp.uniform(-hx + 0.5, hx - 0.5), rp.uniform(-hy + 0.5, hy - 0.5), rp.uniform(0.8, 1.4)])
            inside = any(np.all(q >= b[:3] - 0.3) and np.all(q <= b[3:] + 0.3) for b in world.boxes)
            if not inside:
                poses.append(q)
                break
    dirs = sphere_directions(rc.beams)
    rn, re = rng_for(rc.config_id, STREAM_NOISE), rng_for(rc.config_id, STREAM_EMPTY)
    xs, ls = [], []
    for q in poses:
        r = np.maximum(raycast3(world, q, dirs) + rn.normal(0.0, rc.sigma, size=rc.beams), 0.0)
        xs.append(q[None, :] + r[:, None] * dirs)
        ls.append(np.ones(rc.beams, np.uint8))
        u = re.uniform(0.0, 1.0, size=(rc.beams, rc.empties))
        xs.append((q[None, None, :] + (u * r[:, None])[:, :, None] * dirs[:, None, :]).reshape(-1, 3))
        ls.append(np.zeros(rc.beams * rc.empties, np.uint8))
    xyz = np.concatenate(xs).astype(np.float32)
    label = np.concatenate(ls)
    nx, ny, nz = int(round(2 * hx / rc.res)), int(round(2 * hy / rc.res)), int(round(2 * hz / rc.res))
    layout = (-hx, -hy, 0.0, hx, hy, 2 * hz)
    return Volume(rc.name, rc.D, rc.ell, theta, layout, rc.tiles, (-hx, -hy, 0.0, rc.res), nx, ny, nz,
                  xyz, label, rc.r, rc.r)
