"""Seeded synthetic inputs for the direct-summation linking-number path.

This module builds geometry only: closed polylines stored as a vertex array
``xyz[V, 3]`` plus loop offsets ``offsets[L + 1]`` (loop ``l`` owns vertices
``offsets[l] .. offsets[l+1]-1``; segment ``s`` joins vertex ``s`` to ``s+1``
cyclically, the first vertex is not repeated).  It evaluates no linking
number: the expected values it returns come from how each shape is built
(which ring passes through which, how many clasps a knit row has, how many
turns a companion curve winds), and the test suite checks those construction
rules against the oracle on small instances.  Both the HIP path and the oracle
are fed from here; this module imports neither.

The workloads stand in for the paper's inputs (Sec. 6, Table 1): a small ring
grid, a 4-in-1 chainmail sheet (the paper's chainmail rows), knit-like tubes of
closed yarn rows made from periodic cubic B-splines (the paper's StitchMesh
yarn models, which are not available), and long winding curve pairs (the
paper's ribbon / woundball stress tests).  None of them reproduces a dataset.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


@dataclass
class LoopSet:
    """Closed polylines plus the linking numbers their construction implies.

    ``exp_pairs``/``exp_lk``: every loop pair whose construction gives a
    non-zero linking number, sorted lexicographically with i < j; every other
    pair is expected to be 0.  ``pairs`` is a candidate pair list when the
    generator knows one (otherwise the caller runs the potential link search).
    """

    xyz: np.ndarray
    offsets: np.ndarray
    exp_pairs: np.ndarray
    exp_lk: np.ndarray
    name: str = ""
    seed: int = 0
    pairs: np.ndarray | None = None
    meta: dict = field(default_factory=dict)

    @property
    def n_loops(self) -> int:
        return int(self.offsets.shape[0] - 1)

    @property
    def sizes(self) -> np.ndarray:
        return np.diff(self.offsets)

    def loop(self, i: int) -> np.ndarray:
        return self.xyz[self.offsets[i]:self.offsets[i + 1]]

    def expected_for(self, pairs: np.ndarray) -> np.ndarray:
        """Expected integer for each row of ``pairs`` (0 where not listed)."""
        pairs = np.asarray(pairs, dtype=np.int64).reshape(-1, 2)
        L = self.n_loops
        out = np.zeros(pairs.shape[0], dtype=np.int32)
        if self.exp_pairs.shape[0] == 0 or pairs.shape[0] == 0:
            return out
        ek = self.exp_pairs[:, 0].astype(np.int64) * L + self.exp_pairs[:, 1]
        qk = pairs[:, 0] * L + pairs[:, 1]
        pos = np.searchsorted(ek, qk)
        pos = np.minimum(pos, ek.shape[0] - 1)
        hit = ek[pos] == qk
        out[hit] = self.exp_lk[pos[hit]]
        return out


def terms(sizes: np.ndarray, pairs: np.ndarray) -> int:
    """Number of segment-pair terms of a pair list: sum over pairs of N_a * N_b."""
    pairs = np.asarray(pairs, dtype=np.int64).reshape(-1, 2)
    s = np.asarray(sizes, dtype=np.int64)
    return int(np.sum(s[pairs[:, 0]] * s[pairs[:, 1]]))


def _pack(loops, dtype, exp, name, seed, pairs=None, meta=None) -> LoopSet:
    sizes = np.array([len(x) for x in loops], dtype=np.int64)
    off = np.zeros(len(loops) + 1, dtype=np.int64)
    off[1:] = np.cumsum(sizes)
    xyz = np.ascontiguousarray(np.concatenate(loops, axis=0).astype(dtype))
    if exp:
        items = sorted((min(i, j), max(i, j), v) for (i, j), v in exp.items() if v != 0)
        ep = np.array([[a, b] for a, b, _ in items], dtype=np.int32).reshape(-1, 2)
        ev = np.array([v for _, _, v in items], dtype=np.int32)
    else:
        ep = np.zeros((0, 2), dtype=np.int32)
        ev = np.zeros(0, dtype=np.int32)
    return LoopSet(xyz, off, ep, ev, name, seed, pairs, dict(meta or {}))


# ----------------------------------------------------------------- rotations
def rot_x(a):
    c, s = np.cos(a), np.sin(a)
    return np.array([[1, 0, 0], [0, c, -s], [0, s, c]])


def rot_y(a):
    c, s = np.cos(a), np.sin(a)
    return np.array([[c, 0, s], [0, 1, 0], [-s, 0, c]])


def rot_z(a):
    c, s = np.cos(a), np.sin(a)
    return np.array([[c, -s, 0], [s, c, 0], [0, 0, 1]])


def rot_axis(axis, a):
    """Rodrigues rotation by angle ``a`` about unit vector ``axis``."""
    k = np.asarray(axis, dtype=np.float64)
    k = k / np.linalg.norm(k)
    K = np.array([[0, -k[2], k[1]], [k[2], 0, -k[0]], [-k[1], k[0], 0]])
    return np.eye(3) + np.sin(a) * K + (1 - np.cos(a)) * (K @ K)


def random_rotation(rng) -> np.ndarray:
    """Uniform random proper rotation (QR of a Gaussian matrix)."""
    q, r = np.linalg.qr(rng.standard_normal((3, 3)))
    q = q * np.sign(np.diag(r))
    if np.linalg.det(q) < 0:
        q[:, 0] = -q[:, 0]
    return q


def circle(n: int, radius: float = 1.0) -> np.ndarray:
    t = 2 * np.pi * np.arange(n) / n
    return np.stack([radius * np.cos(t), radius * np.sin(t), np.zeros(n)], axis=1)


# ----------------------------------------------------------- closed-form pins
def hopf(n: int = 64, dtype=np.float64) -> LoopSet:
    """Two unit circles, A in the xy plane and B in the xz plane through A's
    centre region: A = (cos t, sin t, 0), B = (1 + cos t, 0, sin t).
    With these orientations the pair (A, B) has linking number -1."""
    t = 2 * np.pi * np.arange(n) / n
    A = np.stack([np.cos(t), np.sin(t), 0 * t], 1)
    B = np.stack([1 + np.cos(t), 0 * t, np.sin(t)], 1)
    return _pack([A, B], dtype, {(0, 1): -1}, "hopf", 0, np.array([[0, 1]], np.int32))


def torus_link(m: int, n: int, N: int = 400, dtype=np.float64) -> LoopSet:
    """Torus link: A winds m times toroidally and once poloidally on a torus of
    radii (3, 0.3); B winds once toroidally and n times poloidally on a torus of
    radii (3, 0.8).  Linking number -m*n for these orientations (the magnitude
    is the product rule the paper states for its torus stress test)."""
    t = 2 * np.pi * np.arange(N) / N
    A = np.stack([(3 + 0.3 * np.cos(t)) * np.cos(m * t), (3 + 0.3 * np.cos(t)) * np.sin(m * t),
                  0.3 * np.sin(t)], 1)
    B = np.stack([(3 + 0.8 * np.cos(n * t)) * np.cos(t), (3 + 0.8 * np.cos(n * t)) * np.sin(t),
                  0.8 * np.sin(n * t)], 1)
    return _pack([A, B], dtype, {(0, 1): -m * n}, "torus_%d_%d" % (m, n), 0,
                  np.array([[0, 1]], np.int32))


# ---------------------------------------------- near the singularities of Eq. 4
def _ngon(n: int, radius: float) -> np.ndarray:
    """Regular n-gon in the xy plane with vertices at angles (2k + 1) pi / n,
    so that its last segment (vertex n-1 -> vertex 0) is parallel to +y at
    x = radius cos(pi / n) and crosses the x axis at its midpoint."""
    t = np.pi * (2 * np.arange(n) + 1) / n
    return np.stack([radius * np.cos(t), radius * np.sin(t), np.zeros(n)], axis=1)


def near_contact(h_rel, t_a, t_b, seed: int = 0, offset: float = 0.0, n_a: int = 32,
                 n_b: int = 24, r_b: float = 0.6, rotate: bool = True, spacing: float = 10.0,
                 dtype=np.float64) -> LoopSet:
    """Loop pairs that pass within a prescribed distance of each other (Sec. 4.1:
    Eq. 4 is singular only where two segments touch).

    Case k (one entry of each of ``h_rel``, ``t_a``, ``t_b``): A is a unit
    n_a-gon in the xy plane, shifted along y so that its last segment (length
    s_a, parallel to +y) crosses the x axis at fraction t_a of its length; B is
    an n_b-gon of radius r_b in the xz plane, centred on the x axis and shifted
    along z so that its last segment (parallel to +z) crosses the x axis at
    fraction t_b, at distance h = h_rel[k] * s_a beyond A's segment.  The two
    segments are perpendicular and their closest points are h apart; no other
    segments come near.  B's opposite side crosses A's plane inside A, so for
    h > 0 B passes once through A's disk (linking number -1 for these
    orientations, as in :func:`hopf`) and for h < 0 twice in opposite
    directions (0).  Each case gets its own seeded rotation (``rotate``), is
    moved ``spacing`` along x from the previous one (0: all cases share one
    centre; the pair list keeps them apart) and the whole set by ``offset``
    along (1, 1, 1)/sqrt(3).  ``pairs`` lists (2k, 2k + 1); ``meta["h"]`` the
    distances h before rounding to ``dtype``.
    """
    h_rel, t_a, t_b = (np.atleast_1d(np.asarray(v, dtype=np.float64)) for v in (h_rel, t_a, t_b))
    h_rel, t_a, t_b = np.broadcast_arrays(h_rel, t_a, t_b)
    rng = np.random.default_rng(seed)
    A0 = _ngon(n_a, 1.0)
    s_a = 2.0 * np.sin(np.pi / n_a)
    x_a = np.cos(np.pi / n_a)
    B0 = _ngon(n_b, r_b)[:, [0, 2, 1]]  # into the xz plane, last segment along +z
    s_b = 2.0 * r_b * np.sin(np.pi / n_b)
    x_b = r_b * np.cos(np.pi / n_b)
    shift = offset * np.ones(3) / np.sqrt(3.0)
    loops, exp, hs = [], {}, []
    for k in range(h_rel.shape[0]):
        h = float(h_rel[k]) * s_a
        A = A0 + np.array([0.0, s_a * (0.5 - t_a[k]), 0.0])
        B = B0 + np.array([x_a + h - x_b, 0.0, s_b * (0.5 - t_b[k])])
        R = random_rotation(rng) if rotate else np.eye(3)
        c = np.array([spacing * k, 0.0, 0.0]) + shift
        loops += [A @ R.T + c, B @ R.T + c]
        if h > 0:
            exp[(2 * k, 2 * k + 1)] = -1
        hs.append(h)
    pairs = np.array([[2 * k, 2 * k + 1] for k in range(h_rel.shape[0])], np.int32).reshape(-1, 2)
    return _pack(loops, dtype, exp, "near_contact", seed, pairs,
                 meta={"h": np.array(hs), "s_a": s_a})


def near_parallel(h_rel, alpha, seed: int = 0, offset: float = 0.0, per_edge: int = 8,
                  rotate: bool = True, spacing: float = 10.0, dtype=np.float64) -> LoopSet:
    """Linked square loops with a pair of long, nearly parallel sides close
    together (the other end of Sec. 4.1's conditioning: segment pairs whose
    s_j x s_i nearly vanishes next to a near contact).

    Case k, with h = h_rel[k] (in units of the side): A is the unit square
    [0, 1]^2 in the xy plane; B is a 1 x 1 square in the plane y = h, spanning
    x in [-0.5, 0.5] and z in [-1 + h, h], turned by alpha[k] radians about
    the z axis through (0, h, h) (alpha[k] > -2 h keeps B's side x = 0.5 above
    y = 0).  B's top side then runs over A's side y = 0
    at distance about h sqrt(2), nearly parallel to it over half its length,
    and B's side x = 0.5 crosses A's plane inside A at distance about h from
    that side.  B's side x = -0.5 crosses A's plane outside A, so the pair
    links once (-1 for these orientations).  Each side has ``per_edge``
    segments.  Rotation, spacing and ``offset`` as in :func:`near_contact`.
    """
    h_rel, alpha = (np.atleast_1d(np.asarray(v, dtype=np.float64)) for v in (h_rel, alpha))
    h_rel, alpha = np.broadcast_arrays(h_rel, alpha)
    rng = np.random.default_rng(seed)
    u = np.arange(per_edge) / per_edge

    def square(p0, e1, e2):
        pts = [p0 + np.outer(u, e1), p0 + e1 + np.outer(u, e2), p0 + e1 + e2 - np.outer(u, e1),
               p0 + e2 - np.outer(u, e2)]
        return np.concatenate(pts, axis=0)

    ex, ey, ez = np.eye(3)
    A0 = square(np.zeros(3), ex, ey)
    shift = offset * np.ones(3) / np.sqrt(3.0)
    loops, exp = [], {}
    for k in range(h_rel.shape[0]):
        h = float(h_rel[k])
        piv = np.array([0.0, h, h])
        B = square(np.array([-0.5, h, h]), ex, -ez)
        B = (B - piv) @ rot_z(float(alpha[k])).T + piv
        R = random_rotation(rng) if rotate else np.eye(3)
        c = np.array([spacing * k, 0.0, 0.0]) + shift
        loops += [A0 @ R.T + c, B @ R.T + c]
        exp[(2 * k, 2 * k + 1)] = -1
    pairs = np.array([[2 * k, 2 * k + 1] for k in range(h_rel.shape[0])], np.int32).reshape(-1, 2)
    return _pack(loops, dtype, exp, "near_parallel", seed, pairs, meta={"h": h_rel.copy()})


# ------------------------------------------------------------- ring grid (C1)
def ring_grid(seed: int = 0, rows: int = 8, cols: int = 8, nseg: int = 32, spacing: float = 1.6,
              jitter: float = 0.02, dtype=np.float64) -> LoopSet:
    """Grid of unit rings, ring (r, c) centred at (spacing*c, spacing*r, 0).

    Rings with r + c even lie flat (xy plane); rings with r + c odd are turned
    +90 degrees about x ((x, y, z) -> (x, -z, y)) so that every horizontal
    neighbour pair is a Hopf-like link (checkerboard alternation).  Every
    coordinate gets seeded uniform jitter in [-jitter, jitter].  Horizontal
    pairs link with -1 when the flat ring is the left one and +1 when the
    turned ring is; flat diagonal neighbours overlap in their boxes but are
    not linked.
    """
    rng = np.random.default_rng(seed)
    base = circle(nseg)
    turn = np.array([[1, 0, 0], [0, 0, -1], [0, 1, 0]], dtype=np.float64)
    loops = []
    for r in range(rows):
        for c in range(cols):
            P = base @ turn.T if (r + c) % 2 else base.copy()
            P = P + np.array([spacing * c, spacing * r, 0.0])
            P = P + rng.uniform(-jitter, jitter, size=P.shape)
            loops.append(P)
    exp = {}
    for r in range(rows):
        for c in range(cols - 1):
            i, j = r * cols + c, r * cols + c + 1
            exp[(i, j)] = -1 if (r + c) % 2 == 0 else 1
    return _pack(loops, dtype, exp, "ring_grid", seed,
                 meta={"rows": rows, "cols": cols, "nseg": nseg})


# -------------------------------------------------------- 4-in-1 chainmail (C2)
def chainmail(seed: int = 0, rows: int = 100, cols: int = 140, nseg: int = 64,
              spacing: float = 1.1, tilt_deg: float = 40.0, sheet_deg: float = 45.0,
              row_pitch: float | None = None,
              wobble_deg: float = 5.0, sigma: float = 0.01, dtype=np.float32,
              pulled_rings=None, noise_seed: int | None = None) -> LoopSet:
    """European 4-in-1 chainmail sheet of unit rings.

    Ring (r, c) is centred at ((c + (r mod 2)/2) * spacing, r * spacing, 0) and
    tilted by +tilt about y on even rows and -tilt on odd rows, so that each
    ring passes through two rings of the row above and two of the row below.
    The sheet is turned by ``sheet_deg`` about z (this only enlarges the axis-
    aligned boxes, adding unlinked candidate pairs), then every ring is turned
    about its centre by a seeded angle in [0, wobble] about a random axis and
    every coordinate gets Gaussian noise of standard deviation ``sigma``.

    Construction rule for the linking numbers (ring index r * cols + c): ring
    (r, c) links ring (r+1, c) and ring (r+1, c - 1 + 2 (r mod 2)); the pair has
    +1 when r is even and -1 when r is odd, all other pairs 0.

    ``pulled_rings``: ring indices of the first or last row to pull out of the
    sheet: each slides rigidly outwards in its own plane (away from the
    sheet, parallel to its same-row neighbours) through the wires of the two
    rings it hangs from, until it clears them by 0.4; both of its links become
    0 and no other pair changes.  ``meta["pulled"]`` lists the changed pairs.
    ``noise_seed``: seed of the per-vertex noise (default ``seed``), so that
    timesteps of one sheet share its structure and differ in the noise.
    """
    rng = np.random.default_rng(seed)
    base = circle(nseg)
    Rs = rot_z(np.deg2rad(sheet_deg))
    centres, frames = [], []
    for r in range(rows):
        for c in range(cols):
            ctr = np.array([(c + 0.5 * (r % 2)) * spacing, r * (row_pitch or spacing), 0.0])
            R = rot_y(np.deg2rad(tilt_deg if r % 2 == 0 else -tilt_deg))
            centres.append(Rs @ ctr)
            frames.append(Rs @ R)
    centres = np.array(centres)
    frames = np.array(frames)
    L = rows * cols
    axes = rng.standard_normal((L, 3))
    angs = np.deg2rad(rng.uniform(0.0, wobble_deg, size=L))
    exp = {}
    for r in range(rows - 1):
        for c in range(cols):
            for cc in (c, c - 1 + 2 * (r % 2)):
                if 0 <= cc < cols:
                    exp[(r * cols + c, (r + 1) * cols + cc)] = 1 if r % 2 == 0 else -1
    keys = sorted(exp)
    local = [base.copy() for _ in range(L)]
    shift = np.zeros((L, 3))
    changed = []
    if pulled_rings is not None:
        out_dir = Rs @ np.array([0.0, 1.0, 0.0])
        for b in sorted(set(int(x) for x in pulled_rings)):
            r, c = divmod(b, cols)
            if r not in (0, rows - 1) or rows < 2:
                continue  # only edge rings can slide out of the sheet
            partners = [i for (i, j) in keys if j == b] + [j for (i, j) in keys if i == b]
            near = np.nonzero(np.linalg.norm(centres - centres[b], axis=1) < 4.5)[0]
            others = [int(x) for x in near if x != b and x not in partners]
            d = _slide_out(local[b], centres[b], frames[b], partners, others, centres, frames,
                           out_dir if r == rows - 1 else -out_dir)
            if d is None:
                continue
            shift[b] = d
            for q in partners:
                key = (min(b, q), max(b, q))
                exp[key] = 0
                changed.append(key)
    nrng = rng if noise_seed is None else np.random.default_rng(noise_seed)
    loops = []
    for l in range(L):
        W = rot_axis(axes[l], angs[l]) @ frames[l]
        P = local[l] @ W.T + centres[l] + shift[l]
        P = P + nrng.normal(0.0, sigma, size=P.shape)
        loops.append(P)
    return _pack(loops, dtype, exp, "chainmail", seed,
                 meta={"rows": rows, "cols": cols, "nseg": nseg, "sigma": sigma,
                       "pulled": np.array(sorted(changed), np.int32).reshape(-1, 2)})


def _circle_distance(P, c, n):
    """Distance from points P to the unit circle with centre c and normal n."""
    d = P - c
    h = d @ n
    r = np.linalg.norm(d - np.outer(h, n), axis=1)
    return np.sqrt(h * h + (r - 1.0) ** 2)


def _disk_crossings_signed(world, ca, na):
    """Signed count of the closed polyline's crossings of the unit disk
    (centre ca, normal na), and the smallest |radius - 1| of any crossing of
    the disk's plane (how close a crossing comes to the rim)."""
    n = world.shape[0]
    h = (world - ca) @ na
    h1 = np.roll(h, -1)
    idx = np.nonzero(h * h1 < 0)[0]
    if idx.size == 0:
        return 0, np.inf
    t = h[idx] / (h[idx] - h1[idx])
    p = world[idx] + t[:, None] * (np.roll(world, -1, 0)[idx] - world[idx])
    q = p - ca
    rr = np.linalg.norm(q - np.outer(q @ na, na), axis=1)
    inside = rr < 1.0
    sign = np.where(h1[idx] > h[idx], 1, -1)
    return int(np.sum(sign[inside])), float(np.min(np.abs(rr - 1.0)))


def _slide_out(local_b, cb, Fb, partners, others, centres, frames, direction, keep=0.4):
    """Slide ring B rigidly along `direction` (in its own plane) until it no
    longer crosses the disks of its `partners` and stays `keep` away from them
    and from every ring in `others`.  Returns the offset, or None."""
    world = local_b @ Fb.T + cb
    for dist in np.arange(0.5, 3.01, 0.1):
        W = world + dist * direction
        ok = True
        for c in partners:
            k, rim = _disk_crossings_signed(W, centres[c], frames[c][:, 2])
            if k != 0 or rim < 0.1 or _circle_distance(W, centres[c], frames[c][:, 2]).min() < keep:
                ok = False
                break
        if ok:
            for c in others:
                if _circle_distance(W, centres[c], frames[c][:, 2]).min() < keep:
                    ok = False
                    break
        if ok:
            return dist * direction
    return None


# ------------------------------------------------------------- knit tubes (C3)
def bspline_closed(P: np.ndarray, per_span: int) -> np.ndarray:
    """Uniform periodic cubic B-spline through control polygon P (closed),
    sampled at ``per_span`` uniform parameter steps per span."""
    n = P.shape[0]
    t = np.arange(per_span, dtype=np.float64) / per_span
    b0 = (1 - t) ** 3 / 6
    b1 = (3 * t ** 3 - 6 * t ** 2 + 4) / 6
    b2 = (-3 * t ** 3 + 3 * t ** 2 + 3 * t + 1) / 6
    b3 = t ** 3 / 6
    idx = np.arange(n)
    out = (b0[None, :, None] * P[(idx - 1) % n][:, None, :] + b1[None, :, None] * P[idx][:, None, :]
           + b2[None, :, None] * P[(idx + 1) % n][:, None, :]
           + b3[None, :, None] * P[(idx + 2) % n][:, None, :])
    return out.reshape(n * per_span, 3)


_KNIT_D = 1.5      # depth of a stitch dip below the row's baseline (row pitch 1)
_KNIT_DELTA = 0.45  # radial weave of a dip's two legs
_KNIT_RMIN = 1.5


def knit_row_controls(stitches: int, row: int, radius: float, signs) -> np.ndarray:
    """Control polygon (4 points per stitch) of one closed yarn row of a tube.

    The row runs once around the tube axis (z) at height ``row``.  At each
    stitch it dips down below the previous row's baseline; the dip's two legs
    sit at radius +-DELTA around the tube radius, so the dip clasps the row
    below.  ``signs[s]`` = +1 puts the descending leg outside, -1 inside;
    stitches of consecutive rows are staggered by half a stitch.
    """
    dphi = 2 * np.pi / stitches
    pts = []
    for s in range(stitches):
        ph = (s + 0.5 * (row % 2)) * dphi
        sg = float(signs[s])
        for f, dz, dr in ((-0.25, 0.0, 0.0), (-0.09, -_KNIT_D, sg * _KNIT_DELTA),
                          (0.09, -_KNIT_D, -sg * _KNIT_DELTA), (0.25, 0.0, 0.0)):
            phi = ph + f * dphi
            rho = radius + dr
            pts.append([rho * np.cos(phi), rho * np.sin(phi), row + dz])
    return np.array(pts)


def knit_tube(stitches: int, rows: int, per_span: int = 32, pattern: str = "alternating",
              rng=None, flip: set | None = None) -> tuple[list, dict]:
    """Rows of one knit-like tube (local frame, axis z) and their links.

    Construction rule: rows r-1 and r link with the sum of row r's clasp signs
    (a clasp with its descending leg outside counts +1).  ``alternating``
    (the stockinette-like default) alternates the signs, so an even stitch
    count links 0; ``uniform`` makes every sign +1 (linking number = stitch
    count).  ``flip``: set of (row, stitch) clasps whose sign is reversed.
    ``per_span`` = 0 returns the control polygons themselves (the spline
    input of a discretizer) instead of uniform samples.
    """
    radius = max(stitches / (2 * np.pi), _KNIT_RMIN)
    loops, exp = [], {}
    for r in range(rows):
        if pattern == "uniform":
            sg = np.ones(stitches)
        else:
            sg = np.array([(-1.0) ** s for s in range(stitches)])
        if flip:
            for s in range(stitches):
                if (r, s) in flip:
                    sg[s] = -sg[s]
        ctrl = knit_row_controls(stitches, r, radius, sg)
        loops.append(bspline_closed(ctrl, per_span) if per_span > 0 else ctrl)
        if r > 0:
            exp[(r - 1, r)] = int(round(sg.sum()))
    return loops, exp


def knit(seed: int = 0, n_loops: int = 2000, cp_min: int = 16, cp_max: int = 512,
         rows_min: int = 5, rows_max: int = 20, per_span: int = 32, linked_fraction: float = 0.2,
         tilt_deg: float = 35.0, gap: float = 0.3, dtype=np.float32, sigma: float = 0.0,
         pull=None, noise_seed: int | None = None) -> LoopSet:
    """Knit-like tubes of closed periodic cubic B-spline yarn rows.

    Each tube has a log-uniform control-point count per row in [cp_min, cp_max]
    (4 per stitch, an even stitch count) and 5-20 rows; rows are discretised
    uniformly at ``per_span`` segments per span, so row sizes are very uneven.
    Tubes are stockinette-like (alternating clasps, linking 0 between rows,
    the paper's observation for stitch rows) except for a seeded
    ``linked_fraction`` that use the uniform clasp pattern (linking number =
    stitch count between consecutive rows).  Every tube is turned by a seeded
    rotation of up to ``tilt_deg`` off vertical and tubes are packed in a grid
    whose bounding spheres are ``gap`` apart, so axis-aligned boxes of rows of
    the same and of neighbouring tubes overlap without the curves coming close.

    ``pull``: global loop indices of rows whose first clasp is pulled through
    (its sign reversed), which changes the row's linking number with the row
    below by -2 times the clasp's sign; the expected values include the change.
    ``per_span`` = 0: each row is its control polygon (closed uniform cubic
    B-spline control points, for a discretizer); the rotation and placement
    are affine, so they map the spline of the polygon to the spline of the
    mapped polygon.
    ``sigma``: per-vertex Gaussian noise added after construction (seeded by
    ``noise_seed``, default ``seed``); keep it well below the 0.13 clearance
    between clasping rows.
    """
    rng = np.random.default_rng(seed)
    tubes = []
    total = 0
    while total < n_loops:
        nr = int(rng.integers(rows_min, rows_max + 1))
        nr = min(nr, n_loops - total)
        if nr < 2:
            nr = 2
        cp = float(np.exp(rng.uniform(np.log(cp_min), np.log(cp_max))))
        stitches = max(4, 2 * int(round(cp / 8.0)))
        stitches = min(stitches, cp_max // 4)
        pattern = "uniform" if rng.uniform() < linked_fraction else "alternating"
        tubes.append((stitches, nr, pattern))
        total += nr
    loops, exp = [], {}
    # bounding sphere per tube, placed on a square grid (largest first)
    order = sorted(range(len(tubes)), key=lambda t: -tubes[t][0])
    radii = []
    for t in range(len(tubes)):
        st, nr, _ = tubes[t]
        rad = max(st / (2 * np.pi), _KNIT_RMIN) + _KNIT_DELTA + 0.5
        radii.append(float(np.hypot(rad, 0.5 * (nr + _KNIT_D))))
    side = int(np.ceil(np.sqrt(len(tubes))))
    place = {}
    cursor_y = 0.0
    k = 0
    while k < len(order):
        rowt = order[k:k + side]
        h = max(radii[t] for t in rowt)
        x = 0.0
        for t in rowt:
            x += radii[t]
            place[t] = np.array([x, cursor_y + h, 0.0])
            x += radii[t] + gap
        cursor_y += 2 * h + gap
        k += side
    pull = set(int(x) for x in (pull or ()))
    for t in range(len(tubes)):
        st, nr, pattern = tubes[t]
        first = sum(tubes[u][1] for u in range(t))
        flips = {(g - first, 0) for g in pull if first < g < first + nr}
        rows, e = knit_tube(st, nr, per_span, pattern, flip=flips or None)
        axis = rng.standard_normal(3)
        axis[2] = 0.0
        Rt = rot_axis(axis, np.deg2rad(rng.uniform(0.0, tilt_deg))) @ rot_z(rng.uniform(0, 2 * np.pi))
        mid = np.array([0.0, 0.0, 0.5 * (nr - 1) - 0.5 * _KNIT_D])
        base = len(loops)
        for P in rows:
            loops.append((P - mid) @ Rt.T + place[t])
        for (a, b), v in e.items():
            exp[(base + a, base + b)] = v
    if sigma > 0:
        nrng = np.random.default_rng(seed if noise_seed is None else noise_seed)
        loops = [P + nrng.normal(0.0, sigma, size=P.shape) for P in loops]
    return _pack(loops, dtype, exp, "knit", seed,
                 meta={"tubes": len(tubes), "per_span": per_span,
                       "row_starts": [sum(tubes[u][1] for u in range(t)) for t in range(len(tubes))]})


# --------------------------------------------------------- long loop pairs (C4)
def _resample_closed(P: np.ndarray, n: int) -> np.ndarray:
    """Resample a dense closed polyline uniformly in arc length to n points."""
    Q = np.vstack([P, P[:1]])
    seg = np.linalg.norm(np.diff(Q, axis=0), axis=1)
    s = np.concatenate([[0.0], np.cumsum(seg)])
    target = np.arange(n) * (s[-1] / n)
    out = np.empty((n, 3))
    for q in range(3):
        out[:, q] = np.interp(target, s, Q[:, q])
    return out


def _star_outline(phi, a, psi, b, chi, k, petals, amp, pphase):
    """Unit-scale star-shaped outline: polar radius and height as functions of
    the angle phi (arrays evaluated mode by mode to keep memory flat)."""
    r = 1.0 + amp * np.cos(petals * phi + pphase)
    z = np.zeros_like(phi)
    for q in range(k.size):
        r += a[q] * np.cos(k[q] * phi + psi[q])
        z += b[q] * np.cos(k[q] * phi + chi[q])
    return np.stack([r * np.cos(phi), r * np.sin(phi), z], 1)


def winding_pair(seed: int, n_a: int, n_b: int, lk: int, step: float = 1e-3, rho: float = 0.1,
                 modes: int = 6, dense: int = 2):
    """One long closed curve C and a companion D winding ``lk`` times around it.

    C is a smooth random closed curve over a star-shaped top view: polar
    radius R0 (1 + amp cos(K phi) + sum_k a_k cos(k phi + psi_k)) with K petals
    (which keeps a long curve compact) and a random smooth height z(phi); its
    length is n_a * step and the petal count is lowered until the radius of
    curvature stays above 4 rho.  D = C + rho (cos(theta) u + sin(theta) v)
    with u the horizontal normal of C, v = t x u and theta = 2 pi lk s / len.
    With lk = 0, D's top view is a parallel curve of C's simple top view, so
    the two do not link; each full turn of theta adds one: Lk(C, D) = +lk for
    this orientation.  D is resampled to n_b segments.
    """
    rng = np.random.default_rng(seed)
    k = np.arange(2, modes + 2)
    a = rng.uniform(0.0, 0.15, size=k.size) / k
    psi = rng.uniform(0, 2 * np.pi, size=k.size)
    b = rng.uniform(0.0, 0.15, size=k.size) / k
    chi = rng.uniform(0, 2 * np.pi, size=k.size)
    amp = 0.25
    pphase = rng.uniform(0, 2 * np.pi)
    length = n_a * step
    # pick the petal count on a coarse sampling: largest K whose curve, scaled
    # to the target length, keeps every radius of curvature above 4 rho
    coarse = 2 * np.pi * np.arange(20000) / 20000
    petals = 24
    while True:
        P = _star_outline(coarse, a, psi, b, chi, k, petals, amp, pphase)
        Q = np.vstack([P, P[:1]])
        R0 = length / np.sum(np.linalg.norm(np.diff(Q, axis=0), axis=1))
        X = R0 * P
        d1 = (np.roll(X, -1, 0) - np.roll(X, 1, 0)) / 2
        d2 = np.roll(X, -1, 0) - 2 * X + np.roll(X, 1, 0)
        curv = np.linalg.norm(np.cross(d1, d2), axis=1) / np.linalg.norm(d1, axis=1) ** 3
        if petals <= 3 or 1.0 / curv.max() > 4 * rho:
            break
        petals -= 1
    m = dense * max(n_a, n_b)
    phi = 2 * np.pi * np.arange(m) / m
    C = R0 * _star_outline(phi, a, psi, b, chi, k, petals, amp, pphase)
    C = _resample_closed(C, m)
    t = np.roll(C, -1, 0) - np.roll(C, 1, 0)
    t /= np.linalg.norm(t, axis=1)[:, None]
    u = np.stack([-t[:, 1], t[:, 0], 0 * t[:, 0]], 1)
    u /= np.linalg.norm(u, axis=1)[:, None]
    v = np.cross(t, u)
    theta = 2 * np.pi * lk * np.arange(m) / m
    D = C + rho * (np.cos(theta)[:, None] * u + np.sin(theta)[:, None] * v)
    Cn = _resample_closed(C, n_a)
    Dn = _resample_closed(D, n_b)
    return Cn, Dn, lk


def long_pairs(seed: int = 0, n_pairs: int = 16, n_min: int = 1 << 18, n_max: int = 1 << 20,
               lk_max: int = 5, step: float = 1e-3, rho: float = 0.1, dtype=np.float32) -> LoopSet:
    """Long-loop stress test: ``n_pairs`` pairs (C_k, D_k), each loop with a
    seeded size in [n_min, n_max] segments of length ~step, D_k winding a seeded
    number of turns in [-lk_max, lk_max] around C_k.  Pairs sit on a square
    grid around the origin (coordinates stay small, so FP32 resolves the
    steps); the candidate list is the n_pairs (C_k, D_k) pairs."""
    rng = np.random.default_rng(seed)
    made = []
    for q in range(n_pairs):
        na = int(rng.integers(n_min, n_max + 1))
        nb = int(np.clip(na + rng.integers(-na // 16, na // 16 + 1), n_min, n_max))
        target = int(rng.integers(-lk_max, lk_max + 1))
        C, D, val = winding_pair(int(rng.integers(1 << 31)), na, nb, target, step, rho)
        made.append((C, D, val))
    ext = max(float(np.max(np.abs(np.vstack([C[:, :2], D[:, :2]])))) for C, D, _ in made)
    side = int(np.ceil(np.sqrt(n_pairs)))
    pitch = 2 * ext + 1.0
    loops, exp, pairs = [], {}, []
    for q, (C, D, val) in enumerate(made):
        off = np.array([(q % side - 0.5 * (side - 1)) * pitch, (q // side - 0.5 * (side - 1)) * pitch, 0.0])
        i = len(loops)
        loops += [C + off, D + off]
        pairs.append([i, i + 1])
        exp[(i, i + 1)] = val
    return _pack(loops, dtype, exp, "long_pairs", seed, np.array(pairs, np.int32),
                 meta={"n_pairs": n_pairs})


# ------------------------------------------------------------- named configs
def config(name: str, seed: int = 0, **kw) -> LoopSet:
    """The five workloads by name: ``ring_grid`` (8x8 rings x 32 segments,
    FP64), ``chainmail`` (14,000 rings x 64 segments, FP32), ``knit`` (2,000
    B-spline rows, 512-16,384 segments each, FP32), ``long_pairs`` (16 pairs of
    2^18-2^20-segment loops, FP32)."""
    if name == "ring_grid":
        return ring_grid(seed, **kw)
    if name == "chainmail":
        return chainmail(seed, **kw)
    if name == "knit":
        return knit(seed, **kw)
    if name == "long_pairs":
        return long_pairs(seed, **kw)
    raise ValueError("unknown config %r" % name)
