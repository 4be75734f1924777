"""Seeded synthetic contact configurations shaped like the paper's workloads.

This module only draws inputs; it holds none of the QP's arithmetic, so both the
GPU library's tests and the CPU oracle can be fed from it.

Shapes follow the paper's setting: 4-fingertip (Allegro/Leap) and 5-fingertip
(Shadow) hands (Sec. V-A, V-C), objects rescaled to 0.06-0.12 m (Sec. V-A) and
unit desired-wrench directions t_j (Sec. IV-A, Eq. 7).  The object meshes are
stood in by spheres and axis-aligned ellipsoids centred at the origin, the
object's centre of gravity (Sec. III).

Array layout (all float32, C-contiguous, padded to ``m_max`` contacts):
  points  [G, m_max, 3]   contact positions p_i (object frame, metres)
  normals [G, m_max, 3]   inward surface normals n_i (unit)
  mu      [G, m_max]      friction coefficients
  wrench  [W, 6]          desired wrench directions t_j (unit in R^6)
  counts  [G]   int32     contacts per grasp m_g
  woff    [G+1] int32     CSR offsets of each grasp's wrenches (W = woff[G])
Padding entries (contacts beyond m_g) hold p = 0, n = (0, 0, 1), mu = 0.5.
"""
from __future__ import annotations

import dataclasses

import numpy as np

#: Torque scale 1/L with L = 0.05 m (the scale the desired torques are quoted in).
TORQUE_SCALE = 20.0


@dataclasses.dataclass
class Batch:
    points: np.ndarray
    normals: np.ndarray
    mu: np.ndarray
    wrench: np.ndarray
    counts: np.ndarray
    woff: np.ndarray
    name: str = ""

    @property
    def n_grasps(self) -> int:
        return int(self.counts.shape[0])

    @property
    def m_max(self) -> int:
        return int(self.points.shape[1])

    @property
    def n_qps(self) -> int:
        return int(self.woff[-1])

    def subset(self, grasps) -> "Batch":
        """A new batch holding the listed grasps (in that order)."""
        grasps = np.asarray(grasps, dtype=np.int64)
        s = self.woff[1:] - self.woff[:-1]
        ws = [np.arange(self.woff[g], self.woff[g + 1]) for g in grasps]
        widx = np.concatenate(ws) if ws else np.zeros(0, dtype=np.int64)
        woff = np.zeros(len(grasps) + 1, dtype=np.int32)
        woff[1:] = np.cumsum(s[grasps])
        return Batch(self.points[grasps].copy(), self.normals[grasps].copy(),
                     self.mu[grasps].copy(), self.wrench[widx].copy(),
                     self.counts[grasps].copy(), woff, self.name + "[subset]")


def unit_sphere(rng: np.random.Generator, shape) -> np.ndarray:
    """Uniform directions on S^2 (normalised Gaussians)."""
    v = rng.standard_normal(tuple(shape) + (3,))
    return v / np.linalg.norm(v, axis=-1, keepdims=True)


def wrench_dirs(rng: np.random.Generator, w: int) -> np.ndarray:
    """Uniform unit desired-wrench directions on S^5."""
    v = rng.standard_normal((w, 6))
    return (v / np.linalg.norm(v, axis=-1, keepdims=True)).astype(np.float32)


FORCE_AXIS_WRENCHES = np.array([[1, 0, 0, 0, 0, 0], [-1, 0, 0, 0, 0, 0],
                                [0, 1, 0, 0, 0, 0], [0, -1, 0, 0, 0, 0],
                                [0, 0, 1, 0, 0, 0], [0, 0, -1, 0, 0, 0]], dtype=np.float32)


def force_axis_batch(batch: "Batch") -> "Batch":
    """The same grasps with the six desired wrenches the paper uses for
    force closure (Sec. IV-A): unit forces along +-x, +-y, +-z with zero
    torque, for every grasp."""
    g = batch.n_grasps
    woff = (6 * np.arange(g + 1)).astype(np.int32)
    wrench = np.tile(FORCE_AXIS_WRENCHES, (g, 1))
    return Batch(batch.points.copy(), batch.normals.copy(), batch.mu.copy(), wrench,
                 batch.counts.copy(), woff, batch.name + "[force-axis wrenches]")


def sphere_contacts(rng, n_grasps, m, radius=0.05):
    u = unit_sphere(rng, (n_grasps, m))
    return (radius * u).astype(np.float32), (-u).astype(np.float32)


def ellipsoid_contacts(rng, n_grasps, m, lo=0.02, hi=0.08):
    """Points uniform-in-direction on axis-aligned ellipsoids with semi-axes
    ~ U[lo, hi]; inward normals are the negated normalised gradient of
    x^2/a^2 + y^2/b^2 + z^2/c^2."""
    axes = rng.uniform(lo, hi, size=(n_grasps, 1, 3))
    u = unit_sphere(rng, (n_grasps, m))
    p = axes * u
    g = p / axes ** 2
    n = -g / np.linalg.norm(g, axis=-1, keepdims=True)
    return p.astype(np.float32), n.astype(np.float32)


def _pack(points_list, normals_list, mu_list, counts, s_list, wrench, m_max, name):
    G = len(counts)
    P = np.zeros((G, m_max, 3), np.float32)
    N = np.zeros((G, m_max, 3), np.float32)
    N[..., 2] = 1.0
    MU = np.full((G, m_max), 0.5, np.float32)
    for g in range(G):
        m = counts[g]
        P[g, :m] = points_list[g]
        N[g, :m] = normals_list[g]
        MU[g, :m] = mu_list[g]
    woff = np.zeros(G + 1, np.int32)
    woff[1:] = np.cumsum(np.asarray(s_list, np.int64))
    return Batch(P, N, MU, wrench, np.asarray(counts, np.int32), woff, name)


def uniform_batch(seed, n_grasps, m, s, geometry="ellipsoid", mu=None,
                  mu_range=(0.3, 0.8), name=""):
    """Every grasp has m contacts and s wrenches."""
    rng = np.random.Generator(np.random.PCG64(seed))
    if geometry == "sphere":
        p, n = sphere_contacts(rng, n_grasps, m)
    else:
        p, n = ellipsoid_contacts(rng, n_grasps, m)
    if mu is None:
        mug = rng.uniform(mu_range[0], mu_range[1], size=(n_grasps, 1))
        muv = np.repeat(mug, m, axis=1).astype(np.float32)
    else:
        muv = np.full((n_grasps, m), mu, np.float32)
    t = wrench_dirs(rng, n_grasps * s)
    woff = (np.arange(n_grasps + 1, dtype=np.int64) * s).astype(np.int32)
    return Batch(np.ascontiguousarray(p), np.ascontiguousarray(n),
                 np.ascontiguousarray(muv), t,
                 np.full(n_grasps, m, np.int32), woff, name)


def mixed_batch(seed, n_grasps, m_choices=(4, 5), s_range=(6, 32),
                mu_range=(0.3, 0.8), name=""):
    """Equal split over m_choices (shuffled); s uniform integer in s_range
    (inclusive) per grasp; ellipsoid geometry; mu per grasp."""
    rng = np.random.Generator(np.random.PCG64(seed))
    k = len(m_choices)
    counts = np.repeat(np.asarray(m_choices), -(-n_grasps // k))[:n_grasps]
    rng.shuffle(counts)
    m_max = int(max(m_choices))
    p, n = ellipsoid_contacts(rng, n_grasps, m_max)
    mug = rng.uniform(mu_range[0], mu_range[1], size=(n_grasps, 1))
    s = rng.integers(s_range[0], s_range[1] + 1, size=n_grasps)
    t = wrench_dirs(rng, int(s.sum()))
    pl = [p[g, :counts[g]] for g in range(n_grasps)]
    nl = [n[g, :counts[g]] for g in range(n_grasps)]
    ml = [np.repeat(mug[g], counts[g]) for g in range(n_grasps)]
    return _pack(pl, nl, ml, counts, s, t, m_max, name)


# The five benchmark configurations.  ``scale`` shrinks the grasp count for
# quick parity runs while keeping every per-grasp distribution unchanged.
CONFIG_SEEDS = (16490, 16491, 16492, 16493, 16494)


def config(idx: int, n_grasps: int | None = None) -> Batch:
    if idx == 0:
        return uniform_batch(CONFIG_SEEDS[0], n_grasps or 64, 4, 6,
                             geometry="sphere", mu=0.5, name="sphere-m4-s6")
    if idx in (1, 2):
        return uniform_batch(CONFIG_SEEDS[idx], n_grasps or 8192, 5, 16,
                             geometry="ellipsoid", name="ellipsoid-m5-s16")
    if idx == 3:
        return mixed_batch(CONFIG_SEEDS[3], n_grasps or 50000,
                           name="ellipsoid-m45-s6to32")
    raise ValueError("config %d is not a single batch" % idx)


@dataclasses.dataclass
class Request:
    rid: int
    arrival: float      # seconds from stream start
    batch: Batch
    steps: int          # upper-level steps to run
    walk: np.ndarray    # [steps, G, m_max, 3] perturbations of the points


def request_stream(seed=CONFIG_SEEDS[4], rate=200.0, duration=60.0,
                   size_range=(16, 4096), steps=50, sigma=1e-3,
                   max_requests=None, start=0):
    """Poisson arrivals; each request is a mixed batch of log-uniform size,
    with a random walk on its contact points (normals fixed) per step.
    start: yield from request `start` on (the earlier ones are drawn but not
    built, so the stream is the same)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    t = 0.0
    rid = 0
    while True:
        t += rng.exponential(1.0 / rate)
        if t > duration or (max_requests is not None and rid >= max_requests):
            return
        size = int(np.exp(rng.uniform(np.log(size_range[0]), np.log(size_range[1]))))
        sub_seed = int(rng.integers(0, 2 ** 62))
        if rid < start:
            rid += 1
            continue
        b = mixed_batch(sub_seed, size, name="req%d" % rid)
        walk_rng = np.random.Generator(np.random.PCG64(sub_seed ^ 0x5DEECE66D))
        walk = (sigma * walk_rng.standard_normal((steps,) + b.points.shape)).astype(np.float32)
        for g in range(b.n_grasps):
            walk[:, g, b.counts[g]:] = 0.0
        yield Request(rid, t, b, steps, walk)
        rid += 1


@dataclasses.dataclass
class FineContacts:
    """Inputs of the fine-stage surrogate energies (Sec. IV-C, Eq. 10-11).

    link_rot   [G, m_max, 3, 3]  R_i of the link carrying fingertip i (row-major)
    link_trans [G, m_max, 3]     T_i
    hand_fine  [G, m_max, 3]     c^f_{i,w}: nearest point on fingertip i (world)
    obj_fine   [G, m_max, 3]     p^f_i: nearest point on the object
    obj_coarse [G, m_max, 3]     p^c_i: object point from the end of the coarse stage
    counts     [G] int32         fingertips per grasp
    w_q, w_e   [G]               loss weights of Q' and of E^f_d
    Padding contacts hold R = I and zero points.
    """
    link_rot: np.ndarray
    link_trans: np.ndarray
    hand_fine: np.ndarray
    obj_fine: np.ndarray
    obj_coarse: np.ndarray
    counts: np.ndarray
    w_q: np.ndarray
    w_e: np.ndarray

    @property
    def n_grasps(self) -> int:
        return int(self.counts.shape[0])

    @property
    def m_max(self) -> int:
        return int(self.link_trans.shape[1])


def random_rotations(rng, shape) -> np.ndarray:
    """Uniform rotations from normalised Gaussian quaternions."""
    q = rng.standard_normal(tuple(shape) + (4,))
    q /= np.linalg.norm(q, axis=-1, keepdims=True)
    w, x, y, z = q[..., 0], q[..., 1], q[..., 2], q[..., 3]
    R = np.empty(tuple(shape) + (3, 3))
    R[..., 0, 0] = 1 - 2 * (y * y + z * z)
    R[..., 0, 1] = 2 * (x * y - w * z)
    R[..., 0, 2] = 2 * (x * z + w * y)
    R[..., 1, 0] = 2 * (x * y + w * z)
    R[..., 1, 1] = 1 - 2 * (x * x + z * z)
    R[..., 1, 2] = 2 * (y * z - w * x)
    R[..., 2, 0] = 2 * (x * z - w * y)
    R[..., 2, 1] = 2 * (y * z + w * x)
    R[..., 2, 2] = 1 - 2 * (x * x + y * y)
    return R


def fine_contacts(seed, n_grasps, m=5, m_choices=None, tip=0.02, gap=2e-3, drift=1e-3):
    """Fingertips on ellipsoid objects at the end of the coarse stage: p^c on
    the surface, the fine nearest points within a few mm of it (gap: fingertip
    offset, drift: coarse-to-fine shift of the object point), each link's
    origin `tip` metres behind its fingertip point along a random direction
    of the link frame."""
    rng = np.random.Generator(np.random.PCG64(seed))
    if m_choices is None:
        counts = np.full(n_grasps, m, np.int32)
        m_max = m
    else:
        counts = rng.choice(np.asarray(m_choices, np.int32), size=n_grasps)
        m_max = int(max(m_choices))
    pc, _ = ellipsoid_contacts(rng, n_grasps, m_max)
    pc = pc.astype(np.float64)
    pf = pc + drift * rng.standard_normal(pc.shape)
    cw = pf + gap * rng.standard_normal(pc.shape)
    R = random_rotations(rng, (n_grasps, m_max))
    c_l = tip * unit_sphere(rng, (n_grasps, m_max))
    T = cw - np.einsum("gmij,gmj->gmi", R, c_l)
    wq = rng.uniform(0.5, 2.0, n_grasps)
    we = rng.uniform(0.5, 2.0, n_grasps)
    pad = np.arange(m_max)[None, :] >= counts[:, None]
    R[pad] = np.eye(3)
    for a in (T, cw, pf, pc):
        a[pad] = 0.0
    f32 = lambda a: np.ascontiguousarray(a, np.float32)
    return FineContacts(f32(R), f32(T), f32(cw), f32(pf), f32(pc), counts.astype(np.int32),
                        f32(wq), f32(we))


@dataclasses.dataclass
class HandBatch:
    """A floating hand over an analytic object per grasp, with the QP's
    friction coefficients and desired wrenches (the coarse stage of
    Sec. IV-C on analytic shapes).

    tip_local [G, m_max, 3]  c_{i,l}: fingertip sphere centres in the hand frame
    semi_axes [G, 3]         the object: ellipsoid sum (x_k / a_k)^2 <= 1 (a sphere when equal)
    rot       [G, 3, 3]      hand rotation R (row-major)
    trans     [G, 3]         hand translation T
    counts    [G] int32      fingertips per grasp (padding tips are zero)
    woff, mu, wrench         as in Batch
    """
    tip_local: np.ndarray
    semi_axes: np.ndarray
    rot: np.ndarray
    trans: np.ndarray
    counts: np.ndarray
    woff: np.ndarray
    mu: np.ndarray
    wrench: np.ndarray
    name: str = ""

    @property
    def n_grasps(self) -> int:
        return int(self.counts.shape[0])

    @property
    def m_max(self) -> int:
        return int(self.tip_local.shape[1])

    @property
    def n_qps(self) -> int:
        return int(self.woff[-1])

    def qp_batch(self, points, normals) -> Batch:
        """The QP batch of these grasps at the given contacts."""
        return Batch(np.ascontiguousarray(points, np.float32), np.ascontiguousarray(normals, np.float32),
                     self.mu, self.wrench, self.counts, self.woff, self.name)


def hand_batch(seed, n_grasps, m=5, m_choices=None, s=16, shape="ellipsoid", radius=0.01,
               standoff=(0.005, 0.02), shift=0.005, force_axis=False, mu_range=(0.3, 0.8), inside=0.0):
    """Rigid hands placed around analytic objects.  The fingertips sit on a
    thumb-opposes-fingers pattern (the thumb at -y, the fingers spread along
    x at +y, all tilted towards +z) jittered per grasp, at a distance
    max(a) + radius + U[standoff] from the hand origin, so that every
    fingertip sphere starts outside the object; R is a uniform random
    rotation and T ~ U[-shift, shift]^3.  Objects: ellipsoids with semi-axes
    ~ U[0.02, 0.08] m, spheres with radius ~ U[0.03, 0.06] m, or a 50/50 mix.
    Wrenches: s random unit directions per grasp, or the six force axes.
    inside > 0: that fraction of the fingertips (drawn after everything else,
    so the rest of the batch is unchanged) moves along its direction to a
    distance U[0.1, 0.5] min(a) from the hand origin, which with
    |T_k| <= shift <= 0.005 and min(a) >= 0.02 puts its centre inside the
    object."""
    rng = np.random.Generator(np.random.PCG64(seed))
    if m_choices is None:
        counts = np.full(n_grasps, m, np.int32)
        m_max = m
    else:
        counts = rng.choice(np.asarray(m_choices, np.int32), size=n_grasps).astype(np.int32)
        m_max = int(max(m_choices))
    ell = rng.uniform(0.02, 0.08, size=(n_grasps, 3))
    sph = np.repeat(rng.uniform(0.03, 0.06, size=(n_grasps, 1)), 3, axis=1)
    if shape == "ellipsoid":
        axes = ell
    elif shape == "sphere":
        axes = sph
    elif shape == "mixed":
        axes = np.where(rng.random((n_grasps, 1)) < 0.5, ell, sph)
    else:
        raise ValueError(shape)
    tips = np.zeros((n_grasps, m_max, 3))
    for g in range(n_grasps):
        k = int(counts[g])
        dirs = np.zeros((k, 3))
        dirs[0] = (0.0, -1.0, 0.3)
        xs = np.linspace(-0.6, 0.6, k - 1) if k > 2 else np.zeros(max(k - 1, 0))
        for j in range(1, k):
            dirs[j] = (xs[j - 1], 1.0, 0.3)
        dirs += 0.1 * rng.standard_normal(dirs.shape)
        dirs /= np.linalg.norm(dirs, axis=1, keepdims=True)
        r = axes[g].max() + radius + rng.uniform(standoff[0], standoff[1], size=(k, 1))
        tips[g, :k] = r * dirs
    R = random_rotations(rng, (n_grasps,))
    T = rng.uniform(-shift, shift, size=(n_grasps, 3))
    mu = np.zeros((n_grasps, m_max), np.float32)
    mu[:] = rng.uniform(mu_range[0], mu_range[1], size=(n_grasps, 1))
    if force_axis:
        woff = (6 * np.arange(n_grasps + 1)).astype(np.int32)
        wrench = np.tile(FORCE_AXIS_WRENCHES, (n_grasps, 1))
    else:
        woff = (s * np.arange(n_grasps + 1)).astype(np.int32)
        wrench = wrench_dirs(rng, n_grasps * s)
    if inside > 0.0:
        assert shift <= 0.005
        flag = rng.random((n_grasps, m_max)) < inside
        depth = rng.uniform(0.1, 0.5, size=(n_grasps, m_max))
        for g in range(n_grasps):
            for i in range(int(counts[g])):
                if flag[g, i]:
                    tips[g, i] *= depth[g, i] * axes[g].min() / np.linalg.norm(tips[g, i])
    f32 = lambda a: np.ascontiguousarray(a, np.float32)
    return HandBatch(f32(tips), f32(axes), f32(R), f32(T), counts, woff, mu, wrench,
                     "hand-%s-m%s-s%s" % (shape, m if m_choices is None else "".join(map(str, m_choices)),
                                          "6fa" if force_axis else s))
