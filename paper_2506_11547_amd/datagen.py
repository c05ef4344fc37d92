"""Seeded synthetic correspondences for the rotation-voting workloads.

This module only *draws* inputs: a ground-truth rotation, unit directions, noise
and outliers.  It contains none of the voting method's arithmetic (no circle
basis, no sampling, no chart, no binning, no scoring), so both the HIP library
and the CPU oracle can be fed from it without sharing any of the method.

Conventions
-----------
* Quaternions are (w, x, y, z), Hamilton product, unit norm, ``w >= 0``.
* Correspondences are float32 SoA arrays of shape ``[3, N]`` (all x components,
  then y, then z), the layout the C-ABI expects.
* Everything is drawn in float64 from ``numpy.random.default_rng(seed)`` (PCG64)
  in a fixed order and cast to float32 at the end.

Workload shapes follow the synthetic experiments of the paper (Sec. 5.3.1:
N = 1e5..1e6 correspondences, outlier ratios up to 99 %, random mismatches as
outliers; Table 1's same-axis structured outliers) and the named configurations
below.  No external dataset is used.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "Instance",
    "Workload",
    "WORKLOADS",
    "make_instance",
    "make_workload",
    "BatchWorkload",
    "BATCH_WORKLOADS",
    "Batch",
    "make_batch",
    "MultiInstance",
    "make_multi_instance",
    "RigidInstance",
    "make_rigid_instance",
    "quat_to_matrix",
    "rotation_error_deg",
]


@dataclass
class Instance:
    x: np.ndarray          # float32 [3, N]
    y: np.ndarray          # float32 [3, N]
    q_gt: np.ndarray       # float64 [4], w >= 0
    inlier: np.ndarray     # bool [N], ground-truth inlier flags
    seed: int
    params: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.x.shape[1])


@dataclass(frozen=True)
class Workload:
    """One named synthetic solve: input recipe plus the solver settings."""
    name: str
    n: int
    outlier_ratio: float
    sigma_deg: float
    grid: int
    samples: int           # J, samples per circle
    eps_deg: float         # inlier threshold of the rescoring step (degrees)
    topk: int
    seed: int
    radii: tuple | None = None     # (lo, hi): scale x by U[lo, hi] radii
    noise: str = "angular"         # "angular" (tangent Gaussian) or "additive"

    def instance(self) -> Instance:
        return make_instance(self.n, self.outlier_ratio, self.sigma_deg, self.seed,
                             radii=self.radii, noise=self.noise)


# Named single-solve workloads.  "large" is the headline measurement
# (N = 1e6 at 99 % outliers); "small" is the oracle-sized case.
WORKLOADS = {
    "small": Workload("small", n=1000, outlier_ratio=0.90, sigma_deg=0.5, grid=64,
                      samples=512, eps_deg=1.0, topk=16, seed=0),
    "medium": Workload("medium", n=100_000, outlier_ratio=0.95, sigma_deg=0.5, grid=128,
                       samples=1024, eps_deg=1.0, topk=16, seed=1, radii=(0.5, 2.0)),
    "large": Workload("large", n=1_000_000, outlier_ratio=0.99, sigma_deg=1.0, grid=256,
                      samples=2048, eps_deg=1.5, topk=64, seed=2),
    # The paper's default resolution (accumulator step 1/180, i.e. a 360^3 grid,
    # and 180 samples per circle; Sec. 5.1) with its additive noise model.
    "paper_default": Workload("paper_default", n=1_000_000, outlier_ratio=0.99,
                              sigma_deg=0.0, grid=360, samples=180, eps_deg=1.5,
                              topk=16, seed=5, noise="additive"),
}


def make_workload(name: str) -> tuple[Workload, Instance]:
    w = WORKLOADS[name]
    return w, w.instance()


@dataclass
class Batch:
    x: np.ndarray          # float32 [3, sum N_b], instances back to back
    y: np.ndarray
    offsets: np.ndarray    # int64 [B + 1]; instance b is columns offsets[b]:offsets[b+1]
    q_gt: np.ndarray       # float64 [B, 4]
    outlier_ratio: np.ndarray  # float64 [B]

    @property
    def B(self) -> int:
        return len(self.offsets) - 1

    def instance(self, b: int):
        lo, hi = int(self.offsets[b]), int(self.offsets[b + 1])
        return self.x[:, lo:hi], self.y[:, lo:hi]


@dataclass
class BatchWorkload:
    """Many independent instances solved together (same G, J, K, eps): N is
    log-uniform on [n_lo, n_hi], the outlier ratio uniform on [rho_lo, rho_hi]."""
    name: str
    instances: int
    n_lo: int
    n_hi: int
    rho_lo: float
    rho_hi: float
    sigma_deg: float
    grid: int
    samples: int
    eps_deg: float
    topk: int
    seed: int

    def batch(self, instances: int | None = None) -> Batch:
        return make_batch(self.instances if instances is None else instances, self.n_lo,
                          self.n_hi, self.rho_lo, self.rho_hi, self.sigma_deg, self.seed)


BATCH_WORKLOADS = {
    # 4096 uneven instances: N spans 200x (mean about 3756, about 1.54e7 in all).
    "batch": BatchWorkload("batch", instances=4096, n_lo=100, n_hi=20_000, rho_lo=0.5,
                           rho_hi=0.99, sigma_deg=0.5, grid=64, samples=512, eps_deg=1.0,
                           topk=16, seed=3),
}


def make_batch(instances: int, n_lo: int, n_hi: int, rho_lo: float, rho_hi: float,
               sigma_deg: float, seed: int) -> Batch:
    """Draw order (fixed): every N_b (log-uniform, rounded down), every outlier
    ratio, every instance seed; then the instances in order (make_instance)."""
    rng = np.random.default_rng(seed)
    if n_lo > 0:
        ns = np.floor(np.exp(rng.uniform(math.log(n_lo), math.log(n_hi + 1), size=instances)))
        ns = np.minimum(ns, n_hi).astype(np.int64)
    else:
        ns = rng.integers(0, n_hi + 1, size=instances).astype(np.int64)
    rhos = rng.uniform(rho_lo, rho_hi, size=instances)
    seeds = rng.integers(0, 2**62, size=instances)
    offsets = np.zeros(instances + 1, np.int64)
    offsets[1:] = np.cumsum(ns)
    x = np.empty((3, int(offsets[-1])), np.float32)
    y = np.empty_like(x)
    q = np.empty((instances, 4))
    for b in range(instances):
        inst = make_instance(int(ns[b]), float(rhos[b]), sigma_deg, int(seeds[b]))
        x[:, offsets[b]:offsets[b + 1]] = inst.x
        y[:, offsets[b]:offsets[b + 1]] = inst.y
        q[b] = inst.q_gt
    return Batch(x, y, offsets, q, rhos)


@dataclass
class MultiInstance:
    x: np.ndarray          # float32 [3, N]
    y: np.ndarray
    q_gt: np.ndarray       # float64 [M, 4], w >= 0
    model: np.ndarray      # int32 [N]: the model (0..M-1) of an inlier, -1 for an outlier
    seed: int


def make_multi_instance(models: int, per_model: int, outliers: int, delta: float, seed: int,
                        noise: str = "additive") -> MultiInstance:
    """Several rotations in one scene (the paper's multiple-rotation experiment:
    random unit vectors rotated by one of `models` uniformly random rotations,
    per_model correspondences each, noise delta; plus uniform outliers).
    Draw order (fixed): the rotations; per model its directions and noise;
    the outliers; one permutation of all correspondences.  noise="additive":
    y = normalise(R x + delta N(0, I)) (delta = 0.01 in the paper);
    "angular": a tangent-plane rotation with std delta degrees per axis."""
    rng = np.random.default_rng(seed)
    qs = np.array([_random_unit_quat(rng) for _ in range(models)])
    xs, ys, lab = [], [], []
    for m in range(models):
        xh = _unit_rows(rng.normal(size=(per_model, 3)))
        z = xh @ quat_to_matrix(qs[m]).T
        if noise == "additive":
            y = _unit_rows(z + delta * rng.normal(size=z.shape))
        elif noise == "angular":
            y = _angular_noise(rng, z, math.radians(delta))
        else:
            raise ValueError(f"unknown noise model {noise!r}")
        xs.append(xh)
        ys.append(y)
        lab.append(np.full(per_model, m, np.int32))
    if outliers:
        xs.append(_unit_rows(rng.normal(size=(outliers, 3))))
        ys.append(_unit_rows(rng.normal(size=(outliers, 3))))
        lab.append(np.full(outliers, -1, np.int32))
    x = np.concatenate(xs) if xs else np.zeros((0, 3))
    y = np.concatenate(ys) if ys else np.zeros((0, 3))
    lab = np.concatenate(lab) if lab else np.zeros(0, np.int32)
    perm = rng.permutation(len(lab))
    return MultiInstance(np.ascontiguousarray(x[perm].T.astype(np.float32)),
                         np.ascontiguousarray(y[perm].T.astype(np.float32)), qs, lab[perm], seed)


@dataclass
class RigidInstance:
    x: np.ndarray          # float32 [3, N] points (not directions)
    y: np.ndarray          # float32 [3, N]
    q_gt: np.ndarray       # float64 [4], w >= 0
    t_gt: np.ndarray       # float64 [3]
    inlier: np.ndarray     # bool [N]
    seed: int

    @property
    def n(self) -> int:
        return int(self.x.shape[1])


def make_rigid_instance(n: int, outlier_ratio: float, delta: float, seed: int,
                        box: float = 1.0) -> RigidInstance:
    """Point correspondences under one rigid motion with outliers (the paper's
    6-DoF synthetic experiment, Sec. 5.4.1): R uniform, t uniform in
    [-1, 1]^3; x uniform in [-box, box]^3; inliers y = R x + t + delta N(0, I);
    outliers x and y independent and uniform in [-box, box]^3.
    Draw order (fixed): q, t, all x, a permutation whose first
    round((1 - outlier_ratio) n) entries are inliers, inlier noise, outlier y."""
    if n < 0:
        raise ValueError("n must be >= 0")
    rng = np.random.default_rng(seed)
    q = _random_unit_quat(rng)
    t = rng.uniform(-1.0, 1.0, size=3)
    x = rng.uniform(-box, box, size=(n, 3))
    perm = rng.permutation(n)
    n_in = int(round((1.0 - outlier_ratio) * n))
    inl = np.zeros(n, bool)
    inl[perm[:n_in]] = True
    y = np.empty_like(x)
    R = quat_to_matrix(q)
    y[inl] = x[inl] @ R.T + t + delta * rng.normal(size=(n_in, 3))
    y[~inl] = rng.uniform(-box, box, size=(n - n_in, 3))
    return RigidInstance(np.ascontiguousarray(x.T.astype(np.float32)),
                         np.ascontiguousarray(y.T.astype(np.float32)), q, t, inl, seed)


def quat_to_matrix(q) -> np.ndarray:
    """Rotation matrix of a unit quaternion (w, x, y, z) (float64)."""
    w, x, y, z = (float(c) for c in q)
    return np.array([
        [w * w + x * x - y * y - z * z, 2 * (x * y - w * z), 2 * (x * z + w * y)],
        [2 * (x * y + w * z), w * w - x * x + y * y - z * z, 2 * (y * z - w * x)],
        [2 * (x * z - w * y), 2 * (y * z + w * x), w * w - x * x - y * y + z * z],
    ])


def rotation_error_deg(q_a, q_b) -> float:
    """Geodesic angle between two rotations, in degrees (Sec. 5.2's e_R).
    From the relative rotation's axis-angle form, 2 atan2(|sin|, |cos|), which
    stays accurate for small angles (an arccos of the trace does not)."""
    ra, rb = quat_to_matrix(q_a), quat_to_matrix(q_b)
    d = ra.T @ rb
    c = (np.trace(d) - 1.0) * 0.5
    s = 0.5 * math.sqrt((d[2, 1] - d[1, 2]) ** 2 + (d[0, 2] - d[2, 0]) ** 2 + (d[1, 0] - d[0, 1]) ** 2)
    return math.degrees(math.atan2(s, c))


def _unit_rows(v: np.ndarray) -> np.ndarray:
    return v / np.linalg.norm(v, axis=1, keepdims=True)


def _random_unit_quat(rng) -> np.ndarray:
    q = rng.normal(size=4)
    q /= np.linalg.norm(q)
    if q[0] < 0:
        q = -q
    return q


def _rotate_about(v: np.ndarray, axis: np.ndarray, angle: np.ndarray) -> np.ndarray:
    """Rodrigues rotation of rows of v about unit rows of axis by angle (rad)."""
    c = np.cos(angle)[:, None]
    s = np.sin(angle)[:, None]
    kv = np.sum(axis * v, axis=1, keepdims=True)
    return v * c + np.cross(axis, v) * s + axis * kv * (1.0 - c)


def _angular_noise(rng, z: np.ndarray, sigma_rad: float) -> np.ndarray:
    """Perturb unit rows z by a tangent-plane Gaussian rotation (std sigma per axis)."""
    if sigma_rad == 0.0 or len(z) == 0:
        return z.copy()
    helper = np.where(np.abs(z[:, :1]) < 0.9, np.array([[1.0, 0.0, 0.0]]),
                      np.array([[0.0, 1.0, 0.0]]))
    t1 = _unit_rows(np.cross(z, helper))
    t2 = np.cross(z, t1)
    g = rng.normal(size=(len(z), 2)) * sigma_rad
    omega = g[:, :1] * t1 + g[:, 1:] * t2            # rotation vector, tangent to z
    ang = np.linalg.norm(omega, axis=1)
    safe = np.where(ang > 0, ang, 1.0)
    axis = omega / safe[:, None]
    out = _rotate_about(z, axis, ang)
    return np.where(ang[:, None] > 0, out, z)


def make_instance(n: int, outlier_ratio: float, sigma_deg: float, seed: int, *,
                  radii: tuple | None = None, noise: str = "angular",
                  same_axis_ratio: float = 0.0, q_gt=None) -> Instance:
    """Draw one synthetic rotation-estimation instance.

    Draw order (fixed): q_gt; unit x; radii (if any); a permutation whose first
    ``n_in = round((1 - outlier_ratio) * n)`` entries are inliers; inlier noise;
    outlier directions; same-axis structured outliers (Table 1's eta).

    noise="angular": y = Rot(omega) R x with omega a tangent-plane Gaussian of
    std ``sigma_deg`` per axis.  noise="additive": the paper's Sec. 5.2 model,
    y = normalise(R x + delta * N(0, I)) with delta = sigma_deg read as the raw
    perturbation std (0.01 in Table 1); delta defaults to 0.01 when sigma_deg is 0.
    """
    if n < 0:
        raise ValueError("n must be >= 0")
    rng = np.random.default_rng(seed)
    q = _random_unit_quat(rng) if q_gt is None else np.asarray(q_gt, np.float64)
    R = quat_to_matrix(q)
    xh = _unit_rows(rng.normal(size=(n, 3))) if n else np.zeros((0, 3))
    if radii is not None:
        r = rng.uniform(radii[0], radii[1], size=n)
    else:
        r = np.ones(n)
    perm = rng.permutation(n)
    n_in = int(round((1.0 - outlier_ratio) * n))
    inlier = np.zeros(n, dtype=bool)
    inlier[perm[:n_in]] = True
    z = xh @ R.T
    y = np.empty((n, 3))
    idx_in = perm[:n_in]
    if noise == "angular":
        y[idx_in] = _angular_noise(rng, z[idx_in], math.radians(sigma_deg))
    elif noise == "additive":
        delta = sigma_deg if sigma_deg > 0 else 0.01
        y[idx_in] = _unit_rows(z[idx_in] + delta * rng.normal(size=(n_in, 3)))
    else:
        raise ValueError(f"unknown noise model {noise!r}")
    idx_out = perm[n_in:]
    y[idx_out] = _unit_rows(rng.normal(size=(len(idx_out), 3))) if len(idx_out) else y[idx_out]
    if same_axis_ratio > 0.0 and len(idx_out):
        n_sa = min(len(idx_out), int(round(same_axis_ratio * n)))
        sel = idx_out[:n_sa]
        axis = _unit_rows(rng.normal(size=(1, 3)))
        ang = rng.uniform(-math.pi, math.pi, size=n_sa)
        y[sel] = _rotate_about(xh[sel], np.repeat(axis, n_sa, axis=0), ang)
    x_out = (xh * r[:, None]).T.astype(np.float32)
    y_out = y.T.astype(np.float32)
    return Instance(np.ascontiguousarray(x_out), np.ascontiguousarray(y_out), q, inlier,
                    seed, dict(n=n, outlier_ratio=outlier_ratio, sigma_deg=sigma_deg,
                               radii=radii, noise=noise, same_axis_ratio=same_axis_ratio))
