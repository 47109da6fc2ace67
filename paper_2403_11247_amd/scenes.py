"""Seeded synthetic inputs shaped like the paper's RGB-D room workloads.

This module only draws numbers: cameras, poses, Gaussian attributes, voxel
anchors, MLP weights, mask logits, codebooks and request traces.  It holds
none of the renderer's arithmetic, so both the HIP path and the CPU oracle can
consume its output without sharing any of the method's code.

Every array is float32 (int32 for indices) in the layout the C ABI takes:
Gaussian attributes are structure-of-arrays ``[components][n]``.

Workloads (paper: Sec. 4 experiments use Replica 1200x680 and ScanNet/TUM
640x480 RGB-D sequences of indoor rooms; those datasets are replaced here by
procedurally generated rooms of the same image sizes):

* ``random_scene``     -- 2,000 free-floating Gaussians in front of a 128x96 view.
* ``room_anchors``     -- a 6x5x3 m room (walls plus 20 boxes) voxelised into
  anchors on a regular grid (Sec. 3.2: anchor feature 32-d, k offsets, scaling).
* ``room_camera``      -- a 1200x680 pinhole in a room corner, plus the target
  pose perturbed by 2 cm / 1 degree.
* ``mask_and_codebook``-- mask logits and 2-stage codebooks of 4096x7 entries.
* ``ba_window``        -- 12 keyframes on a circle, mixed resolutions.
* ``serve_trace``      -- Poisson request arrivals with random sizes and poses.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

TILE = 16
Z_NEAR = 0.2


@dataclasses.dataclass
class Camera:
    width: int
    height: int
    fx: float
    fy: float
    cx: float
    cy: float
    z_near: float = Z_NEAR
    tile: int = TILE


@dataclasses.dataclass
class Pose:
    """World-to-camera rigid transform: p_cam = R @ p_world + t (OpenCV axes)."""
    R: np.ndarray  # (3, 3) float32
    t: np.ndarray  # (3,) float32


@dataclasses.dataclass
class Gaussians:
    mean: np.ndarray     # (3, n)
    scale: np.ndarray    # (3, n) linear (not log)
    quat: np.ndarray     # (4, n) w, x, y, z (not necessarily unit)
    opacity: np.ndarray  # (n,)
    color: np.ndarray    # (3, n)

    @property
    def n(self) -> int:
        return int(self.opacity.shape[0])


@dataclasses.dataclass
class Anchors:
    xa: np.ndarray       # (3, na) anchor positions
    feat: np.ndarray     # (na, 32) anchor features, row-major
    scaling: np.ndarray  # (3, na) per-anchor scaling factor l
    offset: np.ndarray   # (na, k, 3) learnable offsets O

    @property
    def n(self) -> int:
        return int(self.feat.shape[0])

    @property
    def k(self) -> int:
        return int(self.offset.shape[1])


@dataclasses.dataclass
class MLP:
    W1: np.ndarray  # (hidden, in)  = (32, 32), or (32, 36) with the view input
    b1: np.ndarray  # (hidden,)
    W2: np.ndarray  # (k*11, hidden) = (110, 32)
    b2: np.ndarray  # (k*11,)


# Per-offset output layout of the decoder's second layer (11 values):
# [opacity logit, r, g, b logits, 3 log-scales, quaternion w, x, y, z].
OUT_PER_OFFSET = 11


def _f32(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.float32))


def look_at(position, target, up=(0.0, 0.0, 1.0)) -> Pose:
    """World-to-camera pose of a camera at ``position`` looking at ``target``.

    Camera axes follow the OpenCV convention: +z forward, +x right, +y down.
    """
    p = np.asarray(position, np.float64)
    f = np.asarray(target, np.float64) - p
    f /= np.linalg.norm(f)
    r = np.cross(f, np.asarray(up, np.float64))
    r /= np.linalg.norm(r)
    d = np.cross(f, r)
    R = np.stack([r, d, f])
    t = -R @ p
    return Pose(_f32(R), _f32(t))


def _axis_angle(axis, angle):
    a = np.asarray(axis, np.float64)
    a = a / np.linalg.norm(a)
    K = np.array([[0, -a[2], a[1]], [a[2], 0, -a[0]], [-a[1], a[0], 0]])
    return np.eye(3) + math.sin(angle) * K + (1 - math.cos(angle)) * (K @ K)


def perturb_pose(pose: Pose, seed: int, trans=0.02, rot_deg=1.0) -> Pose:
    """Move the camera centre by ``trans`` metres (random direction) and turn
    it by ``rot_deg`` degrees about a random axis."""
    rng = np.random.default_rng(seed)
    d = rng.normal(size=3)
    d /= np.linalg.norm(d)
    ax = rng.normal(size=3)
    R = pose.R.astype(np.float64)
    centre = -R.T @ pose.t.astype(np.float64)
    centre = centre + trans * d
    R2 = _axis_angle(ax, math.radians(rot_deg)) @ R
    return Pose(_f32(R2), _f32(-R2 @ centre))


# ---------------------------------------------------------------------------
# Small free-floating scene (128x96, 2,000 Gaussians)
# ---------------------------------------------------------------------------

def random_camera() -> Camera:
    return Camera(128, 96, 100.0, 100.0, 64.0, 48.0)


def identity_pose() -> Pose:
    return Pose(np.eye(3, dtype=np.float32), np.zeros(3, np.float32))


def random_scene(n=2000, seed=0, xy=1.0, z=(2.0, 4.0), log_scale=(0.01, 0.05)) -> Gaussians:
    """Means uniform in x,y in [-xy, xy], z in [z0, z1]; scales log-uniform per
    axis; random unit quaternions; opacity sigmoid(N(0,1)); colour U[0,1]^3.
    Draw order: means, scales, quaternions, opacities, colours."""
    rng = np.random.default_rng(seed)
    mean = np.empty((3, n))
    mean[0] = rng.uniform(-xy, xy, n)
    mean[1] = rng.uniform(-xy, xy, n)
    mean[2] = rng.uniform(z[0], z[1], n)
    scale = np.exp(rng.uniform(math.log(log_scale[0]), math.log(log_scale[1]), (3, n)))
    q = rng.normal(size=(4, n))
    q /= np.linalg.norm(q, axis=0, keepdims=True)
    opacity = 1.0 / (1.0 + np.exp(-rng.normal(size=n)))
    color = rng.uniform(0.0, 1.0, (3, n))
    return Gaussians(_f32(mean), _f32(scale), _f32(q), _f32(opacity), _f32(color))


def upstream_grads(width, height, seed=1):
    """Seeded upstream gradients dL/dC (3,H,W), dL/dD (H,W), dL/dA (H,W) ~ N(0,1)."""
    rng = np.random.default_rng(seed)
    return (_f32(rng.normal(size=(3, height, width))),
            _f32(rng.normal(size=(height, width))),
            _f32(rng.normal(size=(height, width))))


# ---------------------------------------------------------------------------
# Voxel-anchored room
# ---------------------------------------------------------------------------

ROOM = (6.0, 5.0, 3.0)


def _room_boxes(rng, n_boxes=20):
    """Axis-aligned boxes standing on the floor: (lo, hi) corners."""
    boxes = []
    for _ in range(n_boxes):
        side = rng.uniform(0.3, 1.2, 3)
        cx = rng.uniform(0.3 + side[0] / 2, ROOM[0] - 0.3 - side[0] / 2)
        cy = rng.uniform(0.3 + side[1] / 2, ROOM[1] - 0.3 - side[1] / 2)
        lo = np.array([cx - side[0] / 2, cy - side[1] / 2, 0.0])
        hi = np.array([cx + side[0] / 2, cy + side[1] / 2, side[2]])
        boxes.append((lo, hi))
    return boxes


def _face_voxels(axis, coord, lo, hi, h, dims):
    """Linear indices of grid voxels (size h) crossed by an axis-aligned face."""
    o1, o2 = [a for a in range(3) if a != axis]
    i_ax = min(max(int(math.floor(coord / h)), 0), dims[axis] - 1)
    r1 = np.arange(max(int(math.floor(lo[o1] / h)), 0), min(int(math.ceil(hi[o1] / h)), dims[o1]))
    r2 = np.arange(max(int(math.floor(lo[o2] / h)), 0), min(int(math.ceil(hi[o2] / h)), dims[o2]))
    g1, g2 = np.meshgrid(r1, r2, indexing="ij")
    idx = [None, None, None]
    idx[axis] = np.full(g1.size, i_ax)
    idx[o1] = g1.ravel()
    idx[o2] = g2.ravel()
    return (idx[0] * dims[1] + idx[1]) * dims[2] + idx[2]


def room_voxels(spacing=0.05, seed=0, n_boxes=20):
    """Centres of every voxel crossed by the room's walls, floor, ceiling and
    the faces of ``n_boxes`` random boxes (sorted by linear voxel index)."""
    rng = np.random.default_rng(seed)
    dims = [int(round(ROOM[a] / spacing)) for a in range(3)]
    lo0, hi0 = np.zeros(3), np.array(ROOM)
    faces = []
    for axis in range(3):
        faces.append((axis, 0.0, lo0, hi0))
        faces.append((axis, ROOM[axis], lo0, hi0))
    for lo, hi in _room_boxes(rng, n_boxes):
        for axis in range(3):
            faces.append((axis, lo[axis], lo, hi))
            faces.append((axis, hi[axis], lo, hi))
    lin = np.unique(np.concatenate([_face_voxels(a, c, lo, hi, spacing, dims) for a, c, lo, hi in faces]))
    iz = lin % dims[2]
    iy = (lin // dims[2]) % dims[1]
    ix = lin // (dims[2] * dims[1])
    centres = (np.stack([ix, iy, iz]).astype(np.float64) + 0.5) * spacing
    return centres


def room_anchors(n_anchors=40000, k=10, spacing=0.05, seed=0, feat_dim=32) -> Anchors:
    """Exactly ``n_anchors`` occupied voxels of the room (drawn without
    replacement), features ~ N(0, 0.1^2), offsets ~ U[-1,1]^3, scaling = spacing."""
    centres = room_voxels(spacing, seed)
    rng = np.random.default_rng(seed + 1)
    if n_anchors > centres.shape[1]:
        raise ValueError(f"room has only {centres.shape[1]} voxels at {spacing} m")
    pick = np.sort(rng.choice(centres.shape[1], n_anchors, replace=False))
    xa = centres[:, pick]
    feat = rng.normal(0.0, 0.1, (n_anchors, feat_dim))
    offset = rng.uniform(-1.0, 1.0, (n_anchors, k, 3))
    scaling = np.full((3, n_anchors), spacing)
    return Anchors(_f32(xa), _f32(feat), _f32(scaling), _f32(offset))


def room_mlp(k=10, hidden=32, feat_dim=32, seed=0, scale_m=0.02) -> MLP:
    """Kaiming-uniform weights; output biases put opacity near sigmoid(0),
    colour near 0.5 and the Gaussian scale near ``scale_m``.  Output rows are
    given per-attribute gains so that colours and shapes vary across anchors."""
    rng = np.random.default_rng(seed + 7)
    b_in = math.sqrt(6.0 / feat_dim)
    W1 = rng.uniform(-b_in, b_in, (hidden, feat_dim))
    b1 = rng.uniform(-0.05, 0.05, hidden)
    b_h = math.sqrt(6.0 / hidden)
    gain = np.array([3.5, 7.0, 7.0, 7.0, 2.0, 2.0, 2.0, 3.5, 3.5, 3.5, 3.5])
    W2 = rng.uniform(-b_h, b_h, (k * OUT_PER_OFFSET, hidden)) * np.tile(gain, k)[:, None]
    bias = np.array([0.0, 0.0, 0.0, 0.0] + [math.log(scale_m)] * 3 + [1.0, 0.0, 0.0, 0.0])
    b2 = np.tile(bias, k)
    return MLP(_f32(W1), _f32(b1), _f32(W2), _f32(b2))


def room_mlp_view(k=10, hidden=32, feat_dim=32, seed=0, scale_m=0.02, view_gain=0.1) -> MLP:
    """The same decoder with the view-dependent input of eq. (9): W1 gets four
    more columns for [delta, d_x, d_y, d_z] (drawn from their own stream, so the
    feature columns equal ``room_mlp``'s), U[-b, b] with b = sqrt(6 / 36) *
    view_gain.  The default gain keeps the room's Gaussians close to the
    feature-only decode (2.59M pairs in the room view instead of 2.28M; at gain
    1 the distance term inflates some Gaussians to 260M pairs)."""
    m = room_mlp(k, hidden, feat_dim, seed, scale_m)
    rng = np.random.default_rng(seed + 13)
    b = math.sqrt(6.0 / (feat_dim + 4)) * view_gain
    Wv = rng.uniform(-b, b, (hidden, 4))
    return MLP(_f32(np.concatenate([m.W1.astype(np.float64), Wv], axis=1)), m.b1, m.W2, m.b2)


def room_camera(width=1200, height=680, f=600.0, position=(0.3, 0.3, 1.5), target=(6.0, 5.0, 1.2)):
    cam = Camera(width, height, f, f, width / 2.0, height / 2.0)
    return cam, look_at(position, target)


def mask_and_codebook(n_gauss, seed=3, size=4096, dim=7, stages=2, mask_mu=2.0, mask_sigma=1.0, scale_m=0.02):
    """Mask logits ~ N(mask_mu, mask_sigma^2) and ``stages`` codebooks of
    ``size`` x ``dim`` entries (3 log-scales + 4 quaternion components) with
    uniformly drawn int32 indices.  Stage 1 codes spread around the room's
    typical shapes; later stages hold small residuals."""
    rng = np.random.default_rng(seed)
    logits = rng.normal(mask_mu, mask_sigma, n_gauss)
    books = np.empty((stages, size, dim))
    books[0, :, 0:3] = math.log(scale_m) + rng.normal(0.0, 0.3, (size, 3))
    books[0, :, 3:7] = np.array([1.0, 0.0, 0.0, 0.0]) + rng.normal(0.0, 0.5, (size, 4))
    for s in range(1, stages):
        books[s] = rng.normal(0.0, 0.05, (size, dim))
    idx = rng.integers(0, size, (stages, n_gauss))
    return _f32(logits), _f32(books), np.ascontiguousarray(idx.astype(np.int32))


def rvq_problem(kind, n, stages, codes, seed=0):
    """Vectors and starting codebooks for residual vector quantization.
    kind: "gauss" (per-Gaussian log-scale and quaternion, 7-d), "scaling"
    (anchor log-scaling, 3-d), "offset" (anchor offsets, k = 10 x 3 = 30-d) or
    "feature" (anchor features, 32-d).  Stage 1 starts from randomly picked
    input vectors; stage l > 1 from N(0, (0.35^(l-1) sigma)^2) residual codes.
    Returns (books (stages, codes, D) float32, x (n, D) float32)."""
    rng = np.random.default_rng(seed)
    if kind == "gauss":
        ls = math.log(0.02) + rng.normal(0.0, 0.3, (n, 3))
        q = np.array([1.0, 0.0, 0.0, 0.0]) + rng.normal(0.0, 0.5, (n, 4))
        q /= np.linalg.norm(q, axis=1, keepdims=True)
        x = np.concatenate([ls, q], 1)
    elif kind == "scaling":
        x = math.log(0.05) + rng.normal(0.0, 0.4, (n, 3))
    elif kind == "offset":
        x = rng.normal(0.0, 0.5, (n, 30))
    elif kind == "feature":
        x = rng.normal(0.0, 1.0, (n, 32))
    else:
        raise ValueError(kind)
    sigma = x.std(0).mean()
    D = x.shape[1]
    books = np.empty((stages, codes, D))
    books[0] = x[rng.integers(0, n, codes)] if n > 0 else rng.normal(0.0, 1.0, (codes, D))
    for l in range(1, stages):
        books[l] = rng.normal(0.0, sigma * 0.35 ** l, (codes, D))
    return _f32(books), _f32(x)


# ---------------------------------------------------------------------------
# Bundle-adjustment window and serving trace
# ---------------------------------------------------------------------------

BA_SIZES = [(320, 240), (640, 480), (1200, 680)]


def ba_window(n_views=12, seed=5, radius=1.5, height=1.5, sizes=BA_SIZES):
    """Keyframes on a circle of ``radius`` m around the room centre, looking
    outward; resolutions cycle through ``sizes``; fx = fy = W/2."""
    rng = np.random.default_rng(seed)
    phase = rng.uniform(0, 2 * math.pi)
    cams, poses = [], []
    centre = np.array([ROOM[0] / 2, ROOM[1] / 2, height])
    for i in range(n_views):
        w, h = sizes[i % len(sizes)]
        ang = phase + 2 * math.pi * i / n_views
        pos = centre + radius * np.array([math.cos(ang), math.sin(ang), 0.0])
        tgt = pos + np.array([math.cos(ang), math.sin(ang), rng.uniform(-0.2, 0.2)])
        cams.append(Camera(w, h, w / 2.0, w / 2.0, w / 2.0, h / 2.0))
        poses.append(look_at(pos, tgt))
    return cams, poses


SERVE_SIZES = [(320, 240), (640, 480), (1200, 680), (1920, 1080)]


def serve_trace(n_requests=2000, qps=100.0, seed=11, sizes=SERVE_SIZES, margin=0.3):
    """Poisson arrivals at ``qps``; each request draws its size uniformly from
    ``sizes``, its position uniformly inside the room shrunk by ``margin``,
    yaw U[0, 2pi), pitch U[-20, 20] degrees, roll 0.
    Returns a list of (arrival_s, Camera, Pose)."""
    rng = np.random.default_rng(seed)
    t = np.cumsum(rng.exponential(1.0 / qps, n_requests))
    out = []
    for i in range(n_requests):
        w, h = sizes[rng.integers(0, len(sizes))]
        pos = np.array([rng.uniform(margin, ROOM[a] - margin) for a in range(3)])
        yaw = rng.uniform(0, 2 * math.pi)
        pitch = math.radians(rng.uniform(-20, 20))
        d = np.array([math.cos(yaw) * math.cos(pitch), math.sin(yaw) * math.cos(pitch), math.sin(pitch)])
        out.append((float(t[i]), Camera(w, h, w / 2.0, w / 2.0, w / 2.0, h / 2.0), look_at(pos, pos + d)))
    return out
