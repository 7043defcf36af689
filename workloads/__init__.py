"""Seeded synthetic inputs for the SNeRG render path.

Everything here is input generation: block-sparse grids (Section 5.1 of the
paper: an indirection grid of (N/B)^3 entries over an atlas of B^3
macroblocks), pinhole cameras (Appendix B: 39 degree horizontal field of
view at 800x800, 53 degrees for the forward-facing 1006x756 captures) and
He-initialised weights for the 34->16->16->3 deferred shading MLP
(Section 4.2).  None of the rendering arithmetic lives here; the oracle and
the GPU library both consume these arrays.

Seeds follow one convention everywhere: grid = 0, cameras = 1, MLP = 2,
perturbations and ray minibatches = 3.

The paper measures on the Blender "Synthetic 360" scenes and real captures.
Those datasets and the trained, baked SNeRGs are not available here; the
procedural shell below stands in for them with the same shapes: grid sizes
512^3 / 1024^3 (paper: 500^3 .. 1000^3), B = 32, thin opaque shells around a
surface (what the sparsity loss of Section 4.3 produces) and the paper's
image sizes and fields of view.
"""
from __future__ import annotations

import ctypes
import dataclasses
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libshellgen.so")
_lib = None

SEED_GRID, SEED_CAMERA, SEED_MLP, SEED_PERTURB = 0, 1, 2, 3

MLP_IN, MLP_HIDDEN, MLP_OUT = 34, 16, 3
SIGMA_SCALE = 50.0  # sigma = 50 * byte / 255


def build_shellgen() -> str:
    """Compiles the C shell generator next to this file (gcc, OpenMP)."""
    cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared",
           "-o", _LIB_PATH, os.path.join(_HERE, "shellgen.c"), "-lm"]
    subprocess.check_call(cmd)
    return _LIB_PATH


def _shellgen():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build_shellgen()
        lib = ctypes.CDLL(_LIB_PATH)
        lib.shellgen_occupancy.restype = ctypes.c_int64
        lib.shellgen_occupancy.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_double,
                                           ctypes.c_double, ctypes.c_double, ctypes.c_uint64,
                                           ctypes.c_void_p]
        lib.shellgen_fill.restype = ctypes.c_int
        lib.shellgen_fill.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_double,
                                      ctypes.c_double, ctypes.c_double, ctypes.c_uint64,
                                      ctypes.c_uint64, ctypes.c_void_p, ctypes.c_int32,
                                      ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
        lib.shellgen_dense.restype = ctypes.c_int
        lib.shellgen_dense.argtypes = [ctypes.c_int32, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                       ctypes.c_uint64, ctypes.c_uint64, ctypes.c_double, ctypes.c_double,
                                       ctypes.c_int32, ctypes.c_double, ctypes.c_void_p, ctypes.c_void_p,
                                       ctypes.c_void_p]
        _lib = lib
    return _lib


@dataclasses.dataclass
class Grid:
    """A SNeRG in canonical layout.

    indirection: int32 [(N/B)^3], x fastest; -1 = empty macroblock, else atlas id.
    dens: uint8 [n_blocks, B, B, B]   (z, y, x), density byte; sigma = 50 * byte / 255
    rgb:  uint8 [n_blocks, B, B, B, 3] diffuse colour byte / 255
    feat: uint8 [n_blocks, B, B, B, 4] feature byte / 255
    """
    N: int
    B: int
    indirection: np.ndarray
    dens: np.ndarray
    rgb: np.ndarray
    feat: np.ndarray
    meta: dict = dataclasses.field(default_factory=dict)

    @property
    def G(self) -> int:
        return self.N // self.B

    @property
    def n_blocks(self) -> int:
        return int(self.dens.shape[0])

    def atlas_bytes(self) -> int:
        return int(self.dens.nbytes + self.rgb.nbytes + self.feat.nbytes)


def tiny_grid(N: int = 64, B: int = 8, n_occupied: int = 8, zero_frac: float = 0.25,
              seed: int = SEED_GRID) -> Grid:
    """Random blocks: `n_occupied` macroblocks chosen uniformly without
    replacement, atlas ids assigned by a seeded permutation; density bytes
    uniform on 0..255 with `zero_frac` of them forced to 0; colour and
    feature bytes uniform on 0..255."""
    rng = np.random.default_rng(seed)
    G = N // B
    chosen = rng.choice(G ** 3, size=n_occupied, replace=False)
    ids = rng.permutation(n_occupied)
    ind = np.full(G ** 3, -1, dtype=np.int32)
    ind[chosen] = ids.astype(np.int32)
    dens = rng.integers(0, 256, size=(n_occupied, B, B, B), dtype=np.uint8)
    dens[rng.random(dens.shape) < zero_frac] = 0
    rgb = rng.integers(0, 256, size=(n_occupied, B, B, B, 3), dtype=np.uint8)
    feat = rng.integers(0, 256, size=(n_occupied, B, B, B, 4), dtype=np.uint8)
    return Grid(N, B, ind, dens, rgb, feat, meta=dict(kind="random_blocks", seed=seed,
                                                      n_occupied=n_occupied, zero_frac=zero_frac))


def grid_from_dense(dens: np.ndarray, rgb: np.ndarray, feat: np.ndarray, B: int,
                    permute_seed: int | None = None) -> Grid:
    """Builds the block-sparse grid of a dense N^3 field (arrays indexed
    [z, y, x(, c)]); a macroblock is stored when any of its density bytes is
    non-zero.  Atlas ids follow scan order, or a seeded permutation."""
    N = dens.shape[0]
    G = N // B
    d = dens.reshape(G, B, G, B, G, B).transpose(0, 2, 4, 1, 3, 5)  # bz,by,bx,z,y,x
    occ = (d.reshape(G, G, G, -1) != 0).any(axis=-1).reshape(-1)
    lin = np.nonzero(occ)[0]
    n = len(lin)
    ids = np.arange(n, dtype=np.int32)
    if permute_seed is not None:
        ids = np.random.default_rng(permute_seed).permutation(n).astype(np.int32)
    ind = np.full(G ** 3, -1, dtype=np.int32)
    ind[lin] = ids
    out_d = np.zeros((n, B, B, B), np.uint8)
    out_r = np.zeros((n, B, B, B, 3), np.uint8)
    out_f = np.zeros((n, B, B, B, 4), np.uint8)
    r = rgb.reshape(G, B, G, B, G, B, 3).transpose(0, 2, 4, 1, 3, 5, 6)
    f = feat.reshape(G, B, G, B, G, B, 4).transpose(0, 2, 4, 1, 3, 5, 6)
    for li, bid in zip(lin, ids):
        bz, by, bx = li // (G * G), (li // G) % G, li % G
        out_d[bid] = d[bz, by, bx]
        out_r[bid] = r[bz, by, bx]
        out_f[bid] = f[bz, by, bx]
    return Grid(N, B, ind, out_d, out_r, out_f, meta=dict(kind="dense", permute_seed=permute_seed))


def shell_grid(N: int, B: int, amplitude: float, seed: int = SEED_GRID, r0: float = 0.6,
               base_freq: float = 4.0) -> Grid:
    """Procedural shell (sphere of radius r0 with 3-octave value-noise
    displacement of the given amplitude); density bytes form a tent three
    voxels wide around the surface, colour and feature bytes are uniform
    over every voxel of an occupied block.  Atlas ids follow scan order."""
    lib = _shellgen()
    G = N // B
    occ = np.zeros(G ** 3, dtype=np.uint8)
    n = lib.shellgen_occupancy(N, B, r0, amplitude, base_freq, seed, occ.ctypes.data)
    if n < 0:
        raise MemoryError("shell generator: allocation failed")
    ind = np.full(G ** 3, -1, dtype=np.int32)
    lin = np.nonzero(occ)[0]
    ind[lin] = np.arange(len(lin), dtype=np.int32)
    dens = np.empty((n, B, B, B), np.uint8)
    rgb = np.empty((n, B, B, B, 3), np.uint8)
    feat = np.empty((n, B, B, B, 4), np.uint8)
    rc = lib.shellgen_fill(N, B, r0, amplitude, base_freq, seed, seed + 1000, ind.ctypes.data,
                           int(n), dens.ctypes.data, rgb.ctypes.data, feat.ctypes.data)
    if rc != 0:
        raise RuntimeError(f"shell generator failed ({rc})")
    return Grid(N, B, ind, dens, rgb, feat,
                meta=dict(kind="shell", seed=seed, amplitude=amplitude, r0=r0, base_freq=base_freq,
                          occupancy=float(n) / G ** 3))


@dataclasses.dataclass
class DenseField:
    """A densely evaluated radiance field (what Section 5.3 bakes from):
    sigma float32 [N, N, N] ([z, y, x]; density per unit length of the world
    box), rgb float32 [N, N, N, 3] and feat float32 [N, N, N, 4] in [0, 1]."""
    N: int
    sigma: np.ndarray
    rgb: np.ndarray
    feat: np.ndarray
    meta: dict = dataclasses.field(default_factory=dict)


def dense_shell_field(N: int, amplitude: float = 0.08, seed: int = SEED_GRID, r0: float = 0.6,
                      base_freq: float = 4.0, sigma_max: float = 1000.0, haze: float = 0.2,
                      n_blobs: int = 12, blob_r: float = 0.08) -> DenseField:
    """Stand-in for a trained NeRF evaluated on the full N^3 grid: an opaque
    displaced shell (the surface of shell_grid, density a tent of height
    sigma_max three voxels wide), n_blobs dense balls inside it that no
    outside camera can see, and a faint haze everywhere (alpha below the
    empty-space threshold at the paper's grid sizes).  Colour and features
    follow the same hash as shell_grid's bytes, divided by 255."""
    lib = _shellgen()
    sigma = np.empty((N, N, N), np.float32)
    rgb = np.empty((N, N, N, 3), np.float32)
    feat = np.empty((N, N, N, 4), np.float32)
    rc = lib.shellgen_dense(N, r0, amplitude, base_freq, seed, seed + 1000, sigma_max, haze, n_blobs, blob_r,
                            sigma.ctypes.data, rgb.ctypes.data, feat.ctypes.data)
    if rc != 0:
        raise RuntimeError(f"dense field generator failed ({rc})")
    return DenseField(N, sigma, rgb, feat, meta=dict(kind="dense_shell", seed=seed, amplitude=amplitude, r0=r0,
                                                     sigma_max=sigma_max, haze=haze, n_blobs=n_blobs,
                                                     blob_r=blob_r))


# --------------------------------------------------------------------------- cameras

@dataclasses.dataclass
class Camera:
    """Pinhole camera: pixel (i, j) (column, row from the top) looks along
    fwd + x*right - y*up with x = (i + 1/2 - W/2)/focal, y = (j + 1/2 - H/2)/focal."""
    eye: np.ndarray
    fwd: np.ndarray
    right: np.ndarray
    up: np.ndarray
    W: int
    H: int
    focal: float

    @property
    def n_rays(self) -> int:
        return self.W * self.H


def look_at(eye, W: int, H: int, fov_deg: float, target=(0.0, 0.0, 0.0)) -> Camera:
    """Camera at `eye` looking at `target`, world up +z (+y when the view is
    within about 8 degrees of vertical); `fov_deg` is the horizontal field of view."""
    eye = np.asarray(eye, dtype=np.float64)
    fwd = np.asarray(target, dtype=np.float64) - eye
    fwd /= np.linalg.norm(fwd)
    up_w = np.array([0.0, 0.0, 1.0]) if abs(fwd[2]) <= 0.99 else np.array([0.0, 1.0, 0.0])
    right = np.cross(fwd, up_w)
    right /= np.linalg.norm(right)
    up = np.cross(right, fwd)
    focal = 0.5 * W / math.tan(0.5 * math.radians(fov_deg))
    return Camera(eye, fwd, right, up, int(W), int(H), float(focal))


def orbit_eye(radius: float, elevation_deg: float, azimuth_rad: float) -> np.ndarray:
    e = math.radians(elevation_deg)
    return radius * np.array([math.cos(e) * math.cos(azimuth_rad),
                              math.cos(e) * math.sin(azimuth_rad), math.sin(e)])


def orbit_camera(W: int, H: int, fov_deg: float = 39.0, seed: int = SEED_CAMERA,
                 radius: float = 2.0, elevation_deg: float = 30.0) -> Camera:
    a = float(np.random.default_rng(seed).uniform(0.0, 2.0 * math.pi))
    return look_at(orbit_eye(radius, elevation_deg, a), W, H, fov_deg)


def sphere_cameras(sizes, seed: int = SEED_CAMERA, radius: float = 2.0):
    """One camera per (W, H, fov_deg) entry, eyes uniform on the sphere."""
    rng = np.random.default_rng(seed)
    cams = []
    for (W, H, fov) in sizes:
        v = rng.normal(size=3)
        v /= np.linalg.norm(v)
        cams.append(look_at(radius * v, W, H, fov))
    return cams


# --------------------------------------------------------------------------- MLP

@dataclasses.dataclass
class MLP:
    """Deferred shading network: W1 [16, 34], W2 [16, 16], W3 [3, 16] ([out][in]), biases."""
    W1: np.ndarray
    b1: np.ndarray
    W2: np.ndarray
    b2: np.ndarray
    W3: np.ndarray
    b3: np.ndarray

    def params(self):
        return [self.W1, self.b1, self.W2, self.b2, self.W3, self.b3]

    def flat(self) -> np.ndarray:
        return np.concatenate([p.reshape(-1) for p in self.params()]).astype(np.float32)

    @staticmethod
    def from_flat(v) -> "MLP":
        v = np.asarray(v, dtype=np.float32)
        shapes = [(16, 34), (16,), (16, 16), (16,), (3, 16), (3,)]
        out, o = [], 0
        for s in shapes:
            n = int(np.prod(s))
            out.append(v[o:o + n].reshape(s).copy())
            o += n
        return MLP(*out)


MLP_N_PARAMS = 16 * 34 + 16 + 16 * 16 + 16 + 3 * 16 + 3  # 883


def mlp_weights(seed: int = SEED_MLP) -> MLP:
    """He-normal weights (std sqrt(2/fan_in)), biases uniform on [-0.1, 0.1], float32."""
    rng = np.random.default_rng(seed)

    def he(o, i):
        return (rng.normal(size=(o, i)) * math.sqrt(2.0 / i)).astype(np.float32)

    def bias(o):
        return rng.uniform(-0.1, 0.1, size=o).astype(np.float32)

    W1 = he(16, 34); b1 = bias(16)
    W2 = he(16, 16); b2 = bias(16)
    W3 = he(3, 16); b3 = bias(3)
    return MLP(W1, b1, W2, b2, W3, b3)


def perturbed(mlp: MLP, grid: Grid, seed: int = SEED_PERTURB, rel: float = 0.05):
    """Perturbed copy for synthetic fine-tuning targets: features scaled by
    (1 + rel*U[-1,1]) and clamped to [0,1] (returned as float32 normalised
    features), weights moved by rel*std(W)*N(0,1)."""
    rng = np.random.default_rng(seed)
    f = grid.feat.astype(np.float32) / 255.0
    f = np.clip(f * (1.0 + rel * rng.uniform(-1.0, 1.0, size=f.shape).astype(np.float32)), 0.0, 1.0)
    ps = []
    for p in mlp.params():
        sd = float(p.std()) if p.size > 1 else 0.0
        ps.append((p + rel * sd * rng.normal(size=p.shape)).astype(np.float32))
    return MLP(*ps), f.astype(np.float32)


# --------------------------------------------------------------------------- configurations

# Shell amplitudes for the target block occupancies at seed 0: 512^3 -> 10.6%
# (433 blocks), 1024^3 at 0.02 -> 5.8% (1908 blocks), 1024^3 at 0.12 -> 8.1%
# (2667 blocks).  The measured occupancy is recorded in the grid's meta.
SHELL_AMPLITUDE = {"plain512": 0.02, "batched1024": 0.02, "large1024": 0.12}

BATCHED_SIZES = [(400, 400, 39.0)] * 4 + [(800, 800, 39.0)] * 8 + [(1008, 756, 53.0)] * 4


def config(name: str) -> dict:
    """Named workloads: grid, cameras, MLP and the render options they use."""
    if name == "tiny":
        g = tiny_grid()
        cams = [orbit_camera(64, 64)]
        return dict(name=name, grid=g, cams=cams, mlp=mlp_weights(), fp16=False)
    if name == "plain512":
        g = shell_grid(512, 32, SHELL_AMPLITUDE["plain512"])
        return dict(name=name, grid=g, cams=[orbit_camera(800, 800)], mlp=mlp_weights(), fp16=False)
    if name == "batched1024":
        g = shell_grid(1024, 32, SHELL_AMPLITUDE["batched1024"])
        return dict(name=name, grid=g, cams=sphere_cameras(BATCHED_SIZES), mlp=mlp_weights(),
                    fp16=True)
    if name == "adjoint512":
        g = shell_grid(512, 32, SHELL_AMPLITUDE["plain512"])
        cams = sphere_cameras([(800, 800, 39.0)] * 8)
        return dict(name=name, grid=g, cams=cams, mlp=mlp_weights(), fp16=False)
    if name == "large1024":
        g = shell_grid(1024, 32, SHELL_AMPLITUDE["large1024"])
        cams = sphere_cameras([(1920, 1080, 39.0)] * 64)
        return dict(name=name, grid=g, cams=cams, mlp=mlp_weights(), fp16=True)
    raise KeyError(name)
