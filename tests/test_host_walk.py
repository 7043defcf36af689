"""The march's macroblock walks, run on the host (tests/host_walk.cpp, built
by build()): the single-loop walk with incremental macroblock stepping that
the render and adjoint kernels use visits exactly the samples of the nested
walk, whose visits the GPU tests pin bit-exactly to the oracle; and the
split centre-ray cost count adds up to the whole ray's count."""
import ctypes
import os

import numpy as np
import pytest

import workloads as W

LIB = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libhostwalk.so")
P = ctypes.c_void_p


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        raise RuntimeError(f"{LIB} is missing: run build() (tests/hostbuild.py)")
    L = ctypes.CDLL(LIB)
    L.walk_flat_vs_nested.restype = ctypes.c_int64
    L.walk_flat_vs_nested.argtypes = [ctypes.c_int, ctypes.c_int, P, ctypes.c_int, P, ctypes.c_int, ctypes.c_int,
                                      ctypes.c_uint32, P]
    L.walk_cost_parts.restype = ctypes.c_int64
    L.walk_cost_parts.argtypes = [ctypes.c_int, ctypes.c_int, P, ctypes.c_int, P, ctypes.c_int, ctypes.c_int, P]
    return L


def _cam(c):
    return np.concatenate([c.eye, c.fwd, c.right, c.up, [c.focal]]).astype(np.float64)


def _cases(n_random, seed):
    """Tiny grids of several N and B, cameras outside and inside the grid,
    and axis-aligned rays along macroblock faces and edges."""
    rng = np.random.default_rng(seed)
    shapes = [(64, 8), (64, 4), (128, 32), (64, 64), (96, 32), (32, 2), (256, 16)]
    for trial in range(n_random):
        N, B = shapes[trial % len(shapes)]
        G = N // B
        g = W.tiny_grid(N=N, B=B, n_occupied=min(G ** 3, int(rng.integers(1, 200))), seed=trial)
        eye = rng.normal(size=3)
        eye = eye / np.linalg.norm(eye) * rng.uniform(1.2, 3.5)
        if trial % 4 == 1:
            eye = rng.uniform(-0.9, 0.9, 3)
        cam = W.look_at(eye, int(rng.integers(5, 32)), int(rng.integers(5, 32)), float(rng.uniform(10, 120)),
                        target=rng.uniform(-0.5, 0.5, 3))
        yield g, cam
    for N, B in [(64, 8), (64, 4), (128, 32)]:
        g = W.tiny_grid(N=N, B=B, n_occupied=min((N // B) ** 3, 60), seed=99)
        for axis in range(3):
            for sign in (1, -1):
                for off in (0.0, 0.5, 6.0 / N):
                    e = np.zeros(3)
                    e[axis] = -2.0 * sign
                    e[(axis + 1) % 3] = -1 + 2.0 * (8 + off * N / 2) / N
                    e[(axis + 2) % 3] = -1 + 2.0 * B / N
                    fwd = np.zeros(3)
                    fwd[axis] = sign
                    up = np.zeros(3)
                    up[(axis + 2) % 3] = 1.0
                    yield g, W.Camera(e, fwd, np.cross(fwd, up), up, 9, 9, 40.0)


def test_flat_walk_visits_the_nested_walks_samples(lib):
    bad = rays = samples = 0
    for i, (g, cam) in enumerate(_cases(70, 1)):
        ind = np.ascontiguousarray(g.indirection, np.int32)
        c = _cam(cam)
        ns = ctypes.c_int64(0)
        bad += lib.walk_flat_vs_nested(g.N, g.B, ind.ctypes.data, g.n_blocks, c.ctypes.data, cam.W, cam.H,
                                       i + 1, ctypes.byref(ns))
        rays += cam.W * cam.H
        samples += ns.value
    assert samples > 100_000  # the cases do reach occupied blocks
    assert bad == 0, f"{bad} of {rays} rays differ"


def test_large_grid_walks_agree(lib):
    # N = 1024 and 4096: long walks, many faces per ray
    rng = np.random.default_rng(5)
    bad = samples = 0
    for N, B, nb in [(1024, 8, 4000), (4096, 64, 300)]:
        g = W.tiny_grid(N=N, B=B, n_occupied=nb, seed=N)
        for inside in (False, True):
            eye = rng.uniform(-0.9, 0.9, 3) if inside else np.array([1.9, 0.7, 1.3])
            cam = W.look_at(eye, 24, 24, 25.0, target=rng.uniform(-0.3, 0.3, 3))
            ind = np.ascontiguousarray(g.indirection, np.int32)
            c = _cam(cam)
            ns = ctypes.c_int64(0)
            bad += lib.walk_flat_vs_nested(g.N, g.B, ind.ctypes.data, g.n_blocks, c.ctypes.data, cam.W, cam.H, 7,
                                           ctypes.byref(ns))
            samples += ns.value
    assert samples > 0
    assert bad == 0


def test_cost_parts_add_up(lib):
    bad = rays = samples = 0
    for g, cam in _cases(40, 2):
        ind = np.ascontiguousarray(g.indirection, np.int32)
        c = _cam(cam)
        ns = ctypes.c_int64(0)
        bad += lib.walk_cost_parts(g.N, g.B, ind.ctypes.data, g.n_blocks, c.ctypes.data, cam.W, cam.H,
                                   ctypes.byref(ns))
        rays += cam.W * cam.H
        samples += ns.value
    assert samples > 100_000
    assert bad == 0, f"{bad} of {rays} rays differ"
