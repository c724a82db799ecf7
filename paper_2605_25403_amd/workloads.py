"""Seeded synthetic workloads (inputs only; no part of the method).

The method is run on generated unit-square / unit-cube meshes with closed-form
manufactured solutions, so every input is a handful of parameters drawn from
numpy's PCG64 generator:
* Taylor-Green wave number k in {pi, 2 pi, 4 pi} and viscosity nu log-uniform
  in [1e-3, 1e-1];
* a serving request stream: Poisson arrivals at a given rate, mesh size n
  drawn from a set, and per-request (k, nu).
"""
import itertools
import math

import numpy as np

K_CHOICES = (math.pi, 2 * math.pi, 4 * math.pi)


def tg_params(seed):
    """(k, nu) for the 2D Taylor-Green workload with this seed."""
    rng = np.random.default_rng(seed)
    k = float(rng.choice(K_CHOICES))
    nu = float(10.0 ** rng.uniform(-3.0, -1.0))
    return k, nu


WORKLOADS = {
    # 16 x 16 squares (512 triangles), TG k = pi, nu = 0.01, dt = 0.01, 10 steps
    "c1": dict(dim=2, n=16, dt=0.01, steps=10, seed=None, k=math.pi, nu=0.01, tol=1e-12,
               precision="fp64"),
    # 512 x 512 squares (524,288 triangles), seed-drawn TG, dt = 1e-3, 100 steps
    "c2": dict(dim=2, n=512, dt=1e-3, steps=100, seed=0, tol=1e-12, precision="fp64"),
    # same mesh and problem in the mixed-precision form
    "c3": dict(dim=2, n=512, dt=1e-3, steps=100, seed=0, tol=1e-12, precision="mixed"),
    # 64^3 cubes x 6 Kuhn tets, Beltrami a = pi/4, d = pi/2, nu = 0.01, 50 steps
    "c4": dict(dim=3, n=64, dt=1e-3, steps=50, seed=None, nu=0.01, tol=1e-12,
               precision="mixed"),
    # the c2 problem with the P3-P2 pair on 256 x 256 squares: P3 velocity
    # (591,361 nodes per component), P2 pressure with as many nodes as c2's P1
    "c2p3": dict(dim=2, n=256, dt=1e-3, steps=100, seed=0, tol=1e-12, precision="fp64",
                 pair=1),
}


def resolve(name):
    w = dict(WORKLOADS[name])
    if w.get("seed") is not None:
        w["k"], w["nu"] = tg_params(w["seed"])
    return w


def serving_requests(seed=0, count=256, rate=20.0, sizes=(32, 64, 128, 256), steps=50,
                     dt=1e-3):
    """Request stream: arrival time (s), mesh size n, k, nu, steps, dt."""
    rng = np.random.default_rng(seed)
    arrivals = np.cumsum(rng.exponential(1.0 / rate, count))
    out = []
    for i in range(count):
        n = int(rng.choice(sizes))
        k = float(rng.choice(K_CHOICES))
        nu = float(10.0 ** rng.uniform(-3.0, -1.0))
        out.append(dict(id=i, t_arrive=float(arrivals[i]), n=n, k=k, nu=nu, steps=steps,
                        dt=dt))
    return out


def dofs(dim, n):
    """d*N2 + N1 on the structured meshes."""
    if dim == 2:
        return 2 * (2 * n + 1) ** 2 + (n + 1) ** 2
    return 3 * (2 * n + 1) ** 3 + (n + 1) ** 3


def jittered_mesh(dim, n, seed, amp=0.2):
    """Unstructured simplicial mesh of the unit square (dim 2) or cube (dim 3):
    an n^dim vertex grid whose interior vertices move by up to amp * h in each
    coordinate (uniform), with vertices relabelled at random, cells listed in a
    random order and about half of them given the opposite orientation. In 2D
    each square is cut along a diagonal picked at random; in 3D each cube gives
    the six tetrahedra around its (0,0,0)-(1,1,1) diagonal (conforming).
    Returns (x (nv, dim) float64, cells (nc, dim + 1) int32)."""
    rng = np.random.default_rng(seed)
    h = 1.0 / n
    ax = np.arange(n + 1)
    grid = np.stack(np.meshgrid(*([ax] * dim), indexing="ij"), axis=-1).reshape(-1, dim)
    x = grid * h
    inner = np.all((grid > 0) & (grid < n), axis=1)
    x[inner] += amp * h * rng.uniform(-1.0, 1.0, (int(inner.sum()), dim))
    stride = np.array([(n + 1) ** (dim - 1 - a) for a in range(dim)])
    cells = []
    for corner in itertools.product(range(n), repeat=dim):
        v0 = np.array(corner)
        if dim == 2:
            a, b, c, d = [int((v0 + o) @ stride) for o in ((0, 0), (1, 0), (1, 1), (0, 1))]
            cells += [(a, b, c), (a, c, d)] if rng.random() < 0.5 else [(a, b, d), (b, c, d)]
        else:
            for perm in itertools.permutations(range(dim)):
                path, v = [int(v0 @ stride)], v0.copy()
                for axis in perm:
                    v = v.copy()
                    v[axis] += 1
                    path.append(int(v @ stride))
                cells.append(tuple(path))
    cells = np.array(cells, dtype=np.int64)
    relabel = rng.permutation(len(x))          # old index -> new index
    xn = np.empty_like(x)
    xn[relabel] = x
    cells = relabel[cells][rng.permutation(len(cells))]
    flip = rng.random(len(cells)) < 0.5
    cells[flip] = cells[flip][:, [1, 0] + list(range(2, dim + 1))]
    return xn, cells.astype(np.int32)
