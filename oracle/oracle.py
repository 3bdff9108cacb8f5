"""FP64 CPU oracle for the FMM-ForceAtlas2 / Kamada-Kawai layout method.

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, by the smoke check and by the
benchmark's CPU-baseline leg, never by the product path.  It shares no code
with the HIP library (``paper_2403_03504_amd``) and does not import it.

The heavy loops live in ``fa2_oracle.c`` (plain C, FP64, OpenMP over target
nodes); this module holds the parts that are a few lines of NumPy.  Section
references are to "Graph Visualization for Blockchain Data" (Dietl et al.).

Readings taken where the paper is silent (each is a parameter):

* repulsion is degree-weighted as in ForceAtlas2: ``kr (deg_i+1)(deg_j+1)/d``;
  the mass of a node is ``deg + 1`` with ``deg`` = distinct neighbours;
* attraction is linear and unweighted (sec. 3.2: proportional to distance);
* gravity is "strong" and mass-weighted about the origin by default
  (sec. 3.2: proportional to the distance to the centre);
* swing and traction are the unweighted sums the paper prints (sec. 3.2);
  the ForceAtlas2 variant (mass-weighted, traction halved) is ``swing_mode=1``;
* the step size follows ForceAtlas2 (Jacomy et al. 2014), which the paper
  defers to: ``s_G = tau * tra / swg`` capped to rise at most ``max_rise`` per
  iteration, ``s_i = ks s_G / (1 + s_G sqrt(swg_i))`` capped at ``ksmax/|F_i|``.
"""
from __future__ import annotations

import ctypes
import dataclasses
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "fa2_oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

GRAV_STRONG_MASS, GRAV_FA2_CONST, GRAV_STRONG_UNIT = 0, 1, 2
SWING_PAPER, SWING_FA2 = 0, 1


def build(force: bool = False) -> str:
    """Compile the C part with gcc (FP64, no fast-math, OpenMP)."""
    if force or not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        subprocess.run(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-fno-fast-math",
                        "-ffp-contract=off", "-o", tmp, _SRC, "-lm"], check=True)
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(_LIB_PATH)
        P = ctypes.c_void_p
        i64, i32, f64 = ctypes.c_int64, ctypes.c_int32, ctypes.c_double
        L.orc_repulsion_exact.argtypes = [i64, P, P, P, f64, i64, P, P, P]
        L.orc_components.argtypes = [i64, P, P, P]
        L.orc_components.restype = i64
        L.orc_bfs_hops.argtypes = [i32, P, P, P]
        L.orc_root.argtypes = [i64, P, P, ctypes.c_int, P]
        L.orc_morton.argtypes = [i64, P, P, ctypes.c_int, P]
        L.orc_sort_by_key.argtypes = [i64, P, P]
        L.orc_tree.argtypes = [i64, P, ctypes.c_int, ctypes.c_int, i64, P]
        L.orc_tree.restype = i64
        L.orc_fmm_repulsion.argtypes = [i64, P, P, P, f64, ctypes.c_int, ctypes.c_int, ctypes.c_int, P, P, P]
        L.orc_fmm_repulsion.restype = ctypes.c_int
        L.orc_fmm_lists.argtypes = [i64, P, P, ctypes.c_int, ctypes.c_int, P, P, P, P, P, P, P, P]
        L.orc_fmm_lists.restype = i64
        L.orc_kk_energy.argtypes = [i32, P, f64, P, P]
        L.orc_kk_energy.restype = f64
        L.orc_kk_steps.argtypes = [i32, P, f64, i32, P, P]
        L.orc_kk_grad_hess.argtypes = [i32, P, f64, i32, P, P, P]
        L.orc_kk_newton.argtypes = [i32, P, f64, f64, i32, i32, P, P]
        L.orc_kk_newton.restype = i32
        L.orc_bh_repulsion.argtypes = [i64, P, P, P, f64, f64, ctypes.c_int, ctypes.c_int, i64, P, P, P]
        L.orc_bh_repulsion.restype = ctypes.c_int
        L.orc_stress.argtypes = [i32, P, P, P]
        L.orc_stress.restype = f64
        L.orc_kk_sweeps.argtypes = [i32, P, i32, P, P]
        L.orc_num_threads.restype = ctypes.c_int
        for nm in ("orc_op_m2m", "orc_op_m2l", "orc_op_l2l"):
            getattr(L, nm).argtypes = [P, P, f64, f64, ctypes.c_int, P, P]
        L.orc_op_p2m.argtypes = [i64, P, P, P, f64, f64, ctypes.c_int, P, P]
        L.orc_op_l2p.argtypes = [P, P, f64, f64, ctypes.c_int, P]
        L.orc_op_m2p.argtypes = [P, P, f64, f64, ctypes.c_int, P]
        L.orc_op_p2l.argtypes = [f64, f64, f64, ctypes.c_int, P, P]
        _lib = L
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


def num_threads() -> int:
    return int(lib().orc_num_threads())


# --- graph preparation (sec. 2 and sec. 4) -----------------------------------

def build_csr(n: int, src, dst):
    """Simple undirected graph in CSR: directions ignored, duplicate pairs and
    self loops dropped, each row sorted ascending (sec. 4: components are
    taken ignoring edge directions; an address may be both input and output of
    one transaction, which is one adjacency).  Returns (row_ptr int64,
    col int32, deg int32)."""
    s = np.asarray(src, dtype=np.int64)
    d = np.asarray(dst, dtype=np.int64)
    if s.size and (s.min() < 0 or d.min() < 0 or s.max() >= n or d.max() >= n):
        raise ValueError("edge endpoint out of range")
    u = np.concatenate([s, d])
    v = np.concatenate([d, s])
    keep = u != v
    pairs = np.unique(u[keep] * n + v[keep])
    rows = pairs // n
    cols = (pairs % n).astype(np.int32)
    deg = np.bincount(rows, minlength=n).astype(np.int32)
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(deg, out=row_ptr[1:])
    return row_ptr, cols, deg


def components(row_ptr, col):
    """label[v] = smallest node id in v's component (sec. 4)."""
    n = row_ptr.shape[0] - 1
    rp = np.ascontiguousarray(row_ptr, dtype=np.int64)
    c = np.ascontiguousarray(col, dtype=np.int32)
    lab = np.empty(n, dtype=np.int32)
    k = lib().orc_components(n, _p(rp), _p(c), _p(lab))
    return lab, int(k)


# --- forces (sec. 3.2) --------------------------------------------------------

def masses(deg) -> np.ndarray:
    return np.asarray(deg, dtype=np.float64) + 1.0


def repulsion_exact(x, y, m, kr: float = 1.0, targets=None):
    """Exact pairwise repulsion kr m_i m_j (p_i - p_j)/|p_i - p_j|^2 (O(n^2))."""
    x, y, m = _f64(x), _f64(y), _f64(m)
    n = x.shape[0]
    if targets is None:
        nt, tp = n, None
    else:
        t = np.ascontiguousarray(targets, dtype=np.int64)
        nt, tp = t.shape[0], _p(t)
    fx = np.empty(nt)
    fy = np.empty(nt)
    lib().orc_repulsion_exact(n, _p(x), _p(y), _p(m), float(kr), nt, tp, _p(fx), _p(fy))
    return fx, fy


def repulsion_fmm(x, y, m, kr: float = 1.0, p: int = 8, leaf_size: int = 64, bits: int = 16,
                  with_stats: bool = False):
    """The paper's FMM repulsion (sec. 3.2.1) in FP64."""
    x, y, m = _f64(x), _f64(y), _f64(m)
    n = x.shape[0]
    fx = np.empty(n)
    fy = np.empty(n)
    st = np.zeros(12, dtype=np.int64)
    rc = lib().orc_fmm_repulsion(n, _p(x), _p(y), _p(m), float(kr), int(p), int(leaf_size), int(bits),
                                 _p(fx), _p(fy), _p(st))
    if rc != 0:
        raise ValueError("invalid FMM parameters")
    if with_stats:
        keys = ("cells", "leaves", "max_level", "near_pairs", "v_entries", "w_entries", "x_entries",
                "coverage_min", "coverage_max", "u_entries", "w_entries2", "x_entries2")
        return fx, fy, dict(zip(keys, (int(v) for v in st)))
    return fx, fy


def repulsion_bh(x, y, m, kr: float = 1.0, theta: float = 0.5, leaf_size: int = 64, bits: int = 16,
                 targets=None):
    """Barnes-Hut repulsion (the comparator of sec. 3.2.1) on the FMM's
    quadtree: a cell not holding the target with side < theta * distance to
    its centre of mass acts as one particle.  theta = 0 is the exact sum."""
    x, y, m = _f64(x), _f64(y), _f64(m)
    n = x.shape[0]
    tg = None if targets is None else np.ascontiguousarray(targets, dtype=np.int64)
    nt = n if tg is None else tg.shape[0]
    fx, fy = np.zeros(nt), np.zeros(nt)
    rc = lib().orc_bh_repulsion(n, _p(x), _p(y), _p(m), float(kr), float(theta), int(leaf_size), int(bits), nt,
                                None if tg is None else _p(tg), _p(fx), _p(fy))
    if rc != 0:
        raise ValueError("bad Barnes-Hut arguments")
    return fx, fy


def attraction(row_ptr, col, x, y, ka: float = 1.0):
    """Linear attraction along every edge: F_a,i = ka sum_{j in N(i)} (p_j - p_i)."""
    x, y = _f64(x), _f64(y)
    n = x.shape[0]
    deg = np.diff(np.asarray(row_ptr, dtype=np.int64))
    rows = np.repeat(np.arange(n), deg)
    col = np.asarray(col, dtype=np.int64)
    fx = np.bincount(rows, weights=x[col] - x[rows], minlength=n)
    fy = np.bincount(rows, weights=y[col] - y[rows], minlength=n)
    return ka * fx, ka * fy


def gravity(x, y, m, kg: float = 1.0, mode: int = GRAV_STRONG_MASS):
    """Gravity towards the origin, proportional to the distance (sec. 3.2)."""
    x, y, m = _f64(x), _f64(y), _f64(m)
    if mode == GRAV_STRONG_MASS:
        return -kg * m * x, -kg * m * y
    if mode == GRAV_STRONG_UNIT:
        return -kg * x, -kg * y
    if mode == GRAV_FA2_CONST:
        r = np.hypot(x, y)
        s = np.where(r > 0, -kg * m / np.where(r > 0, r, 1.0), 0.0)
        return s * x, s * y
    raise ValueError("unknown gravity mode")


@dataclasses.dataclass
class FA2Params:
    kr: float = 1.0
    kg: float = 1.0
    ka: float = 1.0
    gravity_mode: int = GRAV_STRONG_MASS
    swing_mode: int = SWING_PAPER
    tau: float = 1.0
    ks: float = 0.1
    ksmax: float = 10.0
    max_rise: float = 0.5
    repulsion: str = "exact"  # "exact" | "fmm"
    p: int = 8
    leaf_size: int = 64
    bits: int = 16


def forces(row_ptr, col, deg, x, y, prm: FA2Params = FA2Params()):
    """(F_r, F_a, F_g) of every node, each an (fx, fy) pair."""
    m = masses(deg)
    if prm.repulsion == "fmm":
        fr = repulsion_fmm(x, y, m, prm.kr, prm.p, prm.leaf_size, prm.bits)
    else:
        fr = repulsion_exact(x, y, m, prm.kr)
    fa = attraction(row_ptr, col, x, y, prm.ka)
    fg = gravity(x, y, m, prm.kg, prm.gravity_mode)
    return fr, fa, fg


def swing_traction(fx, fy, fpx, fpy, m, mode: int = SWING_PAPER):
    """Per-node swing |F_t - F_{t-1}| and traction |F_t + F_{t-1}| and their
    sums (sec. 3.2).  Returns (swg_i, tra_i, SWG, TRA)."""
    fx, fy, fpx, fpy = _f64(fx), _f64(fy), _f64(fpx), _f64(fpy)
    swg = np.hypot(fx - fpx, fy - fpy)
    tra = np.hypot(fx + fpx, fy + fpy)
    if mode == SWING_FA2:
        w = _f64(m)
        return swg, tra, float(np.sum(w * swg)), float(np.sum(w * tra) / 2.0)
    return swg, tra, float(np.sum(swg)), float(np.sum(tra))


def global_speed(SWG: float, TRA: float, s_prev: float, it: int, prm: FA2Params) -> float:
    """s_G = tau TRA / SWG, at most (1 + max_rise) s_prev after the first
    iteration; SWG = 0 gives 1 on the first iteration and the capped value
    afterwards."""
    if SWG > 0.0:
        s = prm.tau * TRA / SWG
        if it > 0:
            s = min(s, (1.0 + prm.max_rise) * s_prev)
        return s
    return 1.0 if it == 0 else (1.0 + prm.max_rise) * s_prev


def node_speed(swg_i, fx, fy, s_g: float, prm: FA2Params):
    """s_i = ks s_G / (1 + s_G sqrt(swg_i)), capped at ksmax / |F_i|."""
    s = prm.ks * s_g / (1.0 + s_g * np.sqrt(swg_i))
    fn = np.hypot(_f64(fx), _f64(fy))
    cap = np.where(fn > 0, prm.ksmax / np.where(fn > 0, fn, 1.0), np.inf)
    return np.minimum(s, cap)


def fa2_step(row_ptr, col, deg, x, y, fpx, fpy, s_prev: float, it: int, prm: FA2Params = FA2Params(),
             given_forces=None):
    """One ForceAtlas2 iteration (sec. 3.2): forces at the current positions,
    swing and traction against the previous forces, global then per-node step
    size, and the move p += s_i F_i.  With ``it == 0`` the previous forces are
    taken as zero.  ``given_forces`` = (fx, fy) replaces the force evaluation
    (to check the update given identical forces).  Returns a dict."""
    m = masses(deg)
    if given_forces is None:
        fr, fa, fg = forces(row_ptr, col, deg, x, y, prm)
        fx = fr[0] + fa[0] + fg[0]
        fy = fr[1] + fa[1] + fg[1]
    else:
        fx, fy = _f64(given_forces[0]), _f64(given_forces[1])
    if it == 0:
        fpx = np.zeros_like(fx)
        fpy = np.zeros_like(fy)
    swg_i, tra_i, SWG, TRA = swing_traction(fx, fy, fpx, fpy, m, prm.swing_mode)
    s_g = global_speed(SWG, TRA, s_prev, it, prm)
    s_i = node_speed(swg_i, fx, fy, s_g, prm)
    nx = _f64(x) + s_i * fx
    ny = _f64(y) + s_i * fy
    return dict(x=nx, y=ny, fx=fx, fy=fy, swg=SWG, tra=TRA, speed=s_g, s_i=s_i)


# --- Morton order and quadtree (sec. 3.2.1) -----------------------------------

def root_square(x, y, bits: int = 16):
    x, y = _f64(x), _f64(y)
    out = np.empty(4)
    lib().orc_root(x.shape[0], _p(x), _p(y), int(bits), _p(out))
    return out  # xmin, ymin, L, S


def morton(x, y, bits: int = 16) -> np.ndarray:
    x, y = _f64(x), _f64(y)
    k = np.empty(x.shape[0], dtype=np.uint64)
    lib().orc_morton(x.shape[0], _p(x), _p(y), int(bits), _p(k))
    return k


def sort_by_key(key) -> np.ndarray:
    k = np.ascontiguousarray(key, dtype=np.uint64)
    perm = np.empty(k.shape[0], dtype=np.int64)
    lib().orc_sort_by_key(k.shape[0], _p(k), _p(perm))
    return perm


def tree(sorted_keys, bits: int = 16, leaf_size: int = 64) -> np.ndarray:
    """Cells as an int32 array [ncell, 10]: level, ix, iy, begin, end, parent,
    child0..3, in (level, Morton prefix) order."""
    k = np.ascontiguousarray(sorted_keys, dtype=np.uint64)
    cap = max(16, 4 * k.shape[0] + 16)
    out = np.empty((cap, 10), dtype=np.int32)
    c = lib().orc_tree(k.shape[0], _p(k), int(bits), int(leaf_size), cap, _p(out))
    if c < 0:
        raise RuntimeError("tree capacity")
    return out[:c].copy()


def fmm_lists(x, y, leaf_size: int = 64, bits: int = 16):
    """Tree and the U/V/W/X lists of the FMM for these positions."""
    x, y = _f64(x), _f64(y)
    n = x.shape[0]
    caps = np.array([4 * n + 16, 64 * n + 64, 64 * n + 64, 64 * n + 64, 64 * n + 64], dtype=np.int64)
    while True:
        cells = np.empty((caps[0], 10), dtype=np.int32)
        ptrs = np.empty(4 * (caps[0] + 1), dtype=np.int64)
        U = np.empty(caps[1], dtype=np.int32)
        V = np.empty(caps[2], dtype=np.int32)
        W = np.empty(caps[3], dtype=np.int32)
        X = np.empty(caps[4], dtype=np.int32)
        lens = np.zeros(5, dtype=np.int64)
        r = lib().orc_fmm_lists(n, _p(x), _p(y), int(leaf_size), int(bits), _p(caps), _p(cells), _p(ptrs),
                                _p(U), _p(V), _p(W), _p(X), _p(lens))
        if r >= 0:
            break
        caps = np.maximum(caps, lens + 16)
    nc = int(lens[0])
    pt = ptrs[:4 * (nc + 1)].reshape(4, nc + 1)
    return dict(cells=cells[:nc].copy(), U=(pt[0].copy(), U[:lens[1]].copy()), V=(pt[1].copy(), V[:lens[2]].copy()),
                W=(pt[2].copy(), W[:lens[3]].copy()), X=(pt[3].copy(), X[:lens[4]].copy()))


# --- FMM operators, exposed for tests (complex as re/im FP64 arrays) ---------

def _cz(p):
    return np.zeros(p + 1), np.zeros(p + 1)


def op_p2m(zx, zy, q, cx, cy, p):
    zx, zy, q = _f64(zx), _f64(zy), _f64(q)
    re, im = _cz(p)
    lib().orc_op_p2m(zx.shape[0], _p(zx), _p(zy), _p(q), float(cx), float(cy), int(p), _p(re), _p(im))
    return re + 1j * im


def _op3(name, a, z0, p, acc=None):
    are, aim = _f64(np.real(a)), _f64(np.imag(a))
    if acc is None:
        bre, bim = _cz(p)
    else:
        bre, bim = _f64(np.real(acc)).copy(), _f64(np.imag(acc)).copy()
    getattr(lib(), name)(_p(are), _p(aim), float(np.real(z0)), float(np.imag(z0)), int(p), _p(bre), _p(bim))
    return bre + 1j * bim


def op_m2m(a, z0, p, acc=None):
    return _op3("orc_op_m2m", a, z0, p, acc)


def op_m2l(a, z0, p, acc=None):
    return _op3("orc_op_m2l", a, z0, p, acc)


def op_l2l(b, z0, p, acc=None):
    return _op3("orc_op_l2l", b, z0, p, acc)


def op_l2p(b, d, p):
    bre, bim = _f64(np.real(b)), _f64(np.imag(b))
    out = np.empty(2)
    lib().orc_op_l2p(_p(bre), _p(bim), float(np.real(d)), float(np.imag(d)), int(p), _p(out))
    return out[0] + 1j * out[1]


def op_m2p(a, d, p):
    are, aim = _f64(np.real(a)), _f64(np.imag(a))
    out = np.empty(2)
    lib().orc_op_m2p(_p(are), _p(aim), float(np.real(d)), float(np.imag(d)), int(p), _p(out))
    return out[0] + 1j * out[1]


def op_p2l(q, z0, p, acc=None):
    if acc is None:
        bre, bim = _cz(p)
    else:
        bre, bim = _f64(np.real(acc)).copy(), _f64(np.imag(acc)).copy()
    lib().orc_op_p2l(float(q), float(np.real(z0)), float(np.imag(z0)), int(p), _p(bre), _p(bim))
    return bre + 1j * bim


# --- Kamada-Kawai (sec. 3.1) ---------------------------------------------------

def hop_distances(row_ptr, col) -> np.ndarray:
    """All-pairs hop distances of a graph with local ids (BFS per source)."""
    n = row_ptr.shape[0] - 1
    rp = np.ascontiguousarray(row_ptr, dtype=np.int64)
    c = np.ascontiguousarray(col, dtype=np.int32)
    d = np.empty((n, n), dtype=np.int32)
    lib().orc_bfs_hops(n, _p(rp), _p(c), _p(d))
    return d


def floyd_warshall(n: int, row_ptr, col) -> np.ndarray:
    """The paper's all-pairs shortest path algorithm (sec. 3.1), unit weights;
    used only to cross-check the breadth-first distances on tiny graphs."""
    INF = np.iinfo(np.int64).max // 4
    d = np.full((n, n), INF, dtype=np.int64)
    np.fill_diagonal(d, 0)
    for i in range(n):
        for e in range(row_ptr[i], row_ptr[i + 1]):
            d[i, col[e]] = 1
    for k in range(n):
        d = np.minimum(d, d[:, k:k + 1] + d[k:k + 1, :])
    d[d >= INF] = -1
    return d.astype(np.int32)


def kk_energy(dist, x, y, l: float = 1.0) -> float:
    d = np.ascontiguousarray(dist, dtype=np.int32)
    x, y = _f64(x), _f64(y)
    return float(lib().orc_kk_energy(d.shape[0], _p(d), float(l), _p(x), _p(y)))


def kk_steps(dist, x, y, l: float = 1.0, steps: int = 1):
    d = np.ascontiguousarray(dist, dtype=np.int32)
    x, y = _f64(x).copy(), _f64(y).copy()
    lib().orc_kk_steps(d.shape[0], _p(d), float(l), int(steps), _p(x), _p(y))
    return x, y


def kk_grad_hess(dist, x, y, m: int, l: float = 1.0):
    """Gradient (gx, gy) and Hessian (hxx, hxy, hyy) of the KK energy in the
    position of node m."""
    d = np.ascontiguousarray(dist, dtype=np.int32)
    out = np.zeros(5)
    lib().orc_kk_grad_hess(d.shape[0], _p(d), float(l), int(m), _p(_f64(x)), _p(_f64(y)), _p(out))
    return out


def kk_newton(dist, x, y, l: float = 1.0, eps: float = 1e-4, moves: int = 1000, inner: int = 16):
    """Kamada-Kawai's Newton-Raphson minimiser (sec. 3.1) with the safeguards of
    fa2_oracle.c (positive-definite check, step halving); stops when every
    gradient norm is below eps * l.  Returns (x, y, moves made)."""
    d = np.ascontiguousarray(dist, dtype=np.int32)
    x, y = _f64(x).copy(), _f64(y).copy()
    k = lib().orc_kk_newton(d.shape[0], _p(d), float(l), float(eps), int(moves), int(inner), _p(x), _p(y))
    return x, y, int(k)


# --- Cluster / decluster for Kamada-Kawai (sec. 3.1) ---------------------------
#
# Readings (the paper gives the two ideas in a sentence each):
# * a node of degree 1 whose neighbour has degree >= 2 is contracted into the
#   neighbour (one round; a 2-node component keeps both nodes);
# * among the remaining nodes, those with exactly two remaining neighbours
#   form chains; a chain whose two ends are distinct kept nodes is replaced
#   by one edge as long as the chain (its nodes removed).  Chains that close
#   a loop, pure cycles, and every chain but the one with the smallest node
#   id between the same two ends are kept;
# * both reductions keep the shortest-path distances between the remaining
#   nodes, so the layout of the reduced graph is Kamada-Kawai on the kept
#   nodes with their hop distances in the full component;
# * declustering: the i-th node (1..k) of a removed chain from end a (the end
#   with the smaller id) to end b goes to p_a + i/(k+1) (p_b - p_a); then the
#   contracted leaves of node v, j-th of k in id order, go to distance l from
#   p_v: at angle phi + (j - (k-1)/2) pi/k, phi the direction from the centre
#   of gravity c of the placed nodes to p_v, or, where p_v is that centre
#   (|p_v - c| <= 1e-4 (R + l), R the largest |p - c| of a placed node, so
#   that rounding cannot decide a symmetric case), at angle 2 pi j / k.


def kk_reduce(row_ptr, col, leaves: bool = True, chains: bool = True):
    """Which nodes of one component (local ids) the reductions remove and how
    to place them again.  Returns (kept mask, chain records (node, a, b, i,
    k), leaf records (node, v, j, k))."""
    rp = np.asarray(row_ptr, dtype=np.int64)
    cl = np.asarray(col, dtype=np.int64)
    n = rp.shape[0] - 1
    nb = [list(cl[rp[i]:rp[i + 1]]) for i in range(n)]
    deg = [len(v) for v in nb]
    leaf = [leaves and deg[i] == 1 and deg[nb[i][0]] >= 2 for i in range(n)]
    rest = [[j for j in nb[i] if not leaf[j]] for i in range(n)]
    mid = [chains and not leaf[i] and len(rest[i]) == 2 for i in range(n)]
    removed = [False] * n
    seen = [False] * n
    found = []  # (ends, chain nodes from the smaller end)
    for s in range(n):
        if not mid[s] or seen[s]:
            continue
        # walk both ways from s through chain nodes
        sides = []
        for first in rest[s]:
            path, prev, cur = [], s, first
            while mid[cur] and cur != s:
                path.append(cur)
                nxt = rest[cur][0] if rest[cur][0] != prev else rest[cur][1]
                prev, cur = cur, nxt
            sides.append((path, cur))
        (p0, e0), (p1, e1) = sides
        if e0 == s:  # a pure cycle
            for v in [s] + p0:
                seen[v] = True
            continue
        nodes = list(reversed(p0)) + [s] + p1  # from end e0 to end e1
        for v in nodes:
            seen[v] = True
        if e0 == e1:
            continue  # a loop
        a, b = (e0, e1) if e0 < e1 else (e1, e0)
        if a != e0:
            nodes.reverse()
        found.append(((a, b), nodes))
    best = {}
    for ends, nodes in found:
        if ends not in best or min(nodes) < min(best[ends]):
            best[ends] = nodes
    chain_rec = []
    for (a, b), nodes in best.items():
        k = len(nodes)
        for i, v in enumerate(nodes, start=1):
            removed[v] = True
            chain_rec.append((v, a, b, i, k))
    leaf_rec = []
    for v in range(n):
        lv = sorted(u for u in nb[v] if leaf[u])
        for j, u in enumerate(lv):
            leaf_rec.append((u, v, j, len(lv)))
    kept = np.array([not leaf[i] and not removed[i] for i in range(n)])
    return kept, chain_rec, leaf_rec


def kk_reduced_layout(row_ptr, col, x, y, l: float = 1.0, minimiser: str = "majorization", steps: int = 200,
                      eps: float = 1e-3, leaves: bool = True, chains: bool = True):
    """Kamada-Kawai of one component with the reductions of sec. 3.1 (the
    readings above): lay out the kept nodes, then decluster."""
    D = hop_distances(row_ptr, col)
    kept, chain_rec, leaf_rec = kk_reduce(row_ptr, col, leaves, chains)
    K = np.nonzero(kept)[0]
    DK = np.ascontiguousarray(D[np.ix_(K, K)])
    X, Y = _f64(x).copy(), _f64(y).copy()
    if minimiser == "newton":
        xk, yk, _ = kk_newton(DK, X[K], Y[K], l, eps, steps * K.shape[0])
    else:
        xk, yk = kk_steps(DK, X[K], Y[K], l, steps)
    X[K], Y[K] = xk, yk
    for v, a, b, i, k in chain_rec:
        t = i / (k + 1)
        X[v] = X[a] + t * (X[b] - X[a])
        Y[v] = Y[a] + t * (Y[b] - Y[a])
    placed = np.ones(X.shape[0], dtype=bool)
    for u, _, _, _ in leaf_rec:
        placed[u] = False
    cx, cy = np.mean(X[placed]), np.mean(Y[placed])
    R = np.max(np.hypot(X[placed] - cx, Y[placed] - cy))
    for u, v, j, k in leaf_rec:
        dx, dy = X[v] - cx, Y[v] - cy
        if math.hypot(dx, dy) <= 1e-4 * (R + l):
            ang = 2.0 * math.pi * j / k
        else:
            ang = math.atan2(dy, dx) + (j - (k - 1) / 2.0) * math.pi / k
        X[u] = X[v] + l * math.cos(ang)
        Y[u] = Y[v] + l * math.sin(ang)
    return X, Y, kept


def rel_err(ax, ay, bx, by) -> float:
    """Norm-wise relative error |a - b|_2 / |b|_2 over all components."""
    num = np.sqrt(np.sum((_f64(ax) - _f64(bx)) ** 2 + (_f64(ay) - _f64(by)) ** 2))
    den = np.sqrt(np.sum(_f64(bx) ** 2 + _f64(by) ** 2))
    return float(num / den) if den > 0 else float(num)


# --- Assembling the component layouts into one figure (sec. 4) ----------------
#
# Readings taken where the paper is silent:
#
# * density: a component's nodes are taken to fill a uniform disc with the
#   same second moment about their centroid.  A uniform disc of radius a has
#   mean squared distance a^2/2 from its centre, so the equivalent disc of a
#   component whose RMS distance from its centroid is rho has area
#   2 pi rho^2; the component is scaled about its centroid by s so that
#   n / (2 pi (s rho)^2) equals the target density.  rho = 0 (one node, or all
#   nodes coincident): s = 1.
# * diameter: twice the radius R of the smallest circle about the centroid
#   that holds every node, so a meta-edge is R_a + R_b + gap long.
# * "largest" component: the most nodes; on a tie the one earliest in the
#   order.
# * "small enough" / "divide it": the order is cut into consecutive groups of
#   at most max_group components; each group gets its own meta-graph (built
#   by the same rule inside the group) and Kamada-Kawai layout; the groups,
#   in the order they were cut, are then the components of the next level
#   (their node counts add up; centre = node-weighted centroid of their
#   members; radius = the smallest circle about that centre holding the
#   members' circles), until one group remains.
# * starting layout of a group's Kamada-Kawai: item t at distance d(0, t)
#   from the origin at angle 2 pi t / g (the first item at the origin).
# * the energy of a meta-graph with real edge lengths has no extra length
#   scale and is minimised by sequential localized stress majorization
#   (orc_kk_sweeps); the finished drawing is translated so that the centroid
#   of all nodes is the origin.


@dataclasses.dataclass
class AssembleParams:
    density: float = 1.0   # target nodes per unit area
    gap: float = 1.0       # constant added to every meta-edge length (> 0)
    max_group: int = 256   # largest meta-graph laid out in one piece
    sweeps: int = 100      # majorization sweeps per meta-graph


def component_frames(x, y, comp_offsets, density: float):
    """Centroid (K, 2), scale s (K) and radius R after scaling (K) of every
    component (node ranges comp_offsets), per the density reading above."""
    x, y = _f64(x), _f64(y)
    off = np.asarray(comp_offsets, dtype=np.int64)
    K = off.shape[0] - 1
    cen = np.zeros((K, 2))
    scale = np.ones(K)
    rad = np.zeros(K)
    for k in range(K):
        a, b = off[k], off[k + 1]
        n = b - a
        cx, cy = np.sum(x[a:b]) / n, np.sum(y[a:b]) / n
        r2 = (x[a:b] - cx) ** 2 + (y[a:b] - cy) ** 2
        rho = math.sqrt(np.sum(r2) / n)
        s = math.sqrt(n / (2.0 * math.pi * density)) / rho if rho > 0.0 else 1.0
        cen[k] = (cx, cy)
        scale[k] = s
        rad[k] = s * math.sqrt(np.max(r2))
    return cen, scale, rad


def meta_tree(weight, radius, gap: float):
    """Meta-graph of one group, items in their (random) order: item t > 0 is
    linked to the largest of items 0..t-1 by an edge of half the two
    diameters summed plus gap.  Returns (parent, edge length); parent[0] = -1."""
    w = np.asarray(weight)
    R = _f64(radius)
    g = w.shape[0]
    parent = np.full(g, -1, dtype=np.int64)
    elen = np.zeros(g)
    for t in range(1, g):
        q = int(np.argmax(w[:t]))  # first of the largest
        parent[t] = q
        elen[t] = (2.0 * R[t] + 2.0 * R[q]) / 2.0 + gap
    return parent, elen


def tree_distances(parent, elen) -> np.ndarray:
    """All-pairs shortest path lengths of the weighted meta-graph by the
    paper's all-pairs algorithm (Floyd-Warshall, sec. 3.1)."""
    g = len(parent)
    d = np.full((g, g), np.inf)
    np.fill_diagonal(d, 0.0)
    for t in range(g):
        if parent[t] >= 0:
            d[t, parent[t]] = d[parent[t], t] = elen[t]
    for k in range(g):
        d = np.minimum(d, d[:, k:k + 1] + d[k:k + 1, :])
    return d


def meta_initial(dist):
    """Starting positions of a group's Kamada-Kawai (reading above)."""
    g = dist.shape[0]
    t = np.arange(g)
    ang = 2.0 * math.pi * t / g
    return dist[0] * np.cos(ang), dist[0] * np.sin(ang)


def stress(dist, x, y) -> float:
    d = _f64(dist)
    return float(lib().orc_stress(d.shape[0], _p(d), _p(_f64(x)), _p(_f64(y))))


def kk_sweeps(dist, x, y, sweeps: int = 1):
    d = _f64(dist)
    x, y = _f64(x).copy(), _f64(y).copy()
    lib().orc_kk_sweeps(d.shape[0], _p(d), int(sweeps), _p(x), _p(y))
    return x, y


@dataclasses.dataclass
class Assembly:
    x: np.ndarray          # assembled positions
    y: np.ndarray
    centroid: np.ndarray   # (K, 2) centroid of each component before
    scale: np.ndarray      # (K,)
    radius: np.ndarray     # (K,) after scaling
    shift: np.ndarray      # (K, 2): node p of component k goes to s_k (p - c_k) + shift_k
    parent: np.ndarray     # (K,) component linked to in the first-level meta-graph, -1 for a group's first
    levels: int
    groups: int            # groups over all levels


def assemble(x, y, comp_offsets, order, prm: AssembleParams = AssembleParams()) -> Assembly:
    """Rescale every component to the common density, then place the
    components by Kamada-Kawai on the meta-graph (sec. 4), level by level as
    described above.  order: the random order, a permutation of 0..K-1."""
    off = np.asarray(comp_offsets, dtype=np.int64)
    K = off.shape[0] - 1
    order = np.asarray(order, dtype=np.int64)
    assert sorted(order.tolist()) == list(range(K)), "order must be a permutation"
    assert prm.gap > 0.0 and prm.density > 0.0 and prm.max_group >= 2
    cen, scale, rad = component_frames(x, y, off, prm.density)
    nodes = (off[1:] - off[:-1]).astype(np.int64)

    # level items: weight (nodes), centre before placement, radius
    w_it = nodes[order]
    c_it = np.zeros((K, 2))  # scaled components sit about their own centroid
    r_it = rad[order]
    levels = []  # per level: (group start offsets, placed positions P, centres C)
    parent0 = np.full(K, -1, dtype=np.int64)
    n_groups = 0
    while True:
        m = w_it.shape[0]
        starts = list(range(0, m, prm.max_group)) + [m]
        P = np.zeros((m, 2))
        nw, nc, nr = [], [], []
        for a, b in zip(starts[:-1], starts[1:]):
            par, el = meta_tree(w_it[a:b], r_it[a:b], prm.gap)
            if not levels:
                for t in range(1, b - a):
                    parent0[order[a + t]] = order[a + par[t]]
            D = tree_distances(par, el)
            px, py = meta_initial(D)
            px, py = kk_sweeps(D, px, py, prm.sweeps)
            P[a:b, 0], P[a:b, 1] = px, py
            W = np.sum(w_it[a:b])
            C = (np.sum(w_it[a:b] * px) / W, np.sum(w_it[a:b] * py) / W)
            Rg = np.max(np.hypot(px - C[0], py - C[1]) + r_it[a:b])
            nw.append(W)
            nc.append(C)
            nr.append(Rg)
        n_groups += len(starts) - 1
        levels.append((starts, P, c_it))
        if len(starts) == 2:
            top_centre = np.array(nc[0])
            break
        w_it, c_it, r_it = np.array(nw, dtype=np.int64), np.array(nc), np.array(nr)

    # translations, top down: an item moves by (placement - own centre) plus
    # the move of the group holding it; the whole drawing by -centroid
    F = -top_centre[None, :]
    for starts, P, C in reversed(levels):
        m = P.shape[0]
        grp = np.zeros(m, dtype=np.int64)
        for gi, (a, b) in enumerate(zip(starts[:-1], starts[1:])):
            grp[a:b] = gi
        F = P - C + F[grp]
    shift = np.zeros((K, 2))
    shift[order] = F

    xs, ys = _f64(x).copy(), _f64(y).copy()
    for k in range(K):
        a, b = off[k], off[k + 1]
        xs[a:b] = scale[k] * (xs[a:b] - cen[k, 0]) + shift[k, 0]
        ys[a:b] = scale[k] * (ys[a:b] - cen[k, 1]) + shift[k, 1]
    return Assembly(xs, ys, cen, scale, rad, shift, parent0, len(levels), n_groups)
