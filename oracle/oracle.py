"""Test infrastructure only: ctypes binding of the plain FP64 CPU oracle.

Only tests, ``__graft_entry__.smoke`` and the CPU-baseline leg of the
benchmark may import this module.  It builds ``liboracle.so`` from
``fr_oracle.c`` with gcc (no fused multiply-adds) and exposes the residual,
RK4 and wall-force routines on mesh dicts produced by
``paper_2501_05709_amd.workloads``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "fr_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")

_lib = None

_dp = ctypes.POINTER(ctypes.c_double)
_lp = ctypes.POINTER(ctypes.c_long)


def build(force=False):
    """Compile the oracle with gcc -O2 -ffp-contract=off -fopenmp."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        cmd = ["gcc", "-O2", "-ffp-contract=off", "-fopenmp", "-fPIC", "-shared", "-Wall",
               "-o", LIB + ".tmp", SRC, "-lm"]
        subprocess.check_call(cmd)
        os.replace(LIB + ".tmp", LIB)
    return LIB


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(LIB)
        L.orc_create.restype = ctypes.c_int
        L.orc_create.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_long, _dp,
                                 ctypes.c_long, _lp, ctypes.c_int, _dp, ctypes.c_long, _lp,
                                 ctypes.c_double, ctypes.c_double, ctypes.c_double, _dp,
                                 ctypes.POINTER(ctypes.c_void_p)]
        L.orc_create_mixed.restype = ctypes.c_int
        L.orc_create_mixed.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_int), ctypes.c_int,
                                       ctypes.c_long, _dp, ctypes.c_long, _lp, ctypes.c_int, _dp, ctypes.c_long,
                                       _lp, ctypes.c_double, ctypes.c_double, ctypes.c_double, _dp,
                                       ctypes.POINTER(ctypes.c_void_p)]
        L.orc_gradient.argtypes = [ctypes.c_void_p, _dp, _dp]
        L.orc_destroy.argtypes = [ctypes.c_void_p]
        L.orc_residual.argtypes = [ctypes.c_void_p, _dp, _dp]
        L.orc_forces.argtypes = [ctypes.c_void_p, _dp, _dp]
        L.orc_rk4.argtypes = [ctypes.c_void_p, _dp, ctypes.c_double, ctypes.c_long, _dp]
        L.orc_sizes.argtypes = [ctypes.c_void_p, _lp]
        L.orc_neighbours.argtypes = [ctypes.c_void_p, _lp]
        L.orc_solution_points.argtypes = [ctypes.c_void_p, _dp]
        L.orc_flux_points.argtypes = [ctypes.c_void_p, _dp]
        L.orc_metrics.argtypes = [ctypes.c_void_p, _dp, _dp, _dp]
        L.orc_set_mock.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_double]
        L.orc_basis.argtypes = [ctypes.c_int] + [_dp] * 7
        L.orc_num_threads.restype = ctypes.c_int
        L.orc_farfield_state.argtypes = [ctypes.c_void_p, _dp, _dp, _dp]
        _lib = L
    return _lib


def _d(a):
    return a.ctypes.data_as(_dp)


def _l(a):
    return a.ctypes.data_as(_lp)


def basis(order):
    """GL nodes, weights, D[i][j] = l_j'(x_i), l_j(-1), l_j(1), g_L'(x_i), g_R'(x_i)."""
    n = order + 1
    arrs = [np.zeros(n), np.zeros(n), np.zeros(n * n), np.zeros(n), np.zeros(n), np.zeros(n), np.zeros(n)]
    rc = lib().orc_basis(order, *[_d(a) for a in arrs])
    if rc:
        raise ValueError("unsupported order")
    xi, w, D, lm, lp, gl, gr = arrs
    return dict(xi=xi, w=w, D=D.reshape(n, n), lm=lm, lp=lp, gLd=gl, gRd=gr)


def num_threads():
    return lib().orc_num_threads()


class OracleMesh:
    """A mesh dict bound to the oracle: residual, RK4 and forces in FP64.

    A mesh with ``orders`` (one order per element) has a ragged state: arrays are
    [NU][nv] with element e's solution points contiguous, in element order."""

    def __init__(self, mesh):
        L = lib()
        self.mesh = mesh
        self.dim = int(mesh["dim"])
        self.order = int(mesh["order"])
        nodes = np.ascontiguousarray(mesh["nodes"], dtype=np.float64)
        en = np.ascontiguousarray(mesh["elem_nodes"], dtype=np.int64)
        per = np.ascontiguousarray(mesh.get("periodic", np.zeros((0, self.dim))), dtype=np.float64)
        bf = np.ascontiguousarray(mesh.get("bfaces", np.zeros((0, 3))), dtype=np.int64)
        fs = np.ascontiguousarray(mesh.get("freestream", np.array([1.0, 0, 0, 0, 1.0])), dtype=np.float64)
        self.mixed = mesh.get("orders") is not None
        orders = np.ascontiguousarray(mesh["orders"], dtype=np.int32) if self.mixed else None
        self._keep = (nodes, en, per, bf, fs, orders)
        h = ctypes.c_void_p()
        rc = L.orc_create_mixed(self.dim, self.order,
                                orders.ctypes.data_as(ctypes.POINTER(ctypes.c_int)) if self.mixed else None,
                                int(mesh["q"]), nodes.shape[0], _d(nodes),
                                en.shape[0], _l(en), per.shape[0], _d(per) if per.size else None,
                                bf.shape[0], _l(bf) if bf.size else None,
                                float(mesh.get("gamma", 1.4)), float(mesh.get("prandtl", 0.72)),
                                float(mesh.get("mu", 0.0)), _d(fs), ctypes.byref(h))
        if rc != 0:
            raise ValueError(f"oracle rejected the mesh (code {rc})")
        self.h = h
        sz = np.zeros(10, dtype=np.int64)
        L.orc_sizes(h, _l(sz))
        _, _, self.nu, self.nf, self.nv, self.E, self.nfp, self.NU, self.NF, self.n_mortar = (int(v) for v in sz)

    def __del__(self):
        if getattr(self, "h", None):
            lib().orc_destroy(self.h)
            self.h = None

    @property
    def shape(self):
        return (self.NU, self.nv) if self.mixed else (self.E, self.nu, self.nv)

    def _pts(self, per_elem, total):
        return (total,) if self.mixed else (self.E, per_elem)

    def solution_points(self):
        x = np.zeros(self._pts(self.nu, self.NU) + (3,))
        lib().orc_solution_points(self.h, _d(x))
        return x

    def flux_points(self):
        x = np.zeros(self._pts(self.nf, self.NF) + (3,))
        lib().orc_flux_points(self.h, _d(x))
        return x

    def neighbours(self):
        nb = np.zeros(self._pts(self.nf, self.NF), dtype=np.int64)
        lib().orc_neighbours(self.h, _l(nb))
        return nb

    def metrics(self):
        detJ = np.zeros(self._pts(self.nu, self.NU))
        fA = np.zeros(self._pts(self.nf, self.NF))
        fn = np.zeros(self._pts(self.nf, self.NF) + (3,))
        lib().orc_metrics(self.h, _d(detJ), _d(fA), _d(fn))
        return detJ, fA, fn

    def gradient(self, u):
        """Corrected physical gradient at the solution points: [..., 3, nv]."""
        u = np.ascontiguousarray(u, dtype=np.float64).reshape(self.shape)
        g = np.zeros(self.shape[:-1] + (3, self.nv))
        lib().orc_gradient(self.h, _d(u), _d(g))
        return g

    def initial_state(self):
        xyz = self.solution_points().reshape(-1, 3)
        return np.ascontiguousarray(self.mesh["init"](xyz).reshape(self.shape))

    def residual(self, u):
        u = np.ascontiguousarray(u, dtype=np.float64).reshape(self.shape)
        r = np.zeros(self.shape)
        lib().orc_residual(self.h, _d(u), _d(r))
        return r

    def forces(self, u):
        u = np.ascontiguousarray(u, dtype=np.float64).reshape(self.shape)
        F = np.zeros(3)
        lib().orc_forces(self.h, _d(u), _d(F))
        return F

    def rk4(self, u, dt, nsteps, forces=False):
        u = np.array(u, dtype=np.float64).reshape(self.shape)
        hist = np.zeros((nsteps, 3)) if forces else None
        lib().orc_rk4(self.h, _d(u), float(dt), int(nsteps), _d(hist) if forces else None)
        return (u, hist) if forces else u

    def farfield_state(self, uL, nrm):
        uL = np.ascontiguousarray(uL, dtype=np.float64)
        n3 = np.zeros(3)
        n3[:len(nrm)] = nrm
        ub = np.zeros(self.nv)
        lib().orc_farfield_state(self.h, _d(uL), _d(n3), _d(ub))
        return ub

    def set_mock(self, lam):
        lib().orc_set_mock(self.h, 1, float(lam))
