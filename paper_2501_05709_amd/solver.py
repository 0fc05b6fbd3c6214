"""Python handles over the C ABI: one mesh, a batch of designs, a request pool.

Argument marshalling only.  Every step of the solve runs in libfr.so's
kernels; torch provides the device allocator and the HIP streams.
"""
from __future__ import annotations

import atexit
import ctypes
import weakref

import numpy as np

from . import _lib
from ._lib import FR_FP32, FR_FP64, MeshDesc, check

PRECISION = {"fp64": FR_FP64, "fp32": FR_FP32}

# live handles, closed before interpreter teardown (their device memory may
# belong to torch's allocator, which must still be alive to take it back)
_LIVE = weakref.WeakSet()


@atexit.register
def _close_all():
    for h in list(_LIVE):
        try:
            h.close()
        except Exception:
            pass


class _TorchAllocator:
    """Routes the library's device allocations through torch's caching allocator."""

    def __init__(self, device):
        import torch
        self.torch = torch
        self.device = device

        def _alloc(nbytes, ctx, stream):
            try:
                return torch.cuda.caching_allocator_alloc(int(nbytes), self.device, stream)
            except Exception:
                return None

        def _free(ptr, ctx, stream):
            try:
                torch.cuda.caching_allocator_delete(ptr)
            except Exception:
                pass  # interpreter teardown: the process releases device memory

        self.alloc = _lib.ALLOC_FN(_alloc)
        self.free = _lib.FREE_FN(_free)


def _desc(mesh, precision, device=0, stream=None, allocator=None):
    d = MeshDesc()
    keep = []
    nodes = np.ascontiguousarray(mesh["nodes"], dtype=np.float64)
    en = np.ascontiguousarray(mesh["elem_nodes"], dtype=np.int64)
    dim = int(mesh["dim"])
    per = np.ascontiguousarray(mesh.get("periodic", np.zeros((0, dim))), dtype=np.float64).reshape(-1, dim)
    bf = np.ascontiguousarray(mesh.get("bfaces", np.zeros((0, 3))), dtype=np.int64).reshape(-1, 3)
    keep += [nodes, en, per, bf]
    d.dim = dim
    d.order = int(mesh["order"])
    d.geom_order = int(mesh["q"])
    d.precision = PRECISION[precision] if isinstance(precision, str) else int(precision)
    d.n_nodes = nodes.shape[0]
    d.nodes = nodes.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    d.n_elems = en.shape[0]
    d.elem_nodes = en.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))
    d.n_periodic = per.shape[0]
    d.periodic_shift = per.ctypes.data_as(ctypes.POINTER(ctypes.c_double)) if per.size else None
    d.n_bfaces = bf.shape[0]
    d.bfaces = bf.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)) if bf.size else None
    d.gamma = float(mesh.get("gamma", 1.4))
    d.prandtl = float(mesh.get("prandtl", 0.72))
    d.mu = float(mesh.get("mu", 0.0))
    fs = np.asarray(mesh.get("freestream", [1.0, 0, 0, 0, 1.0]), dtype=np.float64)
    for i in range(5):
        d.freestream[i] = fs[i]
    d.ref_area = float(mesh.get("ref_area", 1.0))
    for i, v in enumerate(mesh.get("lift_dir", [0.0, 1.0, 0.0])):
        d.lift_dir[i] = v
    for i, v in enumerate(mesh.get("drag_dir", [1.0, 0.0, 0.0])):
        d.drag_dir[i] = v
    d.dt = float(mesh.get("dt", 1e-3))
    if mesh.get("orders") is not None:
        orders = np.ascontiguousarray(mesh["orders"], dtype=np.int32)
        if orders.shape != (en.shape[0],):
            raise ValueError("one order per element expected")
        keep.append(orders)
        d.elem_order = orders.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
    d.device = device
    d.stream = stream
    if allocator is not None:
        d.alloc = allocator.alloc
        d.free = allocator.free
    return d, keep


def _new_stream(device):
    import torch
    return torch.cuda.Stream(device=device)


class FRMesh:
    """A solver handle for one mesh (``meshes`` = a single dict) or a batch (list of dicts)."""

    def __init__(self, meshes, precision="fp64", device=0, use_torch_allocator=True, stream=None):
        L = _lib.load()
        single = isinstance(meshes, dict)
        meshes = [meshes] if single else list(meshes)
        self.meshes = meshes
        self.stream_obj = stream if stream is not None else _new_stream(device)
        sptr = ctypes.c_void_p(self.stream_obj.cuda_stream)
        self.allocator = _TorchAllocator(device) if use_torch_allocator else None
        descs = (MeshDesc * len(meshes))()
        self._keep = []
        for i, m in enumerate(meshes):
            d, keep = _desc(m, precision, device, sptr, self.allocator)
            descs[i] = d
            self._keep.append(keep)
        h = ctypes.c_void_p()
        if single:
            check(L.fr_mesh_create(descs, ctypes.byref(h)), "fr_mesh_create")
        else:
            check(L.fr_batch_create(descs, len(meshes), ctypes.byref(h)), "fr_batch_create")
        self.h = h
        _LIVE.add(self)
        info = self.info()
        self.dim, self.order, self.n_designs, self.E, self.nu, self.nf, self.nv = (int(v) for v in info[:7])
        self.nblk = int(info[8])
        npts = ctypes.c_int64()
        check(L.fr_mesh_points(self.h, ctypes.byref(npts)), "fr_mesh_points")
        self.n_points = npts.value
        self.mixed = any(m.get("orders") is not None for m in meshes)

    def close(self):
        if getattr(self, "h", None):
            _lib.load().fr_mesh_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def shape(self):
        """Canonical state shape: [E][n_u][nv], or [points][nv] for a variable-order mesh."""
        return (self.n_points, self.nv) if self.mixed else (self.E, self.nu, self.nv)

    def info(self):
        out = np.zeros(10, dtype=np.int64)
        check(_lib.load().fr_mesh_info(self.h, out.ctypes.data_as(_lib._i64p)), "fr_mesh_info")
        return out

    def design_range(self, d):
        a, b = ctypes.c_int64(), ctypes.c_int64()
        check(_lib.load().fr_design_range(self.h, d, ctypes.byref(a), ctypes.byref(b)), "fr_design_range")
        return a.value, b.value

    def solution_points(self):
        x = np.zeros(self.shape[:-1] + (3,))
        check(_lib.load().fr_solution_points(self.h, x.ctypes.data_as(_lib._dp)), "fr_solution_points")
        return x

    def neighbours(self):
        nb = np.zeros((self.E, self.nf), dtype=np.int64)
        check(_lib.load().fr_neighbours(self.h, nb.ctypes.data_as(_lib._i64p)), "fr_neighbours")
        return nb

    def set_state(self, u):
        u = np.ascontiguousarray(u, dtype=np.float64).reshape(self.shape)
        check(_lib.load().fr_set_state(self.h, u.ctypes.data_as(_lib._dp)), "fr_set_state")

    def get_state(self):
        u = np.zeros(self.shape)
        check(_lib.load().fr_get_state(self.h, u.ctypes.data_as(_lib._dp)), "fr_get_state")
        return u

    def step(self, n):
        check(_lib.load().fr_step(self.h, int(n)), "fr_step")

    def step_async(self, n):
        check(_lib.load().fr_step_async(self.h, int(n)), "fr_step_async")

    def sync(self):
        check(_lib.load().fr_sync(self.h), "fr_sync")

    def forces(self, design=0):
        out = np.zeros(8)
        check(_lib.load().fr_forces(self.h, design, out.ctypes.data_as(_lib._dp)), "fr_forces")
        return out

    def residual(self, u):
        u = np.ascontiguousarray(u, dtype=np.float64).reshape(self.shape)
        r = np.zeros(self.shape)
        check(_lib.load().fr_residual(self.h, u.ctypes.data_as(_lib._dp), r.ctypes.data_as(_lib._dp)),
              "fr_residual")
        return r

    def select_kernels(self, mask):
        """Bit 0: fused two-launch stage.  Else bit k (2 grad, 3 visc, 4 divrk, 5 interp):
        sum-factorised variant of that split kernel; clear: dense MFMA."""
        check(_lib.load().fr_select_kernels(self.h, int(mask)), "fr_select_kernels")

    def selected_kernels(self):
        m = ctypes.c_int32()
        check(_lib.load().fr_selected_kernels(self.h, ctypes.byref(m)), "fr_selected_kernels")
        return m.value

    def autotune(self, steps=3):
        m = ctypes.c_int32()
        check(_lib.load().fr_autotune(self.h, int(steps), ctypes.byref(m)), "fr_autotune")
        return m.value

    def profile_kernels(self, steps):
        ms = np.zeros(8)
        n = np.zeros(8, dtype=np.int64)
        check(_lib.load().fr_profile_kernels(self.h, int(steps), ms.ctypes.data_as(_lib._dp),
                                             n.ctypes.data_as(_lib._i64p)), "fr_profile_kernels")
        return ms, n


def connectivity(mesh):
    """Host-only neighbour table and solution points of one mesh (no device needed)."""
    d, keep = _desc(mesh, FR_FP64)
    E, dim, n = len(mesh["elem_nodes"]), int(mesh["dim"]), int(mesh["order"]) + 1
    nf = 2 * dim * n ** (dim - 1)
    nb = np.zeros((E, nf), dtype=np.int64)
    x = np.zeros((E, n ** dim, 3))
    check(_lib.load().fr_connectivity(ctypes.byref(d), nb.ctypes.data_as(_lib._i64p), x.ctypes.data_as(_lib._dp)),
          "fr_connectivity")
    return nb, x


def footprint(mesh, precision="fp32"):
    d, keep = _desc(mesh, precision)
    out = ctypes.c_size_t()
    check(_lib.load().fr_footprint(ctypes.byref(d), ctypes.byref(out)), "fr_footprint")
    return out.value


class FRPool:
    """Continuous-batching request pool with an HBM budget."""

    def __init__(self, budget_bytes, device=0):
        h = ctypes.c_void_p()
        check(_lib.load().fr_pool_create(int(budget_bytes), device, ctypes.byref(h)), "fr_pool_create")
        self.h = h
        _LIVE.add(self)

    def close(self):
        if getattr(self, "h", None):
            _lib.load().fr_pool_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def admit(self, mesh, steps, precision="fp32", u0=None):
        """Returns the slot id, or None if the request does not fit now."""
        d, keep = _desc(mesh, precision)
        slot = ctypes.c_int64()
        up = None
        if u0 is not None:
            u0 = np.ascontiguousarray(u0, dtype=np.float64)
            up = u0.ctypes.data_as(_lib._dp)
        rc = _lib.load().fr_pool_admit(self.h, ctypes.byref(d), up, int(steps), ctypes.byref(slot))
        if rc == _lib.FR_E_NOMEM:
            return None
        check(rc, "fr_pool_admit")
        return slot.value

    def admit_sampled(self, mesh, surface, warmup, every, n_samples, precision="fp32", u0=None):
        """A request whose flow is sampled on a data surface and fed to an FW-H record.

        surface: dict of points [n, 3], normals [n, 3], areas [n], and optionally
        n_copies and copy_shift.  Runs warmup + (n_samples - 1) * every steps.
        Returns the slot id, or None if the request does not fit now."""
        d, keep = _desc(mesh, precision)
        pts = np.ascontiguousarray(surface["points"], dtype=np.float64).reshape(-1, 3)
        nrm = np.ascontiguousarray(surface["normals"], dtype=np.float64).reshape(-1, 3)
        area = np.ascontiguousarray(surface["areas"], dtype=np.float64).reshape(-1)
        if nrm.shape != pts.shape or area.shape[0] != pts.shape[0]:
            raise ValueError("surface points, normals and areas differ in count")
        s = _lib.PoolSurface()
        s.n_points = pts.shape[0]
        s.points, s.normals, s.areas = (a.ctypes.data_as(_lib._dp) for a in (pts, nrm, area))
        s.n_copies = int(surface.get("n_copies", 1))
        s.copy_shift[:] = [float(v) for v in surface.get("copy_shift", (0.0, 0.0, 0.0))]
        s.warmup, s.every, s.n_samples = int(warmup), int(every), int(n_samples)
        slot = ctypes.c_int64()
        up = None
        if u0 is not None:
            u0 = np.ascontiguousarray(u0, dtype=np.float64)
            up = u0.ctypes.data_as(_lib._dp)
        rc = _lib.load().fr_pool_admit_sampled(self.h, ctypes.byref(d), up, ctypes.byref(s), ctypes.byref(slot))
        if rc == _lib.FR_E_NOMEM:
            return None
        check(rc, "fr_pool_admit_sampled")
        return slot.value

    def pressure(self, slot, observer, capacity):
        """(first observer time, p' on the times spaced by the sampling interval) at
        observer of a finished sampled request; call before result()."""
        xo = np.ascontiguousarray(observer, dtype=np.float64).reshape(3)
        p = np.zeros(int(capacity))
        t0 = ctypes.c_double()
        n = ctypes.c_int64()
        check(_lib.load().fr_pool_pressure(self.h, int(slot), xo.ctypes.data_as(_lib._dp), int(capacity),
                                           ctypes.byref(t0), ctypes.byref(n), p.ctypes.data_as(_lib._dp)),
              "fr_pool_pressure")
        return t0.value, p[:n.value].copy()

    def tick(self, k, max_done=256):
        done = np.zeros(max_done, dtype=np.int64)
        n = ctypes.c_int32()
        check(_lib.load().fr_pool_tick(self.h, int(k), done.ctypes.data_as(_lib._i64p), max_done, ctypes.byref(n)),
              "fr_pool_tick")
        return [int(v) for v in done[:n.value]]

    def launch(self, k):
        """Enqueue up to k steps for every running request; returns at once."""
        check(_lib.load().fr_pool_launch(self.h, int(k)), "fr_pool_launch")

    def collect(self, max_done=256):
        """Wait for the enqueued steps; slots of requests that finished."""
        done = np.zeros(max_done, dtype=np.int64)
        n = ctypes.c_int32()
        check(_lib.load().fr_pool_collect(self.h, done.ctypes.data_as(_lib._i64p), max_done, ctypes.byref(n)),
              "fr_pool_collect")
        return [int(v) for v in done[:n.value]]

    def result(self, slot, shape=None):
        out = np.zeros(8)
        u = np.zeros(shape) if shape is not None else None
        check(_lib.load().fr_pool_result(self.h, int(slot), out.ctypes.data_as(_lib._dp),
                                         u.ctypes.data_as(_lib._dp) if u is not None else None), "fr_pool_result")
        return (out, u) if shape is not None else out

    def usage(self):
        u = np.zeros(2, dtype=np.int64)
        check(_lib.load().fr_pool_usage(self.h, u.ctypes.data_as(_lib._i64p)), "fr_pool_usage")
        return int(u[0]), int(u[1])


class FWH:
    """Far-field acoustic pressure from a permeable data surface (FW-H, advanced time)."""

    def __init__(self, points, normals, areas, mach, c0, rho0, p0, dt, capacity, n_copies=1,
                 copy_shift=(0.0, 0.0, 0.0), tau0=0.0, device=0, use_torch_allocator=True, stream=None):
        L = _lib.load()
        self.stream_obj = stream if stream is not None else _new_stream(device)
        self.allocator = _TorchAllocator(device) if use_torch_allocator else None
        self._keep = [np.ascontiguousarray(points, dtype=np.float64).reshape(-1, 3),
                      np.ascontiguousarray(normals, dtype=np.float64).reshape(-1, 3),
                      np.ascontiguousarray(areas, dtype=np.float64).reshape(-1)]
        d = _lib.FwhDesc()
        d.n_points = self._keep[0].shape[0]
        d.points, d.normals, d.areas = (a.ctypes.data_as(_lib._dp) for a in self._keep)
        d.n_copies = int(n_copies)
        for i in range(3):
            d.copy_shift[i] = float(copy_shift[i])
            d.mach[i] = float(mach[i])
        d.c0, d.rho0, d.p0, d.dt, d.tau0 = float(c0), float(rho0), float(p0), float(dt), float(tau0)
        d.capacity = int(capacity)
        d.device = device
        d.stream = ctypes.c_void_p(self.stream_obj.cuda_stream)
        if self.allocator is not None:
            d.alloc, d.free = self.allocator.alloc, self.allocator.free
        h = ctypes.c_void_p()
        check(L.fr_fwh_create(ctypes.byref(d), ctypes.byref(h)), "fr_fwh_create")
        self.h = h
        self.n_points = int(d.n_points)
        self._dt = float(dt)
        _LIVE.add(self)

    def close(self):
        if getattr(self, "h", None):
            _lib.load().fr_fwh_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def append(self, rho, u, p):
        """Append snapshots: rho [n, np], u [n, np, 3] (disturbance velocity), p [n, np]."""
        rho = np.asarray(rho, dtype=np.float64)
        if rho.ndim == 1:
            rho, u, p = rho[None], np.asarray(u)[None], np.asarray(p)[None]
        x = np.ascontiguousarray(np.concatenate([rho[..., None], np.asarray(u, dtype=np.float64),
                                                 np.asarray(p, dtype=np.float64)[..., None]], axis=-1))
        check(_lib.load().fr_fwh_append(self.h, x.shape[0], x.ctypes.data_as(_lib._dp)), "fr_fwh_append")

    def append_probe(self, probe):
        """Append one snapshot of the probe's mesh state at the probe's points."""
        check(_lib.load().fr_fwh_append_probe(self.h, probe.h), "fr_fwh_append_probe")

    def samples(self):
        n = ctypes.c_int64()
        check(_lib.load().fr_fwh_samples(self.h, ctypes.byref(n)), "fr_fwh_samples")
        return n.value

    def window(self, observer):
        x = np.ascontiguousarray(observer, dtype=np.float64)
        t0, n = ctypes.c_double(), ctypes.c_int64()
        check(_lib.load().fr_fwh_window(self.h, x.ctypes.data_as(_lib._dp), ctypes.byref(t0), ctypes.byref(n)),
              "fr_fwh_window")
        return t0.value, n.value

    def pressure_at(self, observer, t_start, n, parts=False):
        """p' at observer times t_start + m dt (m < n) inside the common window."""
        x = np.ascontiguousarray(observer, dtype=np.float64)
        p, pt, pl = np.zeros(n), np.zeros(n), np.zeros(n)
        check(_lib.load().fr_fwh_pressure_at(self.h, x.ctypes.data_as(_lib._dp), float(t_start), int(n),
                                             p.ctypes.data_as(_lib._dp), pt.ctypes.data_as(_lib._dp),
                                             pl.ctypes.data_as(_lib._dp)), "fr_fwh_pressure_at")
        return (p, pt, pl) if parts else p

    def pressure_at_noalloc(self, observer, t_start, n, parts=False):
        """As pressure_at, through the entry point that allocates no device memory (its
        intermediate arrays live in the library's static device scratch)."""
        x = np.ascontiguousarray(observer, dtype=np.float64)
        p, pt, pl = np.zeros(n), np.zeros(n), np.zeros(n)
        check(_lib.load().fr_fwh_pressure_at_noalloc(self.h, x.ctypes.data_as(_lib._dp), float(t_start), int(n),
                                                     p.ctypes.data_as(_lib._dp), pt.ctypes.data_as(_lib._dp),
                                                     pl.ctypes.data_as(_lib._dp)), "fr_fwh_pressure_at_noalloc")
        return (p, pt, pl) if parts else p

    def pressure(self, observer, parts=False):
        """(t, p') at the observer, plus (p'_T, p'_L) when parts is set."""
        x = np.ascontiguousarray(observer, dtype=np.float64)
        _, n = self.window(x)
        p, pt, pl = np.zeros(n), np.zeros(n), np.zeros(n)
        t0, m = ctypes.c_double(), ctypes.c_int64()
        check(_lib.load().fr_fwh_pressure(self.h, x.ctypes.data_as(_lib._dp), n, ctypes.byref(t0), ctypes.byref(m),
                                          p.ctypes.data_as(_lib._dp), pt.ctypes.data_as(_lib._dp),
                                          pl.ctypes.data_as(_lib._dp)), "fr_fwh_pressure")
        t = t0.value + np.arange(m.value) * self._dt
        return (t, p[:m.value], pt[:m.value], pl[:m.value]) if parts else (t, p[:m.value])

    def time_ms(self):
        v = ctypes.c_double()
        check(_lib.load().fr_fwh_time_ms(self.h, ctypes.byref(v)), "fr_fwh_time_ms")
        return v.value


class Probe:
    """Samples of the FR solution of `mesh` (an FRMesh) at points [n, 3]."""

    def __init__(self, mesh, points, design=0):
        self.mesh = mesh  # the probe refers to the mesh: keep it alive
        pts = np.ascontiguousarray(points, dtype=np.float64).reshape(-1, 3)
        self.n = pts.shape[0]
        d, self._keep = _desc(mesh.meshes[design], "fp64")
        h = ctypes.c_void_p()
        check(_lib.load().fr_probe_create(mesh.h, ctypes.byref(d), design, self.n, pts.ctypes.data_as(_lib._dp),
                                          ctypes.byref(h)), "fr_probe_create")
        self.h = h
        _LIVE.add(self)

    def close(self):
        if getattr(self, "h", None):
            _lib.load().fr_probe_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def locate(self):
        elem = np.zeros(self.n, dtype=np.int64)
        xi = np.zeros((self.n, 3))
        check(_lib.load().fr_probe_locate(self.h, elem.ctypes.data_as(_lib._i64p), xi.ctypes.data_as(_lib._dp)),
              "fr_probe_locate")
        return elem, xi

    def sample(self):
        out = np.zeros((self.n, self.mesh.nv))
        check(_lib.load().fr_probe_sample(self.h, out.ctypes.data_as(_lib._dp)), "fr_probe_sample")
        return out
