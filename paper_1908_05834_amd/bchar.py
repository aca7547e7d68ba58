"""Thin ctypes binding of libbchar (include/bchar.h): argument marshalling only.

Every step of the method runs in the HIP library; this module only turns
Python/PyTorch objects into the C structs and pointers the ABI takes, and
raises ``BcharError`` on a non-zero status.  The library must have been
built (``python -m paper_1908_05834_amd.build_lib``); importing this module
without it raises immediately -- there is no fallback path.

PyTorch provides device memory and streams: pass CUDA (HIP) tensors and the
library runs on ``torch.cuda.current_stream()`` unless a stream is given.
"""

from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libbchar.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with "
                      "`python -m paper_1908_05834_amd.build_lib`")
_lib = C.CDLL(LIB_PATH)

# ---------------------------------------------------------------- constants (bchar.h)
OK, E_INVALID_ARG, E_OUT_OF_MEMORY, E_DEVICE, E_VOID_ROW, E_VOID_COLUMN, \
    E_QP_INFEASIBLE, E_QP_NOT_CONVERGED, E_UNSUPPORTED = range(9)
LAYOUT_SUBCELL, LAYOUT_INSCRIBED, LAYOUT_EQUAL_MEASURE, LAYOUT_CUSTOM, LAYOUT_PACKED = \
    0, 1, 2, 3, 4
FP64, FP32_VOLUME, FP32_LENS = 0, 1, 2
BOX_PAPER_THEN_RELAX, BOX_STRICT = 0, 1
STAGE_PAIRS, STAGE_V, STAGE_SCALING, STAGE_ALL = 1, 2, 3, 4
MEM_HOST, MEM_DEVICE = 0, 1
MESH_CARTESIAN, MESH_SIMPLEX = 0, 1
DIV_FREE, DIV_GENERAL = 0, 1

LAYOUTS = {"subcell": LAYOUT_SUBCELL, "inscribed": LAYOUT_INSCRIBED,
           "equal_measure": LAYOUT_EQUAL_MEASURE, "custom": LAYOUT_CUSTOM,
           "packed": LAYOUT_PACKED}


class MeshDesc(C.Structure):
    _fields_ = [("dim", C.c_int), ("n", C.c_int64 * 3), ("origin", C.c_double * 3),
                ("h", C.c_double * 3), ("phi", C.c_void_p), ("phi_mem", C.c_int),
                ("layout", C.c_int), ("kind", C.c_int), ("n_vertices", C.c_int64),
                ("n_simplices", C.c_int64), ("vertices", C.c_void_p), ("cells", C.c_void_p),
                ("geom_mem", C.c_int), ("n_balls", C.c_int64), ("balls", C.c_void_p),
                ("ball_cell", C.c_void_p), ("n_ghost", C.c_int64), ("hash_scale", C.c_double)]


class Velocity(C.Structure):
    _fields_ = [("m", C.c_int64 * 3), ("origin", C.c_double * 3), ("spacing", C.c_double * 3),
                ("u", C.c_void_p * 3)]


class Opts(C.Structure):
    _fields_ = [("precision", C.c_int), ("n_sweeps", C.c_int), ("rk_substeps", C.c_int),
                ("box_policy", C.c_int), ("stop_after", C.c_int), ("qp_tol", C.c_double),
                ("qp_max_newton", C.c_int), ("qp_max_cg", C.c_int), ("keep_pairs", C.c_int),
                ("warm_start", C.c_int), ("max_halvings", C.c_int),
                ("cg_graphs", C.c_int), ("cycle_skip", C.c_int), ("lds_stage", C.c_int),
                ("halve_on_level2", C.c_int), ("z_fuse_max_cells", C.c_int),
                ("divergence", C.c_int), ("tile_aspect", C.c_int)]


class Stats(C.Structure):
    _fields_ = [("n_balls", C.c_int64), ("n_pairs", C.c_int64), ("nnz", C.c_int64),
                ("first_void", C.c_int64), ("scaling_max_col_err", C.c_double),
                ("qp_residual", C.c_double), ("qp_level", C.c_int), ("qp_newton", C.c_int),
                ("qp_cg", C.c_int), ("n_at_lower", C.c_int64), ("n_at_upper", C.c_int64),
                ("qp_ipm", C.c_int), ("qp_coarse_bytes", C.c_int64),
                ("qp_smooth_bytes", C.c_int64), ("dt_halvings", C.c_int),
                ("n_void_rows", C.c_int64), ("n_void_cols", C.c_int64),
                ("trace_precision", C.c_int), ("device_bytes", C.c_int64),
                ("row_target_scale", C.c_double), ("n_target_groups", C.c_int64),
                ("qp_corrected", C.c_int)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_P = C.c_void_p
_i64p = C.POINTER(C.c_int64)
_ip = C.POINTER(C.c_int)


def _sig(name, args, res=C.c_int):
    f = getattr(_lib, name)
    f.argtypes = args
    f.restype = res
    return f


_opts_default = _sig("bchar_opts_default", [C.POINTER(Opts)], None)
_mesh_create = _sig("bchar_mesh_create", [C.POINTER(MeshDesc), _P, C.POINTER(_P)])
_mesh_destroy = _sig("bchar_mesh_destroy", [_P])
_mesh_info = _sig("bchar_mesh_info", [_P, _i64p, _i64p, _ip])
_build = _sig("bchar_build_transfer", [_P, C.POINTER(Velocity), C.c_double, C.POINTER(Opts), _P,
                                       C.POINTER(_P), C.POINTER(Stats)])
_rebuild = _sig("bchar_rebuild_transfer", [_P, C.POINTER(Velocity), C.c_double,
                                           C.POINTER(Opts), _P, C.POINTER(Stats)])
_build_tracked = _sig("bchar_build_transfer_tracked", [_P, _P, _P, C.POINTER(Opts), _P,
                                                       C.POINTER(_P), C.POINTER(Stats)])
_transfer_destroy = _sig("bchar_transfer_destroy", [_P])
_step = _sig("bchar_step", [_P, _P, _P, _P])
_mass = _sig("bchar_mass", [_P, _P, _P, C.POINTER(C.c_double)])
_mass_into = _sig("bchar_mass_into", [_P, _P, _P, _P])
_status_string = _sig("bchar_status_string", [C.c_int], C.c_char_p)
_last_error = _sig("bchar_last_error", [], C.c_char_p)
_transfer_info = _sig("bchar_transfer_info", [_P, _i64p, _i64p, _i64p, _ip])
_export_csr = _sig("bchar_transfer_export_csr", [_P, C.c_int, _P, _P, _P])
_export_pairs = _sig("bchar_transfer_export_pairs", [_P, _P, _P])
_export_tracked = _sig("bchar_transfer_export_tracked", [_P, _P, _P])
_export_targets = _sig("bchar_transfer_export_targets", [_P, _P, _P])
_export_qp = _sig("bchar_transfer_export_qp", [_P, _P, _P, _P])
_export_balls = _sig("bchar_mesh_export_balls", [_P, _P, _P, _P])
_export_qp_dual = _sig("bchar_transfer_export_qp_dual", [_P, _P, _P, _P, _P])
_profile_kernel = _sig("bchar_profile_kernel", [C.c_char_p])
_profile_kernel_sampled = _sig("bchar_profile_kernel_sampled", [C.c_char_p, C.c_int])


class BuildJob(C.Structure):
    _fields_ = [("transfer", C.c_void_p), ("mesh", C.c_void_p), ("u", C.POINTER(Velocity)),
                ("dt", C.c_double), ("warm_from", C.c_void_p), ("status", C.c_int),
                ("stats", Stats)]


class Request(C.Structure):
    _fields_ = [("mesh", C.c_void_p), ("u", C.POINTER(Velocity)), ("dt", C.c_double),
                ("steps", C.c_int), ("c_in", C.c_void_p), ("c_out", C.c_void_p),
                ("c_tmp", C.c_void_p), ("bytes", C.c_int64)]


class RequestResult(C.Structure):
    _fields_ = [("status", C.c_int), ("stats", Stats), ("t_submit", C.c_double),
                ("t_start", C.c_double), ("t_done", C.c_double)]


_server_create = _sig("bchar_server_create", [C.c_int, C.POINTER(C.c_void_p), C.c_int64,
                                              C.POINTER(Opts), C.POINTER(C.c_void_p)])
_server_submit = _sig("bchar_server_submit", [C.c_void_p, C.POINTER(Request),
                                              C.POINTER(C.c_int64)])
_server_wait = _sig("bchar_server_wait", [C.c_void_p, C.c_int64, C.POINTER(RequestResult)])
_server_destroy = _sig("bchar_server_destroy", [C.c_void_p])

_build_batch = _sig("bchar_build_transfer_batch", [C.POINTER(BuildJob), C.c_int, C.POINTER(Opts),
                                                   C.POINTER(C.c_void_p), C.c_int])
_tune_options = _sig("bchar_tune_options", [C.POINTER(BuildJob), C.c_int, C.POINTER(Opts), C.c_int,
                                            C.c_int, C.POINTER(C.c_void_p), C.c_int, _ip,
                                            C.POINTER(C.c_double)])
_profile_read = _sig("bchar_profile_read", [_i64p, C.POINTER(C.c_double)])

EXPORTED = [
    "bchar_opts_default", "bchar_mesh_create", "bchar_mesh_destroy", "bchar_mesh_info",
    "bchar_build_transfer", "bchar_rebuild_transfer", "bchar_build_transfer_tracked",
    "bchar_transfer_destroy", "bchar_step", "bchar_mass", "bchar_mass_into",
    "bchar_status_string",
    "bchar_last_error", "bchar_transfer_info", "bchar_transfer_export_csr",
    "bchar_transfer_export_pairs", "bchar_transfer_export_tracked", "bchar_transfer_export_qp",
    "bchar_mesh_export_balls", "bchar_transfer_export_qp_dual", "bchar_profile_kernel",
    "bchar_profile_read",
    "bchar_build_transfer_batch", "bchar_profile_kernel_sampled",
    "bchar_server_create", "bchar_server_submit", "bchar_server_wait", "bchar_server_destroy",
    "bchar_tune_options", "bchar_transfer_export_targets",
]


class BcharError(RuntimeError):
    def __init__(self, status, msg, stats=None):
        super().__init__(f"{_status_string(status).decode()}: {msg}")
        self.status = status
        self.stats = stats


def _check(rc, stats=None):
    if rc != OK:
        raise BcharError(rc, (_last_error() or b"").decode(), stats)


def status_string(s):
    return _status_string(s).decode()


def _stream_ptr(stream):
    if stream is None:
        import torch
        return C.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, int):
        return C.c_void_p(stream)
    return C.c_void_p(stream.cuda_stream)


def _dptr(t):
    return C.c_void_p(t.data_ptr())


def profile_kernel(name):
    """Time every later launch of kernel ``name`` with HIP events (None: off)."""
    _check(_profile_kernel(name.encode() if name else None))


def profile_kernel_sampled(name, every):
    """Time every ``every``-th launch of kernel ``name`` (None: off)."""
    _check(_profile_kernel_sampled(name.encode() if name else None, int(every)))


def profile_read():
    """(launches, total milliseconds) timed since ``profile_kernel``."""
    n, ms = C.c_int64(), C.c_double()
    _check(_profile_read(C.byref(n), C.byref(ms)))
    return n.value, ms.value


def opts_default(**kw):
    o = Opts()
    _opts_default(C.byref(o))
    for k, v in kw.items():
        if not hasattr(o, k):
            raise TypeError(f"unknown option {k}")
        setattr(o, k, v)
    return o


# ---------------------------------------------------------------- handles

class Mesh:
    """bchar_mesh_create on a Cartesian mesh dict (``inputs.cartesian_mesh``)
    or a simplicial one (``inputs.kuhn_tets``, ``inputs.triangulated_square``:
    layout ``"equal_measure"``).  Layout ``"custom"`` takes the mesh dict's
    ``ball_centres`` (n_balls, dim), ``ball_radii`` and ``ball_cell``.
    ``geom_device=True`` hands vertices, cells and custom balls over in
    device memory (copied to the GPU here first).  ``n_ghost``: layers of
    ghost cells on every side of a Cartesian grid (included in ``n``).
    ``hash_scale``: bucket side of the spatial hash over 2 r_max (0: 1)."""

    def __init__(self, mesh, layout="subcell", stream=None, geom_device=False, n_ghost=0,
                 hash_scale=0.0):
        d = MeshDesc()
        d.n_ghost = int(n_ghost)
        d.hash_scale = float(hash_scale)
        keep = []

        def ptr(a):
            if geom_device:
                import torch
                t = torch.as_tensor(np.ascontiguousarray(a), device="cuda")
                keep.append(t)
                return C.c_void_p(t.data_ptr())
            a = np.ascontiguousarray(a)
            keep.append(a)
            return a.ctypes.data_as(C.c_void_p)
        d.geom_mem = MEM_DEVICE if geom_device else MEM_HOST
        if mesh.get("kind") == "simplex":
            V = np.ascontiguousarray(mesh["vertices"], dtype=np.float64)
            Cc = np.ascontiguousarray(mesh["cells"], dtype=np.int32)
            self.dim = V.shape[1]
            d.dim = self.dim
            d.kind = MESH_SIMPLEX
            d.n_vertices = V.shape[0]
            d.n_simplices = Cc.shape[0]
            d.vertices = ptr(V)
            d.cells = ptr(Cc)
            for a in range(3):
                d.n[a], d.origin[a], d.h[a] = 1, 0.0, 1.0
        else:
            n = tuple(int(v) for v in mesh["n"])
            self.dim = len(n)
            d.dim = self.dim
            d.kind = MESH_CARTESIAN
            for a in range(3):
                d.n[a] = n[a] if a < self.dim else 1
                d.origin[a] = mesh["origin"][a] if a < self.dim else 0.0
                d.h[a] = mesh["h"][a] if a < self.dim else 1.0
        phi = np.ascontiguousarray(mesh["phi"], dtype=np.float64)
        self._phi_host = phi
        d.phi = phi.ctypes.data_as(C.c_void_p)
        d.phi_mem = MEM_HOST
        d.layout = LAYOUTS[layout] if isinstance(layout, str) else int(layout)
        if d.layout == LAYOUT_CUSTOM:
            bc = np.asarray(mesh["ball_centres"], dtype=np.float64)
            br = np.asarray(mesh["ball_radii"], dtype=np.float64)
            d.n_balls = br.shape[0]
            d.balls = ptr(np.concatenate([bc, br[:, None]], axis=1))
            d.ball_cell = ptr(np.asarray(mesh["ball_cell"], dtype=np.int32))
        h = C.c_void_p()
        _check(_mesh_create(C.byref(d), _stream_ptr(stream), C.byref(h)))
        if geom_device:
            import torch
            torch.cuda.current_stream().synchronize()
        del keep
        self.handle = h
        nc, nb, bpc = C.c_int64(), C.c_int64(), C.c_int()
        _check(_mesh_info(h, C.byref(nc), C.byref(nb), C.byref(bpc)))
        self.n_cells, self.n_balls, self.balls_per_cell = nc.value, nb.value, bpc.value

    def close(self):
        if self.handle:
            _mesh_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def mass(self, c, stream=None):
        out = C.c_double()
        _check(_mass(self.handle, _dptr(c), _stream_ptr(stream), C.byref(out)))
        return out.value

    def mass_into(self, c, out, stream=None):
        """bchar_mass_into: the mass written to the one-element device
        tensor ``out``, asynchronous, allocating nothing."""
        _check(_mass_into(self.handle, _dptr(c), _dptr(out), _stream_ptr(stream)))

    def export_balls(self):
        cen = np.empty(self.dim * self.n_balls)
        rad = np.empty(self.n_balls)
        cell = np.empty(self.n_balls, dtype=np.int32)
        _check(_export_balls(self.handle, cen.ctypes.data_as(_P), rad.ctypes.data_as(_P),
                             cell.ctypes.data_as(_P)))
        return cen.reshape(self.dim, self.n_balls).T.copy(), rad, cell


class VelocityLattice:
    """Device copy of a velocity lattice dict (``inputs.sample_velocity``)."""

    def __init__(self, vel, device="cuda"):
        import torch
        self.dim = len(vel["m"])
        self.comps = [torch.as_tensor(np.ascontiguousarray(vel["u"][a]), dtype=torch.float64,
                                      device=device) for a in range(self.dim)]
        v = Velocity()
        for a in range(3):
            v.m[a] = vel["m"][a] if a < self.dim else 1
            v.origin[a] = vel["origin"][a] if a < self.dim else 0.0
            v.spacing[a] = vel["spacing"][a] if a < self.dim else 1.0
            v.u[a] = self.comps[a].data_ptr() if a < self.dim else None
        self.struct = v


class Transfer:
    """A built transfer (bchar_build_transfer / _tracked / rebuild)."""

    def __init__(self, handle, mesh, stats):
        self.handle = handle
        self.mesh = mesh
        self.stats = stats

    @classmethod
    def build(cls, mesh, velocity, dt, opts=None, stream=None):
        o = opts if opts is not None else opts_default()
        st = Stats()
        h = C.c_void_p()
        rc = _build(mesh.handle, C.byref(velocity.struct), float(dt), C.byref(o),
                    _stream_ptr(stream), C.byref(h), C.byref(st))
        _check(rc, st.as_dict())
        return cls(h, mesh, st.as_dict())

    @classmethod
    def build_tracked(cls, mesh, tracked, r_hat, opts=None, stream=None):
        """``tracked``: device tensor (dim, n_balls); ``r_hat``: (n_balls,)."""
        o = opts if opts is not None else opts_default()
        st = Stats()
        h = C.c_void_p()
        rc = _build_tracked(mesh.handle, _dptr(tracked), _dptr(r_hat), C.byref(o),
                            _stream_ptr(stream), C.byref(h), C.byref(st))
        _check(rc, st.as_dict())
        return cls(h, mesh, st.as_dict())

    def rebuild(self, velocity, dt, opts=None, stream=None):
        o = opts if opts is not None else opts_default()
        st = Stats()
        rc = _rebuild(self.handle, C.byref(velocity.struct), float(dt), C.byref(o),
                      _stream_ptr(stream), C.byref(st))
        self.stats = st.as_dict()
        _check(rc, self.stats)
        return self.stats

    def step(self, c_in, c_out, stream=None):
        _check(_step(self.handle, _dptr(c_in), _dptr(c_out), _stream_ptr(stream)))

    def close(self):
        if self.handle:
            _transfer_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def info(self):
        nr, nnz, npairs, stage = C.c_int64(), C.c_int64(), C.c_int64(), C.c_int()
        _check(_transfer_info(self.handle, C.byref(nr), C.byref(nnz), C.byref(npairs),
                              C.byref(stage)))
        return nr.value, nnz.value, npairs.value, stage.value

    def export_csr(self, stage=STAGE_ALL):
        nr, nnz, _, _ = self.info()
        rp = np.empty(nr + 1, dtype=np.int64)
        col = np.empty(nnz, dtype=np.int32)
        val = np.empty(nnz)
        _check(_export_csr(self.handle, stage, rp.ctypes.data_as(_P), col.ctypes.data_as(_P),
                           val.ctypes.data_as(_P)))
        return rp, col.astype(np.int64), val

    def export_pairs(self):
        _, _, npairs, _ = self.info()
        a = np.empty(npairs, dtype=np.int32)
        b = np.empty(npairs, dtype=np.int32)
        _check(_export_pairs(self.handle, a.ctypes.data_as(_P), b.ctypes.data_as(_P)))
        return a.astype(np.int64), b.astype(np.int64)

    def export_tracked(self):
        dim, nb = self.mesh.dim, self.mesh.n_balls
        t = np.empty(dim * nb)
        r = np.empty(nb)
        _check(_export_tracked(self.handle, t.ctypes.data_as(_P), r.ctypes.data_as(_P)))
        return t.reshape(dim, nb).T.copy(), r

    def export_targets(self):
        """Per-ball log growth and per-cell row targets of the last build."""
        lam = np.empty(self.mesh.n_balls)
        b = np.empty(self.mesh.n_cells)
        _check(_export_targets(self.handle, lam.ctypes.data_as(_P), b.ctypes.data_as(_P)))
        return lam, b

    def export_qp(self):
        nr, nnz, _, _ = self.info()
        x = np.empty(nnz)
        mu = np.empty(nr)
        nu = np.empty(nr)
        _check(_export_qp(self.handle, x.ctypes.data_as(_P), mu.ctypes.data_as(_P),
                          nu.ctypes.data_as(_P)))
        return x, mu, nu

    def export_qp_dual(self):
        """Per-cell multipliers of the last solve (see bchar.h): leading
        parts s, g and their compensations s_lo, g_lo."""
        nr, _, _, _ = self.info()
        out = [np.empty(nr) for _ in range(4)]
        _check(_export_qp_dual(self.handle, *[o.ctypes.data_as(_P) for o in out]))
        return tuple(out)


def _handle_value(h):
    return h.value if isinstance(h, C.c_void_p) else h


def build_batch(jobs, opts=None, streams=None, check=True):
    """Build transfers of independent jobs at once (bchar_build_transfer_batch).

    ``jobs``: a list of ``(transfer, mesh, velocity, dt)`` or ``(transfer,
    mesh, velocity, dt, warm_from)``; ``transfer`` is a Transfer to rebuild,
    or None to create one on ``mesh``; ``warm_from`` an optional Transfer of
    the same mesh whose last solve warm-starts the job.  ``streams``:
    torch streams (or raw handles), one host worker each.  Returns the list
    of Transfer objects (the given ones, rebuilt, or new ones; None where a
    creation failed) after every job ended; raises BcharError (first failed
    job) if any failed, or with ``check=False`` returns ``(transfers,
    statuses)`` instead.
    """
    import torch
    if streams is None:
        streams = [torch.cuda.current_stream()]
    o = opts if opts is not None else opts_default()
    arr = (BuildJob * len(jobs))()
    for i, job in enumerate(jobs):
        tr, mesh, vel, dt = job[:4]
        wf = job[4] if len(job) > 4 else None
        arr[i].transfer = _handle_value(tr.handle) if tr is not None else None
        arr[i].mesh = _handle_value(mesh.handle) if mesh is not None else None
        arr[i].u = C.pointer(vel.struct)
        arr[i].dt = float(dt)
        arr[i].warm_from = _handle_value(wf.handle) if wf is not None else None
    sp = (C.c_void_p * len(streams))(*[_stream_ptr(s).value for s in streams])
    rc = _build_batch(arr, len(jobs), C.byref(o), sp, len(streams))
    out = []
    for i, job in enumerate(jobs):
        tr, mesh = job[0], job[1]
        st = arr[i].stats.as_dict()
        if tr is None:
            tr = Transfer(C.c_void_p(arr[i].transfer), mesh, st) if arr[i].transfer else None
        else:
            tr.stats = st
        out.append(tr)
    if not check:
        return out, [arr[i].status for i in range(len(jobs))]
    _check(rc)
    return out


def tune_options(jobs, candidates, streams=None, rounds=2):
    """Which option set builds ``jobs`` fastest (bchar_tune_options).

    ``jobs``: ``(mesh, velocity, dt)`` triples; ``candidates``: Opts;
    ``streams``: torch streams (or raw handles), one worker each.  Returns
    ``(best_index, seconds)`` with the summed wall time of every candidate
    (inf where its builds failed)."""
    import torch
    if streams is None:
        streams = [torch.cuda.current_stream()]
    arr = (BuildJob * len(jobs))()
    for i, (mesh, vel, dt) in enumerate(jobs):
        arr[i].mesh = _handle_value(mesh.handle)
        arr[i].u = C.pointer(vel.struct)
        arr[i].dt = float(dt)
    cands = (Opts * len(candidates))(*candidates)
    sp = (C.c_void_p * len(streams))(*[_stream_ptr(s).value for s in streams])
    best = C.c_int(-1)
    secs = (C.c_double * len(candidates))()
    _check(_tune_options(arr, len(jobs), cands, len(candidates), int(rounds), sp, len(streams),
                         C.byref(best), secs))
    return best.value, list(secs)


class Server:
    """A queue of independent requests (bchar_server_*): each request builds
    the transfer of one step on a resident mesh and applies it ``steps``
    times; ``workers`` host threads, each on its own stream."""

    def __init__(self, workers, mem_budget=0, opts=None, streams=None):
        import torch
        self.streams = streams or [torch.cuda.Stream() for _ in range(workers)]
        sp = (C.c_void_p * len(self.streams))(*[_stream_ptr(s).value for s in self.streams])
        o = opts if opts is not None else opts_default()
        h = C.c_void_p()
        _check(_server_create(len(self.streams), sp, int(mem_budget), C.byref(o), C.byref(h)))
        self.handle = h
        self._keep = {}

    def submit(self, mesh, velocity, dt, steps, c_in, c_out, c_tmp=None, nbytes=0):
        """Queue a request; the tensors must stay alive until ``wait``."""
        r = Request()
        r.mesh = _handle_value(mesh.handle)
        r.u = C.pointer(velocity.struct)
        r.dt = float(dt)
        r.steps = int(steps)
        r.c_in = c_in.data_ptr()
        r.c_out = c_out.data_ptr()
        r.c_tmp = c_tmp.data_ptr() if c_tmp is not None else None
        r.bytes = int(nbytes)
        t = C.c_int64()
        _check(_server_submit(self.handle, C.byref(r), C.byref(t)))
        self._keep[t.value] = (velocity, c_in, c_out, c_tmp)
        return t.value

    def wait(self, ticket):
        """Block until the request ended: its status, stats and the host
        clock at submission, start and end (seconds)."""
        res = RequestResult()
        _check(_server_wait(self.handle, int(ticket), C.byref(res)))
        self._keep.pop(ticket, None)
        return {"status": res.status, "stats": res.stats.as_dict(), "t_submit": res.t_submit,
                "t_start": res.t_start, "t_done": res.t_done}

    def close(self):
        if self.handle:
            _server_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
