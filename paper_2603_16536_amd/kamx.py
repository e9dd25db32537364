"""Python binding of libkamx (ctypes): argument marshalling only.

Every step of the solver runs in the HIP kernels of ``libkamx.so``; this
module builds descriptor arrays from a :class:`scenes.Scene`, hands torch
device pointers and streams to the C entry points, and wraps the results as
torch tensors.  It fails loudly when the library has not been built.
"""
from __future__ import annotations

import ctypes as C
import dataclasses
import math
import os

import numpy as np
import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libkamx.so")

OK, EINVAL, ENOMEM, EDEVICE, ESTATE, EUNSUPPORTED = 0, -1, -2, -3, -4, -5
WORLD_OK, WORLD_MAXITER, WORLD_NONFINITE, WORLD_FACTOR_FAIL = 0, 1, 2, 4
WARM_COLD, WARM_PREVIOUS, WARM_EXTERNAL, WARM_LEARNED = 0, 1, 2, 3
SCHED_INDEX, SCHED_LPT, SCHED_CHAIN = 0, 1, 2
EULER, MOREAU_JEAN = 0, 1
SOLVER_AUTO, SOLVER_DENSE, SOLVER_SPARSE = 0, 1, 2
MAX_BODIES_SPARSE, MAX_JOINTS_SPARSE, MAX_THREAD_ROWS_SPARSE = 160, 200, 1024
MAX_CONTACTS_PER_WORLD = 64


class kamx_params(C.Structure):
    _fields_ = [
        ("dt", C.c_float), ("gravity", C.c_float * 3), ("eta", C.c_float), ("rho_bilateral", C.c_float),
        ("rho_contact", C.c_float), ("eps", C.c_float), ("max_iters", C.c_int32), ("fixed_iters", C.c_int32),
        ("accel", C.c_int32), ("restart_factor", C.c_float), ("precond", C.c_int32), ("baumgarte", C.c_float),
        ("warmstart", C.c_int32), ("contact_margin", C.c_float), ("torque_sigma", C.c_float),
        ("seed", C.c_uint64), ("reset_height", C.c_float), ("log_restarts", C.c_int32),
        ("integrator", C.c_int32), ("linear_solver", C.c_int32), ("cr_iters", C.c_int32),
        ("adapt_ratio", C.c_float), ("adapt_factor", C.c_float), ("adapt_first", C.c_int32),
    ]


class kamx_body_desc(C.Structure):
    _fields_ = [("world", C.c_int32), ("mass", C.c_float), ("inertia", C.c_float * 3)]


class kamx_joint_desc(C.Structure):
    _fields_ = [
        ("type", C.c_int32), ("world", C.c_int32), ("body_a", C.c_int32), ("body_b", C.c_int32),
        ("frame_a", C.c_float * 7), ("frame_b", C.c_float * 7), ("limit_lo", C.c_float), ("limit_hi", C.c_float),
        ("kp", C.c_float), ("kd", C.c_float), ("ref", C.c_float), ("actuated", C.c_int32),
        ("damping", C.c_float), ("armature", C.c_float), ("implicit_drive", C.c_int32),
    ]


class kamx_probe_desc(C.Structure):
    _fields_ = [("world", C.c_int32), ("body", C.c_int32), ("point", C.c_float * 3), ("mu", C.c_float)]


BODY_DTYPE = np.dtype([("world", "<i4"), ("mass", "<f4"), ("inertia", "<f4", 3)])
JOINT_DTYPE = np.dtype([("type", "<i4"), ("world", "<i4"), ("body_a", "<i4"), ("body_b", "<i4"),
                        ("frame_a", "<f4", 7), ("frame_b", "<f4", 7), ("limit_lo", "<f4"), ("limit_hi", "<f4"),
                        ("kp", "<f4"), ("kd", "<f4"), ("ref", "<f4"), ("actuated", "<i4"),
                        ("damping", "<f4"), ("armature", "<f4"), ("implicit_drive", "<i4")])
PROBE_DTYPE = np.dtype([("world", "<i4"), ("body", "<i4"), ("point", "<f4", 3), ("mu", "<f4")])
CONTACT_DTYPE = np.dtype([("body_a", "<i4"), ("body_b", "<i4"), ("point", "<f4", 3), ("normal", "<f4", 3),
                          ("gap", "<f4"), ("mu", "<f4"), ("key", "<i4")])
assert CONTACT_DTYPE.itemsize == 44 and BODY_DTYPE.itemsize == 20
assert JOINT_DTYPE.itemsize == 108 and PROBE_DTYPE.itemsize == 24

_lib = None


def lib():
    """Load libkamx.so; raises if it is missing (there is no fallback)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built; run __graft_entry__.build() (hipcc, gfx950)")
        L = C.CDLL(LIB_PATH)
        vp, i32, i64p = C.c_void_p, C.c_int32, C.POINTER(C.c_int64)
        L.kamx_default_params.argtypes = [C.POINTER(kamx_params)]
        L.kamx_default_params.restype = None
        L.kamx_last_error.restype = C.c_char_p
        L.kamx_model_create.argtypes = [C.POINTER(kamx_body_desc), i32, C.POINTER(kamx_joint_desc), i32,
                                        C.POINTER(kamx_probe_desc), i32, C.POINTER(C.c_int32), i32, i32,
                                        C.POINTER(kamx_params), C.POINTER(vp)]
        L.kamx_model_destroy.argtypes = [vp]
        L.kamx_set_params.argtypes = [vp, C.POINTER(kamx_params)]
        L.kamx_model_info.argtypes = [vp, C.POINTER(C.c_int32), C.POINTER(C.c_int32), C.POINTER(C.c_int32),
                                      C.POINTER(C.c_int32), C.POINTER(C.c_int32)]
        L.kamx_state_upload.argtypes = [vp, vp, vp, i32, vp]
        L.kamx_state_download.argtypes = [vp, vp, vp, vp]
        L.kamx_contacts_upload.argtypes = [vp, vp, C.POINTER(C.c_int32), vp]
        L.kamx_set_external.argtypes = [vp, vp, vp]
        L.kamx_set_warmstart.argtypes = [vp, vp, vp]
        L.kamx_step.argtypes = [vp, i32, vp]
        L.kamx_set_schedule.argtypes = [vp, i32]
        L.kamx_bucket_count.argtypes = [vp, C.POINTER(C.c_int32)]
        L.kamx_bucket_info.argtypes = [vp, i32] + [C.POINTER(C.c_int32)] * 5
        L.kamx_set_bucket_threads.argtypes = [vp, i32, i32]
        L.kamx_autotune.argtypes = [vp, i32, C.POINTER(C.c_float)]
        L.kamx_set_iteration_log.argtypes = [vp, vp, vp, vp, i32]
        L.kamx_set_iterate_log.argtypes = [vp, vp]
        L.kamx_forward_kinematics.argtypes = [vp, vp, i32, C.c_float, vp, vp, vp]
        L.kamx_mlp_create.argtypes = [i32, i32, i32, i32, C.c_uint64, C.POINTER(vp)]
        L.kamx_mlp_destroy.argtypes = [vp]
        L.kamx_mlp_info.argtypes = [vp, C.POINTER(C.c_int32), C.POINTER(C.c_int32), i64p]
        L.kamx_mlp_set_normalization.argtypes = [vp, vp, vp, vp, vp, vp]
        L.kamx_mlp_forward.argtypes = [vp, vp, i32, vp, vp]
        L.kamx_mlp_forward_noalloc.argtypes = [vp, vp, i32, vp, vp]
        L.kamx_mlp_train_step.argtypes = [vp, vp, vp, i32, C.c_float, vp, vp]
        L.kamx_mlp_weights.argtypes = [vp, vp, i32, vp]
        L.kamx_mlp_gradients.argtypes = [vp, vp, vp]
        L.kamx_model_feature_dims.argtypes = [vp, C.POINTER(C.c_int32), C.POINTER(C.c_int32)]
        L.kamx_model_features.argtypes = [vp, vp, vp]
        L.kamx_read_impulse_slots.argtypes = [vp, vp, vp]
        L.kamx_model_attach_mlp.argtypes = [vp, vp]
        L.kamx_contacts_box_bin.argtypes = [vp, vp, C.c_float, C.c_float, C.c_float]
        L.kamx_read_impulses.argtypes = [vp, vp, vp]
        L.kamx_read_stats.argtypes = [vp, vp, vp, vp, vp, vp]
        L.kamx_read_restart_log.argtypes = [vp, vp, vp]
        L.kamx_read_torques.argtypes = [vp, vp, vp]
        L.kamx_read_contacts.argtypes = [vp, vp, vp, vp]
        L.kamx_reset_count.argtypes = [vp, i64p, vp]
        L.kamx_read_phase_clock.argtypes = [vp, vp, vp]
        for name in ("kamx_model_create", "kamx_model_destroy", "kamx_set_params", "kamx_model_info",
                     "kamx_state_upload", "kamx_state_download", "kamx_contacts_upload", "kamx_set_external",
                     "kamx_set_warmstart", "kamx_step", "kamx_read_impulses", "kamx_read_stats",
                     "kamx_read_restart_log", "kamx_read_torques", "kamx_read_contacts", "kamx_reset_count",
                     "kamx_read_phase_clock", "kamx_set_schedule", "kamx_mlp_create", "kamx_mlp_destroy",
                     "kamx_mlp_info", "kamx_mlp_set_normalization", "kamx_mlp_forward", "kamx_mlp_forward_noalloc",
                     "kamx_mlp_train_step",
                     "kamx_mlp_weights", "kamx_mlp_gradients", "kamx_model_feature_dims", "kamx_model_features",
                     "kamx_read_impulse_slots", "kamx_model_attach_mlp", "kamx_contacts_box_bin",
                     "kamx_set_iteration_log", "kamx_set_iterate_log", "kamx_forward_kinematics"):
            getattr(L, name).restype = C.c_int32
        _lib = L
    return _lib


class KamxError(RuntimeError):
    pass


def _check(status):
    if status != OK:
        raise KamxError(f"kamx error {status}: {lib().kamx_last_error().decode()}")


def default_params():
    p = kamx_params()
    lib().kamx_default_params(C.byref(p))
    return p


def make_params(**kw):
    """A kamx_params struct: library defaults overridden by keyword values
    (gravity given as a 3-sequence)."""
    p = default_params()
    for k, v in kw.items():
        if k == "gravity":
            for e in range(3):
                p.gravity[e] = float(v[e])
        elif not hasattr(p, k):
            raise KeyError(k)
        else:
            setattr(p, k, v)
    return p


def _stream(stream):
    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream)


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else None


def contacts_tensor(scene, device):
    """The scene's explicit contacts as a device byte tensor of kamx_contact
    records plus host world offsets."""
    n = scene.n_contacts
    arr = np.zeros(max(n, 1), CONTACT_DTYPE)
    if n:
        arr["body_a"] = scene.contact_body[:, 0]
        arr["body_b"] = scene.contact_body[:, 1]
        arr["point"] = scene.contact_point
        arr["normal"] = scene.contact_normal
        arr["gap"] = scene.contact_gap
        arr["mu"] = scene.contact_mu
        arr["key"] = scene.contact_key
    dev = torch.from_numpy(arr.view(np.uint8).copy()).to(device)
    off = scene.contact_offsets().astype(np.int32)
    return dev, off


def decode_contacts(byte_tensor):
    a = byte_tensor.detach().cpu().numpy().view(CONTACT_DTYPE)
    return a


class Model:
    """A batch of worlds on one GPU.

    ``scene``: a scenes.Scene; ``params``: keyword overrides of the library
    defaults; ``max_contacts``: capacity for explicit contacts per world
    (0 = probe contacts only); ``pd``: optional (kp, kd) for every actuated
    joint (without it the scene's per-joint gains apply), driving the joint
    coordinate toward ``refs`` (default 0, the assembled pose of joints
    whose frames coincide at assembly)."""

    def __init__(self, scene, params=None, max_contacts=0, pd=None, refs=None, device="cuda:0"):
        self.device = torch.device(device)
        self.scene = scene
        self.n_worlds = scene.n_worlds
        nb, nj, np_ = scene.n_bodies, scene.n_joints, int(scene.probe_body.shape[0])
        bodies = np.zeros(max(nb, 1), BODY_DTYPE)
        bodies["world"][:nb] = scene.body_world
        bodies["mass"][:nb] = scene.body_mass
        bodies["inertia"][:nb] = scene.body_inertia
        joints = np.zeros(max(nj, 1), JOINT_DTYPE)
        if nj:
            joints["type"][:nj] = scene.joint_type
            joints["world"][:nj] = scene.joint_world
            joints["body_a"][:nj] = scene.joint_body[:, 0]
            joints["body_b"][:nj] = scene.joint_body[:, 1]
            joints["frame_a"][:nj] = scene.joint_frame[:, :7]
            joints["frame_b"][:nj] = scene.joint_frame[:, 7:]
            joints["limit_lo"][:nj] = scene.joint_limit[:, 0]
            joints["limit_hi"][:nj] = scene.joint_limit[:, 1]
            act = scene.joint_actuated.astype(np.int32)
            joints["actuated"][:nj] = act
            on = act != 0
            if pd is not None:
                joints["kp"][:nj][on] = float(pd[0])
                joints["kd"][:nj][on] = float(pd[1])
            elif scene.joint_pd.shape[0] == nj:
                joints["kp"][:nj][on] = scene.joint_pd[on, 0]
                joints["kd"][:nj][on] = scene.joint_pd[on, 1]
            if refs is not None:
                joints["ref"][:nj][on] = np.asarray(refs, np.float32)[on]
            # implicit drives (kp, kd, damping, armature, ref): a drive row
            # replaces the explicit PD of those joints
            drv = getattr(scene, "joint_drive", None)
            if drv is not None and drv.shape[0] == nj:
                dj = np.any(drv[:, :4] != 0.0, axis=1)
                joints["implicit_drive"][:nj] = dj.astype(np.int32)
                joints["kp"][:nj][dj] = drv[dj, 0]
                joints["kd"][:nj][dj] = drv[dj, 1]
                joints["damping"][:nj][dj] = drv[dj, 2]
                joints["armature"][:nj][dj] = drv[dj, 3]
                joints["ref"][:nj][dj] = drv[dj, 4]
        probes = np.zeros(max(np_, 1), PROBE_DTYPE)
        if np_:
            probes["world"][:np_] = scene.probe_world
            probes["body"][:np_] = scene.probe_body
            probes["point"][:np_] = scene.probe_point
            probes["mu"][:np_] = scene.probe_mu
        B = C.cast(bodies.ctypes.data, C.POINTER(kamx_body_desc))
        J = C.cast(joints.ctypes.data, C.POINTER(kamx_joint_desc))
        Pr = C.cast(probes.ctypes.data, C.POINTER(kamx_probe_desc))
        rb = (C.c_int32 * self.n_worlds)()
        if scene.reset_body.size == self.n_worlds:
            for w in range(self.n_worlds):
                rb[w] = int(scene.reset_body[w])
        else:
            for w in range(self.n_worlds):
                rb[w] = -1
        kw = dict(dt=scene.dt, gravity=scene.gravity)
        if scene.reset_height > -1e29:
            kw["reset_height"] = scene.reset_height
        kw.update(params or {})
        self.params = make_params(**kw)
        h = C.c_void_p()
        with torch.cuda.device(self.device):
            _check(lib().kamx_model_create(B, nb, J, nj, Pr, np_, rb, self.n_worlds, int(max_contacts),
                                           C.byref(self.params), C.byref(h)))
        self.handle = h
        nbo, njo, rows, nbk = C.c_int32(), C.c_int32(), C.c_int32(), C.c_int32()
        offs = (C.c_int32 * (self.n_worlds + 1))()
        _check(lib().kamx_model_info(h, C.byref(nbo), C.byref(njo), C.byref(rows), C.byref(nbk), offs))
        self.n_bodies, self.n_joints = nbo.value, njo.value
        self.rows_capacity, self.n_buckets = rows.value, nbk.value
        self.row_offsets = np.array(offs[:], dtype=np.int64)
        self._keep = []
        self.upload_state(scene.q, scene.u, as_reset_state=True)

    # -- lifetime ------------------------------------------------------------
    def close(self):
        if getattr(self, "handle", None):
            lib().kamx_model_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- inputs --------------------------------------------------------------
    def set_params(self, **kw):
        for k, v in kw.items():
            if k == "gravity":
                for e in range(3):
                    self.params.gravity[e] = float(v[e])
            else:
                setattr(self.params, k, v)
        _check(lib().kamx_set_params(self.handle, C.byref(self.params)))

    def upload_state(self, q, u, as_reset_state=False, stream=None):
        qt = torch.as_tensor(np.asarray(q, np.float32) if not torch.is_tensor(q) else q,
                             dtype=torch.float32, device=self.device).contiguous()
        ut = torch.as_tensor(np.asarray(u, np.float32) if not torch.is_tensor(u) else u,
                             dtype=torch.float32, device=self.device).contiguous()
        _check(lib().kamx_state_upload(self.handle, _ptr(qt), _ptr(ut), int(as_reset_state), _stream(stream)))
        self._keep.append((qt, ut))
        torch.cuda.current_stream(self.device).synchronize()
        self._keep.clear()

    def upload_contacts(self, scene=None, stream=None):
        """Use the scene's explicit contacts (or probes again when scene is None)."""
        if scene is None:
            _check(lib().kamx_contacts_upload(self.handle, None, None, _stream(stream)))
            self._contacts = None
            return
        dev, off = contacts_tensor(scene, self.device)
        offs = (C.c_int32 * (self.n_worlds + 1))(*[int(x) for x in off])
        _check(lib().kamx_contacts_upload(self.handle, _ptr(dev), offs, _stream(stream)))
        self._contacts = dev

    def set_external(self, tau=None, stream=None):
        if tau is None:
            self._ext = None
            _check(lib().kamx_set_external(self.handle, None, _stream(stream)))
            return
        t = torch.as_tensor(tau, dtype=torch.float32, device=self.device).contiguous()
        self._ext = t
        _check(lib().kamx_set_external(self.handle, _ptr(t), _stream(stream)))

    def set_warmstart(self, lam, stream=None):
        t = torch.as_tensor(lam, dtype=torch.float32, device=self.device).contiguous()
        _check(lib().kamx_set_warmstart(self.handle, _ptr(t), _stream(stream)))
        torch.cuda.current_stream(self.device).synchronize()

    # -- stepping ------------------------------------------------------------
    def contacts_box_bin(self, half=(0.15, 0.15), margin=0.01, boxes=None):
        """Generate contacts every step from the scene's box geometry
        (``scene.body_box``: half extents and mu per body) against a bin of
        the given half widths; ``boxes=False`` turns generation off."""
        if boxes is False:
            _check(lib().kamx_contacts_box_bin(self.handle, None, 0.0, 0.0, 0.0))
            return
        bx = np.asarray(self.scene.body_box if boxes is None else boxes, np.float32).reshape(-1, 4)
        assert bx.shape[0] == self.scene.n_bodies
        arr = np.ascontiguousarray(bx)
        _check(lib().kamx_contacts_box_bin(self.handle, C.c_void_p(arr.ctypes.data), float(half[0]), float(half[1]),
                                           float(margin)))

    # -- learned warm start --------------------------------------------------
    def feature_dims(self):
        """(n_features, n_slots) of a model whose worlds share one structure."""
        nf, ns = C.c_int32(), C.c_int32()
        _check(lib().kamx_model_feature_dims(self.handle, C.byref(nf), C.byref(ns)))
        return nf.value, ns.value

    def features(self, out=None, stream=None):
        """Features of the coming step, [n_worlds, n_features] (device)."""
        nf, _ = self.feature_dims()
        x = out if out is not None else torch.empty((self.n_worlds, nf), dtype=torch.float32, device=self.device)
        _check(lib().kamx_model_features(self.handle, _ptr(x), _stream(stream)))
        return x

    def impulse_slots(self, out=None, stream=None):
        """Impulses of the last step by slot, [n_worlds, n_slots] (device)."""
        _, ns = self.feature_dims()
        y = out if out is not None else torch.empty((self.n_worlds, ns), dtype=torch.float32, device=self.device)
        _check(lib().kamx_read_impulse_slots(self.handle, _ptr(y), _stream(stream)))
        return y

    def attach_mlp(self, net):
        """Network for the LEARNED warm start (None detaches); the model
        keeps a reference so the network outlives its use."""
        _check(lib().kamx_model_attach_mlp(self.handle, net.handle if net is not None else None))
        self._mlp = net

    def set_iteration_log(self, iters, rows=None, status=None):
        """Device int32 tensors [steps, n_worlds] that receive the iteration
        count (and active rows and status bits) of every step of the
        following step() calls (None: off)."""
        if iters is None:
            _check(lib().kamx_set_iteration_log(self.handle, None, None, None, 0))
        else:
            for t in (iters, rows, status):
                assert t is None or (t.dtype == torch.int32 and t.is_contiguous() and t.shape[1] == self.n_worlds)
            _check(lib().kamx_set_iteration_log(self.handle, _ptr(iters), _ptr(rows), _ptr(status),
                                                int(iters.shape[0])))
        self._iter_log = (iters, rows, status)

    def forward_kinematics(self, targets, max_iters=50, tol=3e-7, stream=None):
        """Poses consistent with every joint and with the target joint
        coordinates ([n_joints], NaN = free), reset bodies held; twists set to
        zero.  Returns device tensors (iterations, |F|_inf) per world."""
        t = torch.as_tensor(np.asarray(targets, np.float32) if not torch.is_tensor(targets) else targets,
                            dtype=torch.float32, device=self.device).contiguous()
        it = torch.zeros(self.n_worlds, dtype=torch.int32, device=self.device)
        res = torch.zeros(self.n_worlds, dtype=torch.float32, device=self.device)
        _check(lib().kamx_forward_kinematics(self.handle, _ptr(t), int(max_iters), float(tol), _ptr(it), _ptr(res),
                                             _stream(stream)))
        self._fk_targets = t
        return it, res

    def set_iterate_log(self, on=True):
        """Record the last step's final iterate (x~, y~, z~, p) per row
        into a device tensor [rows_capacity, 4] (returned); on=False stops."""
        if not on:
            _check(lib().kamx_set_iterate_log(self.handle, None))
            self._iterate = None
            return None
        t = torch.zeros((max(self.rows_capacity, 1), 4), dtype=torch.float32, device=self.device)
        _check(lib().kamx_set_iterate_log(self.handle, _ptr(t)))
        self._iterate = t
        return t

    def set_schedule(self, mode):
        """Mapping of steps onto workgroups: SCHED_CHAIN (default), SCHED_LPT
        or SCHED_INDEX (results are identical under all three)."""
        _check(lib().kamx_set_schedule(self.handle, int(mode)))

    def buckets(self):
        """Size buckets as dicts: rows (capacity), worlds, threads (current
        workgroup size) and variants (the sizes the bucket is built for)."""
        n = C.c_int32()
        _check(lib().kamx_bucket_count(self.handle, C.byref(n)))
        out = []
        for b in range(n.value):
            rows, worlds, threads, nv = C.c_int32(), C.c_int32(), C.c_int32(), C.c_int32()
            var = (C.c_int32 * 4)()
            _check(lib().kamx_bucket_info(self.handle, b, C.byref(rows), C.byref(worlds), C.byref(threads),
                                          C.byref(nv), var))
            out.append(dict(rows=rows.value, worlds=worlds.value, threads=threads.value,
                            variants=[var[k] for k in range(nv.value)]))
        return out

    def set_bucket_threads(self, bucket, threads):
        _check(lib().kamx_set_bucket_threads(self.handle, int(bucket), int(threads)))

    def autotune(self, trial_steps=8):
        """Time every bucket's workgroup-size variants on trial_steps steps
        from the current state (restored afterwards) and keep the fastest.
        Returns the milliseconds per bucket and variant."""
        n = len(self.buckets())
        ms = (C.c_float * max(4 * n, 1))()
        _check(lib().kamx_autotune(self.handle, int(trial_steps), ms))
        return [[ms[4 * b + v] for v in range(len(bk["variants"]))] for b, bk in enumerate(self.buckets())]

    def step(self, n=1, stream=None):
        _check(lib().kamx_step(self.handle, int(n), _stream(stream)))

    # -- outputs -------------------------------------------------------------
    def state(self, stream=None):
        q = torch.empty((self.n_bodies, 7), dtype=torch.float32, device=self.device)
        u = torch.empty((self.n_bodies, 6), dtype=torch.float32, device=self.device)
        _check(lib().kamx_state_download(self.handle, _ptr(q), _ptr(u), _stream(stream)))
        return q, u

    def impulses(self, stream=None):
        lam = torch.empty(max(self.rows_capacity, 1), dtype=torch.float32, device=self.device)
        _check(lib().kamx_read_impulses(self.handle, _ptr(lam), _stream(stream)))
        return lam[: self.rows_capacity]

    def stats(self, stream=None):
        n = self.n_worlds
        it = torch.empty(n, dtype=torch.int32, device=self.device)
        res = torch.empty((n, 4), dtype=torch.float32, device=self.device)
        st = torch.empty(n, dtype=torch.int32, device=self.device)
        rows = torch.empty(n, dtype=torch.int32, device=self.device)
        _check(lib().kamx_read_stats(self.handle, _ptr(it), _ptr(res), _ptr(st), _ptr(rows), _stream(stream)))
        return dict(iters=it, resid=res, status=st, rows=rows)

    def stats_into(self, iters=None, resid=None, status=None, rows=None, stream=None):
        """Stream-ordered copy of the last step's per-world stats into the
        given device tensors (no host synchronization)."""
        _check(lib().kamx_read_stats(self.handle, _ptr(iters), _ptr(resid), _ptr(status), _ptr(rows),
                                     _stream(stream)))

    def restart_log(self, stream=None):
        t = torch.empty((self.n_worlds, self.params.max_iters), dtype=torch.uint8, device=self.device)
        _check(lib().kamx_read_restart_log(self.handle, _ptr(t), _stream(stream)))
        return t

    def torques(self, stream=None):
        t = torch.empty(max(self.n_joints, 1), dtype=torch.float32, device=self.device)
        _check(lib().kamx_read_torques(self.handle, _ptr(t), _stream(stream)))
        return t[: self.n_joints]

    def contacts(self, stream=None):
        raw = torch.empty(self.n_worlds * MAX_CONTACTS_PER_WORLD * CONTACT_DTYPE.itemsize, dtype=torch.uint8,
                          device=self.device)
        cnt = torch.empty(self.n_worlds, dtype=torch.int32, device=self.device)
        _check(lib().kamx_read_contacts(self.handle, _ptr(raw), _ptr(cnt), _stream(stream)))
        return raw, cnt

    def phase_clock(self, stream=None):
        t = torch.empty((self.n_worlds, 16), dtype=torch.int64, device=self.device)
        _check(lib().kamx_read_phase_clock(self.handle, _ptr(t), _stream(stream)))
        return t

    def reset_count(self, stream=None):
        c = C.c_int64()
        _check(lib().kamx_reset_count(self.handle, C.byref(c), _stream(stream)))
        return c.value


def contacts_to_scene(scene, raw, counts):
    """A copy of ``scene`` whose explicit contacts are the ones the library
    used in its last step (for feeding the same rows to a reference)."""
    recs = decode_contacts(raw).reshape(scene.n_worlds, MAX_CONTACTS_PER_WORLD)
    counts = counts.detach().cpu().numpy()
    cw, cb, cp, cn, cg, cm, ck = [], [], [], [], [], [], []
    for w in range(scene.n_worlds):
        for k in range(int(counts[w])):
            r = recs[w, k]
            cw.append(w)
            cb.append((r["body_a"], r["body_b"]))
            cp.append(r["point"])
            cn.append(r["normal"])
            cg.append(r["gap"])
            cm.append(r["mu"])
            ck.append(r["key"])
    n = len(cw)
    return scene.replace(
        contact_world=np.array(cw, np.int32), contact_body=np.array(cb, np.int32).reshape(n, 2),
        contact_point=np.array(cp, np.float64).reshape(n, 3), contact_normal=np.array(cn, np.float64).reshape(n, 3),
        contact_gap=np.array(cg, np.float64), contact_mu=np.array(cm, np.float64), contact_key=np.array(ck, np.int32))


class MLP:
    """The learned warm-start network (device weights; every product on the
    matrix cores in BF16 with FP32 accumulation)."""

    def __init__(self, n_in, n_out, n_hidden=256, max_batch=4096, seed=0, device="cuda:0"):
        self.device = torch.device(device)
        self.n_in, self.n_out, self.n_hidden = int(n_in), int(n_out), int(n_hidden)
        h = C.c_void_p()
        _check(lib().kamx_mlp_create(self.n_in, self.n_hidden, self.n_out, int(max_batch), C.c_uint64(seed),
                                     C.byref(h)))
        self.handle = h
        fp, op, n = C.c_int32(), C.c_int32(), C.c_int64()
        _check(lib().kamx_mlp_info(h, C.byref(fp), C.byref(op), C.byref(n)))
        self.n_in_pad, self.n_out_pad, self.n_params = fp.value, op.value, n.value
        self.max_batch = int(max_batch)

    def close(self):
        if getattr(self, "handle", None):
            lib().kamx_mlp_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _f32(self, a):
        return torch.as_tensor(a, dtype=torch.float32, device=self.device).contiguous()

    def set_normalization(self, mu_in, sigma_in, mu_out, sigma_out, stream=None):
        t = [self._f32(a) for a in (mu_in, sigma_in, mu_out, sigma_out)]
        _check(lib().kamx_mlp_set_normalization(self.handle, *[_ptr(x) for x in t], _stream(stream)))
        torch.cuda.current_stream(self.device).synchronize()

    def forward(self, x, out=None, stream=None):
        x = self._f32(x)
        b = x.shape[0]
        y = out if out is not None else torch.empty((b, self.n_out), dtype=torch.float32, device=self.device)
        _check(lib().kamx_mlp_forward(self.handle, _ptr(x), b, _ptr(y), _stream(stream)))
        return y

    def forward_noalloc(self, x, out, stream=None):
        """The same prediction as forward(), with the activations in the
        library's fixed per-GPU workspace (no device allocation inside);
        ``x`` and ``out`` must be contiguous FP32 device tensors."""
        assert x.dtype == torch.float32 and out.dtype == torch.float32 and x.is_contiguous() and out.is_contiguous()
        _check(lib().kamx_mlp_forward_noalloc(self.handle, _ptr(x), x.shape[0], _ptr(out), _stream(stream)))
        return out

    def train_step(self, x, y, lr, loss=None, stream=None):
        """One Adam step; ``loss`` (a one-element device tensor) receives the
        loss before the update."""
        x, y = self._f32(x), self._f32(y)
        _check(lib().kamx_mlp_train_step(self.handle, _ptr(x), _ptr(y), x.shape[0], float(lr), _ptr(loss),
                                         _stream(stream)))

    def weights(self):
        w = torch.empty(self.n_params, dtype=torch.float32, device=self.device)
        _check(lib().kamx_mlp_weights(self.handle, _ptr(w), 0, _stream(None)))
        return w

    def set_weights(self, w):
        w = self._f32(w)
        _check(lib().kamx_mlp_weights(self.handle, _ptr(w), 1, _stream(None)))
        torch.cuda.current_stream(self.device).synchronize()

    def gradients(self):
        g = torch.empty(self.n_params, dtype=torch.float32, device=self.device)
        _check(lib().kamx_mlp_gradients(self.handle, _ptr(g), _stream(None)))
        return g
