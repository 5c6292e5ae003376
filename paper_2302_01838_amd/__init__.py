"""Python binding of libvmap: vectorised per-object neural-field training on MI355X (gfx950).

Thin ctypes marshalling over the C ABI in ``include/vmap.h``: every step of the computation runs
in the library's HIP kernels. PyTorch supplies device memory (tensors) and the current HIP
stream. There is no fallback: if ``libvmap.so`` is missing, importing the binding's entry points
raises.

    objs = ObjectSet(max_objects=50, B=B, precision="bf16", max_rays=40000)
    ids = [objs.add(centre, scale, seed=s) for centre, scale, s in ...]
    batch = DeviceBatch(batch_dict)            # rays of several objects, CSR-segmented
    losses = objs.step(batch)                  # one vectorised training step
"""
from __future__ import annotations

import ctypes
import os
from typing import Dict, Optional, Sequence

import numpy as np

__all__ = ["VmapError", "load_library", "library_path", "ObjectSet", "DeviceBatch", "RenderLoss",
           "VMAP_FP32", "VMAP_BF16", "STATE_PARAMS", "STATE_ADAM_M", "STATE_ADAM_V",
           "STATE_GRAD", "STATE_STEP", "STATE_SCALER", "DERR_OBJECT", "DERR_PAIRS",
           "DERR_OFFSETS", "DERR_T_ORDER", "DERR_DUP_ID", "EXPORTED"]

VMAP_FP32, VMAP_BF16 = 0, 1
STATE_PARAMS, STATE_ADAM_M, STATE_ADAM_V, STATE_GRAD, STATE_STEP, STATE_SCALER = 0, 1, 2, 3, 4, 5
# device error bits reported by step_info() (include/vmap.h, vmap_step_info)
DERR_OBJECT, DERR_PAIRS, DERR_OFFSETS, DERR_T_ORDER, DERR_DUP_ID = 1, 2, 4, 8, 16
_STATUS = {0: "VMAP_OK", 1: "VMAP_EINVAL", 2: "VMAP_ECAPACITY", 3: "VMAP_EHIP", 4: "VMAP_ESTATE",
           5: "VMAP_ENOTSUP"}

_HERE = os.path.dirname(os.path.abspath(__file__))


def library_path() -> str:
    return os.path.join(_HERE, "libvmap.so")


class VmapError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{_STATUS.get(code, code)}: {msg}")
        self.code = code


class VmapConfig(ctypes.Structure):
    _fields_ = [("max_objects", ctypes.c_int32), ("n_features", ctypes.c_int32),
                ("hidden", ctypes.c_int32), ("n_hidden_layers", ctypes.c_int32),
                ("max_hidden", ctypes.c_int32), ("max_samples_per_ray", ctypes.c_int32),
                ("max_rays", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("rays_per_tile", ctypes.c_int32), ("scale_growth_interval", ctypes.c_int32),
                ("rays_per_tile_wide", ctypes.c_int32), ("split_step", ctypes.c_int32),
                ("lr", ctypes.c_double), ("beta1", ctypes.c_double), ("beta2", ctypes.c_double),
                ("eps", ctypes.c_double), ("lambda_colour", ctypes.c_double),
                ("lambda_occ", ctypes.c_double), ("loss_scale_init", ctypes.c_double)]


class VmapObjectDesc(ctypes.Structure):
    _fields_ = [("centre", ctypes.c_float * 3), ("scale", ctypes.c_float),
                ("hidden", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("seed", ctypes.c_uint64)]


class VmapBatch(ctypes.Structure):
    _fields_ = [("n_objects", ctypes.c_int32), ("n_rays_total", ctypes.c_int32),
                ("samples_per_ray", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("object_ids", ctypes.c_void_p), ("ray_offsets", ctypes.c_void_p),
                ("rays_o", ctypes.c_void_p), ("rays_d", ctypes.c_void_p), ("t", ctypes.c_void_p),
                ("depth", ctypes.c_void_p), ("rgb", ctypes.c_void_p), ("mask", ctypes.c_void_p),
                ("var", ctypes.c_void_p)]


_P = ctypes.c_void_p
_I = ctypes.c_int32
_CFG = ctypes.POINTER(VmapConfig)
_BATCH = ctypes.POINTER(VmapBatch)

# name -> (restype, argtypes); the exported C ABI of include/vmap.h
EXPORTED = {
    "vmap_state_bytes": (ctypes.c_size_t, [_CFG]),
    "vmap_workspace_bytes": (ctypes.c_size_t, [_CFG]),
    "vmap_object_params": (_I, [_CFG, _I]),
    "vmap_init_objects": (ctypes.c_int, [_CFG, _P, _P, ctypes.c_size_t, _P, ctypes.c_size_t, _P,
                                         ctypes.POINTER(_P)]),
    "vmap_add_object": (ctypes.c_int, [_P, ctypes.POINTER(VmapObjectDesc), _P, _P,
                                       ctypes.POINTER(_I)]),
    "vmap_train_step": (ctypes.c_int, [_P, _BATCH, _P, _P]),
    "vmap_render": (ctypes.c_int, [_P, _BATCH, _P, _P, _P, _P]),
    "vmap_query_occupancy": (ctypes.c_int, [_P, _I, _P, ctypes.c_int64, _P, _P, _P]),
    "vmap_scene_scratch_bytes": (ctypes.c_size_t, [_I, _I, _I, _I]),
    "vmap_render_scene": (ctypes.c_int, [_P, _I, _P, _P, _I, _P, _I, ctypes.c_float,
                                         ctypes.c_float, _I, _P, ctypes.c_size_t, _P, _P, _P,
                                         _P, _P, _P]),
    "vmap_render_scene_static": (ctypes.c_int, [_P, _I, _P, _P, _I, _P, _I, ctypes.c_float,
                                                ctypes.c_float, _I, _P, _P, _P, _P, _P, _P]),
    "vmap_sample_rays": (ctypes.c_int, [_P, _I, _I, _I, _P, _P, _P, ctypes.c_float, ctypes.c_uint64,
                                        _P, _P]),
    "vmap_forward": (ctypes.c_int, [_P, _BATCH, _P, _P, _P, _P, _P]),
    "vmap_backward": (ctypes.c_int, [_P, _BATCH, _P, _P, _P]),
    "vmap_adam_step": (ctypes.c_int, [_P, _BATCH, _P]),
    "vmap_get_state": (ctypes.c_int, [_P, _I, _I, _P, ctypes.c_size_t, _P]),
    "vmap_set_state": (ctypes.c_int, [_P, _I, _I, _P, ctypes.c_size_t, _P]),
    "vmap_step_info": (ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_float), ctypes.POINTER(_I),
                                      ctypes.POINTER(_I), _P]),
    "vmap_param_layout": (ctypes.c_int, [_P, _I, ctypes.POINTER(_I), ctypes.POINTER(_I)]),
    "vmap_set_graph_mode": (ctypes.c_int, [_P, _I]),
    "vmap_set_launch": (ctypes.c_int, [_P, _I, _I]),
    "vmap_kernel_timing": (ctypes.c_int, [_P, _I, ctypes.POINTER(ctypes.c_double),
                                          ctypes.POINTER(_I)]),
    "vmap_last_error": (ctypes.c_char_p, [_P]),
    "vmap_destroy": (None, [_P]),
}

_lib = None


def load_library():
    """Load libvmap.so (built by ``__graft_entry__.build()``); raises if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    path = library_path()
    if not os.path.exists(path):
        raise ImportError(f"{path} is not built; run `python -m paper_2302_01838_amd.build`")
    # torch first: the library then binds to the HIP runtime torch has already loaded, so the
    # process holds one runtime (a second copy loaded first finds no device once torch's runtime
    # owns it)
    _torch()
    lib = ctypes.CDLL(path)
    for name, (res, args) in EXPORTED.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def default_config(**kw) -> VmapConfig:
    c = VmapConfig(max_objects=64, n_features=16, hidden=32, n_hidden_layers=4, max_hidden=0,
                   max_samples_per_ray=32, max_rays=1 << 16, precision=VMAP_FP32,
                   rays_per_tile=0, scale_growth_interval=2000, lr=1e-3, beta1=0.9, beta2=0.999,
                   eps=1e-8, lambda_colour=5.0, lambda_occ=10.0, loss_scale_init=4096.0)
    for k, v in kw.items():
        setattr(c, k, v)
    if c.max_hidden == 0:
        c.max_hidden = c.hidden
    return c


def _torch():
    import torch
    return torch


def _stream():
    return ctypes.c_void_p(_torch().cuda.current_stream().cuda_stream)


class DeviceBatch:
    """A batch resident in device memory (torch tensors), with its C ``vmap_batch`` view."""

    FIELDS = ("object_ids", "ray_offsets", "rays_o", "rays_d", "t", "depth", "rgb", "mask")

    def __init__(self, batch: Dict[str, np.ndarray], device=None):
        torch = _torch()
        dev = device or torch.device("cuda", torch.cuda.current_device())
        self.S = int(batch["S"])
        self.tensors = {}
        for k in self.FIELDS:
            arr = np.ascontiguousarray(batch[k])
            dt = torch.int32 if k in ("object_ids", "ray_offsets") else torch.float32
            self.tensors[k] = torch.as_tensor(arr).to(device=dev, dtype=dt).contiguous()
        self.n_objects = int(self.tensors["object_ids"].numel())
        self.n_rays = int(np.asarray(batch["ray_offsets"])[-1]) if self.n_objects else 0
        self.n_samples = self.n_rays * self.S
        self.object_ids = np.asarray(batch["object_ids"], dtype=np.int32)
        self.ray_offsets = np.asarray(batch["ray_offsets"], dtype=np.int64)
        if batch.get("var") is not None:  # integrated encoding: per-sample variances [R, S]
            self.tensors["var"] = torch.as_tensor(np.ascontiguousarray(batch["var"])).to(
                device=dev, dtype=torch.float32).contiguous()
        self.c = VmapBatch(n_objects=self.n_objects, n_rays_total=self.n_rays,
                           samples_per_ray=self.S, reserved=0,
                           **{k: self.tensors[k].data_ptr() for k in self.FIELDS},
                           var=self.tensors["var"].data_ptr() if "var" in self.tensors else None)

    def __getitem__(self, k):
        return self.tensors[k]


class ObjectSet:
    """A stack of per-object MLPs trained together (the library context plus its buffers)."""

    def __init__(self, max_objects: int, B: np.ndarray, hidden: int = 32, precision: str = "fp32",
                 max_rays: int = 1 << 16, max_samples_per_ray: int = 32,
                 max_hidden: Optional[int] = None, rays_per_tile: int = 0,
                 rays_per_tile_wide: int = 0, lr: float = 1e-3,
                 betas=(0.9, 0.999), eps: float = 1e-8, lambda_colour: float = 5.0,
                 lambda_occ: float = 10.0, loss_scale_init: float = 4096.0,
                 scale_growth_interval: int = 2000, device=None, autotune: bool = True,
                 split_step: bool = False, log_path: Optional[str] = None):
        torch = _torch()
        self.lib = load_library()
        # per-step JSON lines (step, per-object losses, total, loss scale, skipped objects, step
        # time); each logged step synchronises the stream to read them
        self.log_path = log_path
        self.steps_taken = 0
        self.device = device or torch.device("cuda", torch.cuda.current_device())
        # launch shape from the autotuner's cache when none is given
        self.tuned = None
        if rays_per_tile == 0 and autotune:
            from .tune import lookup
            # hidden 16 runs in the width-32 kernels (zero-padded) and takes their tuned shape
            self.tuned = lookup(32 if hidden == 16 else hidden, max_samples_per_ray, precision)
            if self.tuned:
                rays_per_tile = int(self.tuned["rays_per_tile"])
        if rays_per_tile_wide == 0 and autotune and (max_hidden or hidden) > 32:
            from .tune import lookup
            wide = lookup(max_hidden or hidden, max_samples_per_ray, precision)
            if wide and wide.get("rays_per_tile_wide"):
                rays_per_tile_wide = int(wide["rays_per_tile_wide"])
        self.cfg = default_config(
            max_objects=max_objects, hidden=hidden, max_hidden=max_hidden or hidden,
            max_samples_per_ray=max_samples_per_ray, max_rays=max_rays,
            precision=VMAP_BF16 if precision == "bf16" else VMAP_FP32,
            rays_per_tile=rays_per_tile, rays_per_tile_wide=rays_per_tile_wide,
            scale_growth_interval=scale_growth_interval, lr=lr,
            beta1=betas[0], beta2=betas[1], eps=eps, lambda_colour=lambda_colour,
            lambda_occ=lambda_occ, loss_scale_init=loss_scale_init,
            split_step=1 if split_step else 0)
        self.precision = precision
        sb = self.lib.vmap_state_bytes(ctypes.byref(self.cfg))
        wb = self.lib.vmap_workspace_bytes(ctypes.byref(self.cfg))
        if sb == 0 or wb == 0:
            raise VmapError(1, "invalid configuration")
        self.state = torch.empty(sb, dtype=torch.uint8, device=self.device)
        self.workspace = torch.empty(wb, dtype=torch.uint8, device=self.device)
        Bc = np.ascontiguousarray(B, dtype=np.float32)
        assert Bc.shape == (3, 16)
        ctx = ctypes.c_void_p()
        rc = self.lib.vmap_init_objects(ctypes.byref(self.cfg), Bc.ctypes.data,
                                        self.state.data_ptr(), sb, self.workspace.data_ptr(), wb,
                                        _stream(), ctypes.byref(ctx))
        if rc != 0:
            raise VmapError(rc, self.lib.vmap_last_error(None).decode())
        self.ctx = ctx
        self.n_params: Dict[int, int] = {}
        self.p_stride = 0
        # launch shape (the library's default tile: two sub-tiles of floor(64 / S) rays for each
        # of four waves)
        self.rays_per_tile = rays_per_tile or max(1, 64 // max_samples_per_ray) * 8
        self.waves, self.grid = 4, 0
        if self.tuned:
            self.set_launch(int(self.tuned["waves"]), int(self.tuned["grid"]))

    # -- helpers
    def _check(self, rc: int):
        if rc != 0:
            raise VmapError(rc, self.lib.vmap_last_error(self.ctx).decode())

    def close(self):
        if getattr(self, "ctx", None):
            self.lib.vmap_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- model stack
    def add(self, centre, scale: float, hidden: int = 0, seed: int = 0,
            init: Optional[np.ndarray] = None) -> int:
        d = VmapObjectDesc(hidden=hidden, reserved=0, seed=int(seed) & ((1 << 64) - 1))
        for i in range(3):
            d.centre[i] = float(centre[i])
        d.scale = float(scale)
        oid = ctypes.c_int32()
        ptr = None
        if init is not None:
            init = np.ascontiguousarray(init, dtype=np.float32)
            ptr = init.ctypes.data
        self._check(self.lib.vmap_add_object(self.ctx, ctypes.byref(d), ptr, _stream(),
                                             ctypes.byref(oid)))
        k = oid.value
        n, s = ctypes.c_int32(), ctypes.c_int32()
        self._check(self.lib.vmap_param_layout(self.ctx, k, ctypes.byref(n), ctypes.byref(s)))
        self.n_params[k] = n.value
        self.p_stride = s.value
        return k

    # -- the step and its parts
    def step(self, batch: DeviceBatch, losses=None):
        torch = _torch()
        if losses is None:
            losses = torch.empty(batch.n_objects, dtype=torch.float32, device=self.device)
        if self.log_path:
            ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
            ev[0].record()
        self._check(self.lib.vmap_train_step(self.ctx, ctypes.byref(batch.c),
                                             losses.data_ptr() if batch.n_objects else None,
                                             _stream()))
        self.steps_taken += 1
        if self.log_path:
            ev[1].record()
            ev[1].synchronize()
            self._log_step(batch, losses, ev[0].elapsed_time(ev[1]))
        return losses

    def _log_step(self, batch: DeviceBatch, losses, ms):
        import json
        scale, skipped, err = self.step_info()
        lv = losses.cpu().numpy().astype(float)
        rec = {"step": self.steps_taken, "objects": batch.object_ids.tolist(),
               "loss": lv.tolist(), "total": float(lv.sum()), "loss_scale": scale,
               "skipped": skipped, "device_error": err, "step_us": ms * 1e3}
        with open(self.log_path, "a") as f:
            f.write(json.dumps(rec) + "\n")

    def forward(self, batch: DeviceBatch, renders: bool = True):
        torch = _torch()
        loss = torch.empty(batch.n_objects, dtype=torch.float32, device=self.device)
        R = batch.n_rays
        depth = torch.empty(R, dtype=torch.float32, device=self.device) if renders else None
        rgb = torch.empty(R, 3, dtype=torch.float32, device=self.device) if renders else None
        occ = torch.empty(R, dtype=torch.float32, device=self.device) if renders else None
        ptr = lambda x: None if x is None or x.numel() == 0 else x.data_ptr()
        self._check(self.lib.vmap_forward(self.ctx, ctypes.byref(batch.c), ptr(loss), ptr(depth),
                                          ptr(rgb), ptr(occ), _stream()))
        return loss, depth, rgb, occ

    def backward(self, batch: DeviceBatch, dloss):
        torch = _torch()
        dloss = dloss.to(device=self.device, dtype=torch.float32).contiguous()
        grad = torch.empty(batch.n_objects, self.p_stride, dtype=torch.float32, device=self.device)
        self._check(self.lib.vmap_backward(self.ctx, ctypes.byref(batch.c),
                                           dloss.data_ptr() if batch.n_objects else None,
                                           grad.data_ptr() if batch.n_objects else None,
                                           _stream()))
        return grad

    def adam_step(self, batch: DeviceBatch):
        self._check(self.lib.vmap_adam_step(self.ctx, ctypes.byref(batch.c), _stream()))

    def render(self, batch: DeviceBatch):
        torch = _torch()
        R = batch.n_rays
        depth = torch.empty(R, dtype=torch.float32, device=self.device)
        rgb = torch.empty(R, 3, dtype=torch.float32, device=self.device)
        occ = torch.empty(R, dtype=torch.float32, device=self.device)
        self._check(self.lib.vmap_render(self.ctx, ctypes.byref(batch.c),
                                         depth.data_ptr() if R else None,
                                         rgb.data_ptr() if R else None,
                                         occ.data_ptr() if R else None, _stream()))
        return depth, rgb, occ

    def render_scene(self, rays_o, rays_d, object_ids=None, S: int = 32, t_min: float = 0.0,
                     occ_threshold: float = 0.5, max_pairs: Optional[int] = None):
        """Scene render from the object models (Sec. 3.4): per ray the nearest object (by
        rendered depth) whose rendered occupancy reaches ``occ_threshold``. Returns depth [R],
        rgb [R, 3], occupancy [R], object id [R] (-1: none) and the number of (ray, object)
        pairs found (a device scalar)."""
        torch = _torch()
        f = lambda x: torch.as_tensor(x).to(device=self.device, dtype=torch.float32).contiguous()
        ro, rd = f(rays_o), f(rays_d)
        R = ro.shape[0]
        if object_ids is None:
            object_ids = [k for k in range(self.cfg.max_objects) if k in self.n_params]
        ids = torch.as_tensor(np.asarray(object_ids, np.int32)).to(self.device)
        n = int(ids.numel())
        if max_pairs is None:
            max_pairs = min(R * n, self.cfg.max_rays)
        nbytes = self.lib.vmap_scene_scratch_bytes(R, n, max_pairs, S)
        scratch = torch.empty(max(nbytes, 1) + 256, dtype=torch.uint8, device=self.device)
        base = (scratch.data_ptr() + 255) // 256 * 256
        depth = torch.zeros(R, dtype=torch.float32, device=self.device)
        rgb = torch.zeros(R, 3, dtype=torch.float32, device=self.device)
        occ = torch.zeros(R, dtype=torch.float32, device=self.device)
        kid = torch.full((R,), -1, dtype=torch.int32, device=self.device)
        npairs = torch.zeros(1, dtype=torch.int32, device=self.device)
        ptr = lambda t: t.data_ptr() if t.numel() else None
        self._check(self.lib.vmap_render_scene(
            self.ctx, R, ptr(ro), ptr(rd), n, ptr(ids), S, float(t_min), float(occ_threshold),
            int(max_pairs), base, nbytes, ptr(depth), ptr(rgb), ptr(occ), ptr(kid), ptr(npairs),
            _stream()))
        return depth, rgb, occ, kid, npairs

    def query(self, k: int, pts):
        torch = _torch()
        pts = torch.as_tensor(pts).to(device=self.device, dtype=torch.float32).contiguous()
        n = pts.shape[0]
        occ = torch.empty(n, dtype=torch.float32, device=self.device)
        rgb = torch.empty(n, 3, dtype=torch.float32, device=self.device)
        self._check(self.lib.vmap_query_occupancy(self.ctx, k, pts.data_ptr() if n else None, n,
                                                  occ.data_ptr() if n else None,
                                                  rgb.data_ptr() if n else None, _stream()))
        return occ, rgb

    def sample_rays(self, t_near, t_far, depth, S: int, n_strat: int, sigma: float = 0.03,
                    seed: int = 0, out=None):
        """Depth-guided, sorted sample depths [R, S] on the device (Sec. 3.3, Eqs. 1-2), into
        ``out`` (a contiguous FP32 device tensor of R x S values, e.g. a batch's ``t``) if given."""
        torch = _torch()
        f = lambda x: torch.as_tensor(x).to(device=self.device, dtype=torch.float32).contiguous()
        tn, tf, d = f(t_near), f(t_far), f(depth)
        R = tn.numel()
        if out is None:
            out = torch.empty(R, S, dtype=torch.float32, device=self.device)
        elif (out.dtype != torch.float32 or not out.is_contiguous() or out.numel() != R * S
              or out.device != self.device):
            raise ValueError("out must be a contiguous float32 tensor of n_rays x S on the stack's device")
        ptr = lambda x: x.data_ptr() if R else None
        self._check(self.lib.vmap_sample_rays(self.ctx, R, S, n_strat, ptr(tn), ptr(tf), ptr(d),
                                              float(sigma), int(seed) & ((1 << 64) - 1),
                                              ptr(out), _stream()))
        return out

    # -- state I/O and diagnostics
    def get_state(self, k: int, which: int = STATE_PARAMS):
        if which == STATE_SCALER:  # (scale, consecutive good steps); k is ignored
            out = np.zeros(2, dtype=np.int32)
            self._check(self.lib.vmap_get_state(self.ctx, -1, which, out.ctypes.data, 8, _stream()))
            return float(out[:1].view(np.float32)[0]), int(out[1])
        if which == STATE_STEP:
            out = np.zeros(1, dtype=np.int32)
        else:
            out = np.zeros(self.n_params[k], dtype=np.float32)
        self._check(self.lib.vmap_get_state(self.ctx, k, which, out.ctypes.data, out.nbytes,
                                            _stream()))
        return out if which != STATE_STEP else int(out[0])

    def set_state(self, k: int, which: int, value) -> None:
        if which == STATE_SCALER:
            arr = np.zeros(2, dtype=np.int32)
            arr[:1].view(np.float32)[0] = value[0]
            arr[1] = value[1]
            k = -1
        elif which == STATE_STEP:
            arr = np.asarray([value], dtype=np.int32)
        else:
            arr = np.ascontiguousarray(value, dtype=np.float32)
        self._check(self.lib.vmap_set_state(self.ctx, k, which, arr.ctypes.data, arr.nbytes,
                                            _stream()))

    def save(self, path: str) -> None:
        """Checkpoint every object's parameters, Adam moments and step count, and the loss
        scaler, to an .npz file (plain arrays, no pickled objects)."""
        arrays = {}
        for k in sorted(self.n_params):
            arrays[f"theta_{k}"] = self.get_state(k, STATE_PARAMS)
            arrays[f"m_{k}"] = self.get_state(k, STATE_ADAM_M)
            arrays[f"v_{k}"] = self.get_state(k, STATE_ADAM_V)
            arrays[f"step_{k}"] = np.asarray([self.get_state(k, STATE_STEP)], np.int32)
        scale, good = self.get_state(-1, STATE_SCALER)
        arrays["scaler_scale"] = np.asarray([scale], np.float32)
        arrays["scaler_good"] = np.asarray([good], np.int32)
        np.savez(path, **arrays)

    def load(self, path: str) -> None:
        """Restore a checkpoint written by save() into objects already added with the same ids
        and widths."""
        with np.load(path, allow_pickle=False) as z:
            for k in sorted(self.n_params):
                self.set_state(k, STATE_PARAMS, z[f"theta_{k}"])
                self.set_state(k, STATE_ADAM_M, z[f"m_{k}"])
                self.set_state(k, STATE_ADAM_V, z[f"v_{k}"])
                self.set_state(k, STATE_STEP, int(z[f"step_{k}"][0]))
            self.set_state(-1, STATE_SCALER, (float(z["scaler_scale"][0]), int(z["scaler_good"][0])))

    def step_info(self):
        s = ctypes.c_float()
        sk, er = ctypes.c_int32(), ctypes.c_int32()
        self._check(self.lib.vmap_step_info(self.ctx, ctypes.byref(s), ctypes.byref(sk),
                                            ctypes.byref(er), _stream()))
        return s.value, sk.value, er.value

    def set_graph_mode(self, on: bool):
        self._check(self.lib.vmap_set_graph_mode(self.ctx, 1 if on else 0))

    def set_launch(self, waves: int = 4, grid_blocks: int = 0):
        self._check(self.lib.vmap_set_launch(self.ctx, waves, grid_blocks))
        self.waves, self.grid = int(waves), int(grid_blocks)

    def kernel_timing(self, enable: int = -1):
        avg = ctypes.c_double()
        cnt = ctypes.c_int32()
        self._check(self.lib.vmap_kernel_timing(self.ctx, enable, ctypes.byref(avg),
                                                ctypes.byref(cnt)))
        return avg.value, cnt.value


def _render_loss_backward(ctx, dloss, *unused):
    grad = ctx.objset.backward(ctx.batch, dloss)
    return grad, None, None


class RenderLoss:
    """``torch.autograd.Function`` over the library's forward and hand-written adjoint.

    ``RenderLoss.apply(token, objset, batch)`` returns the per-object losses of the batch;
    ``token`` is a [n_objects, p_stride] tensor with ``requires_grad`` that carries the gradient
    of the batch objects' parameters (the parameters themselves live in the library state).
    After ``backward`` the library's gradient slots hold the same gradient, so
    ``objset.adam_step(batch)`` applies the update.
    """

    _fn = None

    @classmethod
    def function(cls):
        if cls._fn is None:
            torch = _torch()

            class _RenderLoss(torch.autograd.Function):
                @staticmethod
                def forward(ctx, token, objset, batch):
                    ctx.objset = objset
                    ctx.batch = batch
                    loss, _, _, _ = objset.forward(batch, renders=False)
                    return loss

                @staticmethod
                def backward(ctx, dloss):
                    return _render_loss_backward(ctx, dloss)

            cls._fn = _RenderLoss
        return cls._fn

    @classmethod
    def apply(cls, token, objset, batch):
        return cls.function().apply(token, objset, batch)
