"""ctypes binding of libhandtrack.so (argument marshalling only).

Device memory and streams come from PyTorch (ROCm): tensors are passed by ``data_ptr()`` and
the current stream by ``torch.cuda.current_stream().cuda_stream``.  Every compute step runs in
the library's HIP kernels; if the library is missing or fails, the calls raise.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libhandtrack.so")

HT_OK, HT_ERR_ARG, HT_ERR_STATE, HT_ERR_OOM, HT_ERR_HIP, HT_ERR_UNSUPPORTED = 0, -1, -2, -3, -4, -5
HT_PTR_HOST, HT_PTR_DEVICE = 0, 1
HT_DEVERR_UNSET_SLOT = 1
_NAMES = {0: "HT_OK", -1: "HT_ERR_ARG", -2: "HT_ERR_STATE", -3: "HT_ERR_OOM", -4: "HT_ERR_HIP",
          -5: "HT_ERR_UNSUPPORTED"}


class HandtrackError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{_NAMES.get(status, status)}: {message}")
        self.status = status


class Model(C.Structure):
    _fields_ = [
        ("n_dof", C.c_int32), ("n_seg", C.c_int32), ("n_prim", C.c_int32), ("n_kc", C.c_int32),
        ("seg_parent", C.c_void_p), ("seg_root_dof", C.c_void_p), ("seg_offset", C.c_void_p),
        ("seg_joint_axis", C.c_void_p), ("seg_joint_dof", C.c_void_p),
        ("prim_type", C.c_void_p), ("prim_seg", C.c_void_p), ("prim_frame", C.c_void_p),
        ("prim_size", C.c_void_p), ("bounds_lo", C.c_void_p), ("bounds_hi", C.c_void_p),
        ("mutate_mask", C.c_void_p), ("kc_pairs", C.c_void_p),
    ]


class Camera(C.Structure):
    _fields_ = [("fx", C.c_float), ("fy", C.c_float), ("cx", C.c_float), ("cy", C.c_float)]


class Debug(C.Structure):
    _fields_ = [("slot", C.c_int32), ("depth", C.c_void_p), ("hit", C.c_void_p),
                ("rm", C.c_void_p), ("winner", C.c_void_p), ("margin", C.c_void_p)]


class Swarm(C.Structure):
    _fields_ = [
        ("n_frames", C.c_int32), ("n_particles", C.c_int32), ("frame_slots", C.c_void_p),
        ("x", C.c_void_p), ("v", C.c_void_p), ("pbest_x", C.c_void_p), ("pbest_cost", C.c_void_p),
        ("gbest_x", C.c_void_p), ("gbest_cost", C.c_void_p), ("cost", C.c_void_p),
        ("gen", C.c_void_p), ("init_lo", C.c_void_p), ("init_hi", C.c_void_p),
        ("seed", C.c_uint64), ("stop_gen", C.c_void_p), ("seed_dev", C.c_void_p),
    ]


class PsoParams(C.Structure):
    _fields_ = [("w", C.c_float), ("c1", C.c_float), ("c2", C.c_float),
                ("mutate_every", C.c_int32), ("mutate_frac", C.c_float),
                ("refine_topk", C.c_int32), ("refine_steps", C.c_int32),
                ("eta_rot", C.c_float), ("eta_trans", C.c_float), ("stop_cost", C.c_float)]


class SegParams(C.Structure):
    _fields_ = [("cb_lo", C.c_int32), ("cb_hi", C.c_int32), ("cr_lo", C.c_int32),
                ("cr_hi", C.c_int32), ("band_mm", C.c_int32), ("bg_depth_mm", C.c_float)]


class LaunchConfig(C.Structure):
    _fields_ = [("tiles_per_item", C.c_int32), ("groups_per_cu", C.c_int32), ("cull", C.c_int32)]


class KernelStat(C.Structure):
    _fields_ = [("launches", C.c_int32), ("particles", C.c_int64), ("total_ms", C.c_double)]


KERNEL_KINDS = ("fk", "sched", "raycast", "raycast_grad", "finalize", "pso", "refine")


_lib = None


def load_library(path: str = LIB_PATH):
    """Load libhandtrack.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with paper_2005_07068_amd.build.build()")
    lib = C.CDLL(path)
    P, I, F, S = C.c_void_p, C.c_int, C.c_float, C.c_int
    lib.ht_last_error.restype = C.c_char_p
    lib.ht_version.restype = C.c_char_p
    lib.ht_create.argtypes = [C.POINTER(C.c_void_p), I]
    lib.ht_destroy.argtypes = [P]
    lib.ht_destroy.restype = None
    lib.ht_set_model.argtypes = [P, C.POINTER(Model)]
    lib.ht_check_model.argtypes = [C.POINTER(Model)]
    lib.ht_check_model.restype = S
    lib.ht_set_observation.argtypes = [P, I, I, I, P, P, Camera, F, I, P]
    lib.ht_set_pixel_mask.argtypes = [P, I, P, I, P]
    lib.ht_reserve.argtypes = [P, I, I]
    lib.ht_eval_particles.argtypes = [P, I, P, I, P, P, C.POINTER(Debug), P]
    lib.ht_eval_particles_grad.argtypes = [P, I, P, I, P, P, P, P, P]
    lib.ht_eval_particles_noalloc.argtypes = [P, I, P, I, P, P, P]
    lib.ht_pso_init.argtypes = [P, C.POINTER(Swarm), P]
    lib.ht_pso_step.argtypes = [P, C.POINTER(Swarm), C.POINTER(PsoParams), P]
    lib.ht_pso_run_graph.argtypes = [P, C.POINTER(Swarm), C.POINTER(PsoParams), I, P]
    lib.ht_pso_box_around.argtypes = [P, I, P, P, P, P, P]
    lib.ht_preprocess_rgbd.argtypes = [P, I, I, P, P, C.POINTER(SegParams), P, P, P]
    lib.ht_get_launch_config.argtypes = [P, C.POINTER(LaunchConfig)]
    lib.ht_set_launch_config.argtypes = [P, C.POINTER(LaunchConfig)]
    lib.ht_autotune.argtypes = [P, I, P, I, P, P, I, C.POINTER(LaunchConfig), P]
    lib.ht_profile_begin.argtypes = [P]
    lib.ht_profile_end.argtypes = [P, C.POINTER(KernelStat)]
    lib.ht_eval_counts.argtypes = [P, C.POINTER(C.c_int64), C.POINTER(C.c_int64), I]
    lib.ht_device_errors.argtypes = [P, C.POINTER(C.c_uint32), I]
    for name in ("ht_profile_begin", "ht_profile_end", "ht_create", "ht_set_model", "ht_set_observation", "ht_set_pixel_mask",
                 "ht_reserve",
                 "ht_eval_particles", "ht_eval_particles_grad", "ht_eval_particles_noalloc",
                 "ht_pso_init", "ht_pso_step",
                 "ht_pso_run_graph", "ht_get_launch_config", "ht_set_launch_config",
                 "ht_autotune", "ht_eval_counts", "ht_device_errors"):
        getattr(lib, name).restype = S
    _lib = lib
    return lib


def _check(status: int):
    if status != HT_OK:
        raise HandtrackError(status, load_library().ht_last_error().decode())


def _ptr(t):
    return C.c_void_p(0 if t is None else t.data_ptr())


def _dev(t, dtype, shape, name):
    """Check that t is a contiguous cuda tensor of the given torch dtype and shape (None in
    shape: any size), so that the library never receives a host pointer or a misread type."""
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError(f"{name} must be a cuda tensor (got a {t.device} tensor)")
    if t.dtype != dtype:
        raise ValueError(f"{name} must be {dtype} (got {t.dtype})")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if len(shape) != t.dim() or any(e is not None and e != g for e, g in zip(shape, t.shape)):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {shape}")
    return t


def _stream():
    import torch
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def torch_float32():
    import torch
    return torch.float32


def pso_params(w=0.72, c1=2.05, c2=2.05, mutate_every=3, mutate_frac=0.5, refine_topk=0,
               refine_steps=0, eta_rot=0.02, eta_trans=2.0, stop_cost=0.0) -> PsoParams:
    return PsoParams(w, c1, c2, mutate_every, mutate_frac, refine_topk, refine_steps, eta_rot,
                     eta_trans, stop_cost)


def model_struct(m: dict):
    """ctypes ht_model over contiguous copies of the tables; returns (struct, arrays to keep)."""
    arrs = {
        "seg_parent": np.ascontiguousarray(m["seg_parent"], np.int32),
        "seg_root_dof": np.ascontiguousarray(m["seg_root_dof"], np.int32),
        "seg_offset": np.ascontiguousarray(m["seg_offset"], np.float64),
        "seg_joint_axis": np.ascontiguousarray(m["seg_joint_axis"], np.float64),
        "seg_joint_dof": np.ascontiguousarray(m["seg_joint_dof"], np.int32),
        "prim_type": np.ascontiguousarray(m["prim_type"], np.int32),
        "prim_seg": np.ascontiguousarray(m["prim_seg"], np.int32),
        "prim_frame": np.ascontiguousarray(m["prim_frame"], np.float64),
        "prim_size": np.ascontiguousarray(m["prim_size"], np.float64),
        "bounds_lo": np.ascontiguousarray(m["bounds_lo"], np.float64),
        "bounds_hi": np.ascontiguousarray(m["bounds_hi"], np.float64),
        "mutate_mask": np.ascontiguousarray(m["mutate_mask"], np.uint8),
        "kc_pairs": np.ascontiguousarray(m["kc_pairs"], np.int32).reshape(-1, 2),
    }
    mm = Model(int(m["n_dof"]), int(m["n_seg"]), int(m["n_prim"]), len(arrs["kc_pairs"]),
               *[a.ctypes.data for a in arrs.values()])
    return mm, arrs


def check_model(m: dict) -> None:
    """Validate model tables with the library's checks (no device needed)."""
    mm, keep = model_struct(m)
    _check(load_library().ht_check_model(C.byref(mm)))
    del keep


class Context:
    """One library context on a HIP device (see include/handtrack.h for every call)."""

    def __init__(self, device: int = 0):
        self.lib = load_library()
        self.handle = C.c_void_p()
        _check(self.lib.ht_create(C.byref(self.handle), device))
        self.device = device
        self._keep = []
        self.n_dof = 0
        self.slots = {}

    def close(self):
        if self.handle:
            self.lib.ht_destroy(self.handle)
            self.handle = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- set-up -------------------------------------------------------------------------
    def set_model(self, m: dict):
        mm, keep = model_struct(m)
        _check(self.lib.ht_set_model(self.handle, C.byref(mm)))
        del keep
        self.n_dof = int(m["n_dof"])

    def set_observation(self, slot: int, depth, skin, cam, bg: float):
        """depth: uint16 [H, W], skin: uint8 [H, W] as numpy arrays (host) or torch tensors
        (host or device)."""
        import torch
        if isinstance(depth, torch.Tensor):
            kind = HT_PTR_DEVICE if depth.is_cuda else HT_PTR_HOST
            depth_t = depth.contiguous()
            skin_t = skin.to(torch.uint8).contiguous()
            H, W = depth_t.shape
            dp, sp = depth_t.data_ptr(), skin_t.data_ptr()
            self._keep = [depth_t, skin_t]
        else:
            kind = HT_PTR_HOST
            d = np.ascontiguousarray(depth, np.uint16)
            s = np.ascontiguousarray(skin, np.uint8)
            H, W = d.shape
            dp, sp = d.ctypes.data, s.ctypes.data
            self._keep = [d, s]
        fx, fy, cx, cy = (float(c) for c in cam)
        _check(self.lib.ht_set_observation(self.handle, slot, W, H, C.c_void_p(dp),
                                           C.c_void_p(sp), Camera(fx, fy, cx, cy), float(bg),
                                           kind, _stream()))
        self.slots[slot] = (W, H, float(bg))

    def set_pixel_mask(self, slot: int, mask=None):
        """Gradient pixel mask of a frame slot: uint8 [H, W] of the slot's ROI (numpy array, or
        torch tensor on the host or the device); None clears it."""
        import torch
        if mask is None:
            _check(self.lib.ht_set_pixel_mask(self.handle, slot, None, HT_PTR_HOST, _stream()))
            return
        if slot not in self.slots:
            raise ValueError(f"frame slot {slot} has no observation")
        W, H = self.slots[slot][:2]
        if isinstance(mask, torch.Tensor):
            m = mask.to(torch.uint8).contiguous()
            kind, ptr = (HT_PTR_DEVICE if m.is_cuda else HT_PTR_HOST), m.data_ptr()
        else:
            m = np.ascontiguousarray(mask, np.uint8)
            kind, ptr = HT_PTR_HOST, m.ctypes.data
        if tuple(m.shape) != (H, W):
            raise ValueError(f"mask shape {tuple(m.shape)} is not the slot's ({H}, {W})")
        _check(self.lib.ht_set_pixel_mask(self.handle, slot, C.c_void_p(ptr), kind, _stream()))

    def reserve(self, max_particles: int, max_pixels: int):
        _check(self.lib.ht_reserve(self.handle, max_particles, max_pixels))

    # -- evaluation ---------------------------------------------------------------------
    def eval(self, poses, frame_slots, cost=None, debug=None):
        """poses: float32 cuda tensor [F, P, D] (or [P, D] for one frame); frame_slots: int32
        cuda tensor [F].  Returns cost [F, P] (or [P])."""
        import torch
        squeeze = poses.dim() == 2
        p3 = poses.unsqueeze(0) if squeeze else poses
        F, P, D = p3.shape
        if D != self.n_dof:
            raise ValueError(f"poses have {D} parameters, model has {self.n_dof}")
        p3 = _dev(p3.contiguous(), torch.float32, (F, P, D), "poses")
        _dev(frame_slots, torch.int32, (F,), "frame_slots")
        if cost is None:
            cost = torch.empty((F, P), device=poses.device, dtype=torch.float32)
        _dev(cost, torch.float32, (F, P), "cost")
        dbg = None
        if debug is not None:
            slot = int(debug["slot"])
            if F != 1 or slot not in self.slots:
                raise ValueError("debug images need one frame whose slot is set")
            W, H, _ = self.slots[slot]
            keys = ("depth", "hit", "rm", "winner", "margin")
            for k, dt in zip(keys, (torch.float32, torch.uint8, torch.uint8, torch.int32,
                                    torch.float32)):
                _dev(debug.get(k), dt, (P, H, W), "debug " + k)
            dbg = Debug(slot, *[_ptr(debug.get(k)) for k in keys])
        _check(self.lib.ht_eval_particles(self.handle, F, _ptr(frame_slots), P, _ptr(p3),
                                          _ptr(cost), C.byref(dbg) if dbg else None, _stream()))
        return cost[0] if squeeze else cost

    def eval_noalloc(self, poses, frame_slots, cost=None):
        """eval through ht_eval_particles_noalloc (the library's fixed scratch array, no
        allocation on the device)."""
        import torch
        squeeze = poses.dim() == 2
        p3 = (poses.unsqueeze(0) if squeeze else poses).contiguous()
        F, P, D = p3.shape
        _dev(p3, torch.float32, (F, P, self.n_dof), "poses")
        _dev(frame_slots, torch.int32, (F,), "frame_slots")
        if cost is None:
            cost = torch.empty((F, P), device=poses.device, dtype=torch.float32)
        _dev(cost, torch.float32, (F, P), "cost")
        _check(self.lib.ht_eval_particles_noalloc(self.handle, F, _ptr(frame_slots), P,
                                                  _ptr(p3), _ptr(cost), _stream()))
        return cost[0] if squeeze else cost

    def eval_grad(self, poses, frame_slots, pixel_mask=None):
        import torch
        squeeze = poses.dim() == 2
        p3 = (poses.unsqueeze(0) if squeeze else poses).contiguous()
        F, P, D = p3.shape
        _dev(p3, torch.float32, (F, P, self.n_dof), "poses")
        _dev(frame_slots, torch.int32, (F,), "frame_slots")
        if pixel_mask is not None:
            # the frame's slot is on the device: the mask must fit one of the set slots
            _dev(pixel_mask, torch.uint8, (None, None), "pixel_mask")
            H, W = pixel_mask.shape
            if F != 1 or (int(W), int(H)) not in {sl[:2] for sl in self.slots.values()}:
                raise ValueError("pixel_mask needs one frame and the [H, W] of a set slot")
        cost = torch.empty((F, P), device=poses.device, dtype=torch.float32)
        grad = torch.empty((F, P, D), device=poses.device, dtype=torch.float32)
        _check(self.lib.ht_eval_particles_grad(self.handle, F, _ptr(frame_slots), P, _ptr(p3),
                                               _ptr(cost), _ptr(grad), _ptr(pixel_mask),
                                               _stream()))
        if squeeze:
            return cost[0], grad[0]
        return cost, grad

    # -- swarm --------------------------------------------------------------------------
    def swarm(self, frame_slots, n_particles: int, init_lo, init_hi, seed: int,
              device_seed: bool = False):
        """Allocate swarm state tensors; returns a dict (tensors) and its ctypes struct.
        With device_seed the Philox key is the int64 tensor t["seed_dev"] (initialised to seed),
        which the caller may rewrite between graph replays."""
        import torch
        dev = frame_slots.device
        F, D = int(frame_slots.numel()), self.n_dof
        t = {
            "frame_slots": frame_slots,
            "x": torch.zeros((F, n_particles, D), device=dev),
            "v": torch.zeros((F, n_particles, D), device=dev),
            "pbest_x": torch.zeros((F, n_particles, D), device=dev),
            "pbest_cost": torch.zeros((F, n_particles), device=dev),
            "gbest_x": torch.zeros((F, D), device=dev),
            "gbest_cost": torch.zeros((F,), device=dev),
            "cost": torch.zeros((F, n_particles), device=dev),
            "gen": torch.zeros((F,), device=dev, dtype=torch.int32),
            "init_lo": init_lo.to(dev, torch.float32).reshape(F, D).contiguous(),
            "init_hi": init_hi.to(dev, torch.float32).reshape(F, D).contiguous(),
            "stop_gen": torch.zeros((F,), device=dev, dtype=torch.int32),
        }
        if device_seed:
            t["seed_dev"] = torch.tensor([seed], device=dev, dtype=torch.int64)
        s = Swarm(F, n_particles, _ptr(t["frame_slots"]), _ptr(t["x"]), _ptr(t["v"]),
                  _ptr(t["pbest_x"]), _ptr(t["pbest_cost"]), _ptr(t["gbest_x"]),
                  _ptr(t["gbest_cost"]), _ptr(t["cost"]), _ptr(t["gen"]), _ptr(t["init_lo"]),
                  _ptr(t["init_hi"]), C.c_uint64(seed), _ptr(t["stop_gen"]),
                  _ptr(t.get("seed_dev")))
        t["_struct"] = s
        return t

    def pso_init(self, sw):
        _check(self.lib.ht_pso_init(self.handle, C.byref(sw["_struct"]), _stream()))

    def pso_step(self, sw, params: PsoParams):
        _check(self.lib.ht_pso_step(self.handle, C.byref(sw["_struct"]), C.byref(params),
                                    _stream()))

    def preprocess_rgbd(self, rgb, depth, bg_depth_mm: float, box=(77, 127, 133, 173),
                        band_mm: int = 150):
        """Skin-colour and depth segmentation of an RGB-D frame.  rgb: uint8 cuda tensor
        [H, W, 3]; depth: 16-bit cuda tensor [H, W] holding the uint16 depths (torch.uint16,
        or int16 with the same bits).  Returns (depth_out like depth, skin_out uint8)."""
        import torch
        if rgb.dim() != 3 or rgb.shape[2] != 3 or rgb.dtype != torch.uint8 or not rgb.is_cuda:
            raise ValueError("rgb must be a uint8 cuda tensor [H, W, 3]")
        H, W = int(rgb.shape[0]), int(rgb.shape[1])
        if tuple(depth.shape) != (H, W) or depth.element_size() != 2 or not depth.is_cuda:
            raise ValueError("depth must be a 16-bit cuda tensor [H, W]")
        rgb, depth = rgb.contiguous(), depth.contiguous()
        d_out = torch.empty((H, W), device=rgb.device, dtype=depth.dtype)
        s_out = torch.empty((H, W), device=rgb.device, dtype=torch.uint8)
        p = SegParams(*box, int(band_mm), float(bg_depth_mm))
        _check(self.lib.ht_preprocess_rgbd(self.handle, W, H, _ptr(rgb), _ptr(depth), C.byref(p),
                                           _ptr(d_out), _ptr(s_out), _stream()))
        return d_out, s_out

    def box_around(self, center, halfwidth, lo, hi):
        """lo, hi <- the model-bounded box center -/+ halfwidth (all float32 cuda tensors:
        center, lo, hi [F, n_dof]; halfwidth [n_dof])."""
        F = int(center.shape[0]) if center.dim() == 2 else 1
        for t in (center, halfwidth, lo, hi):
            if not (t.is_cuda and t.dtype == torch_float32() and t.is_contiguous()):
                raise ValueError("box_around takes contiguous float32 cuda tensors")
        if halfwidth.numel() != self.n_dof or center.numel() != F * self.n_dof or \
                lo.numel() != F * self.n_dof or hi.numel() != F * self.n_dof:
            raise ValueError("box_around: shape mismatch")
        _check(self.lib.ht_pso_box_around(self.handle, F, _ptr(center), _ptr(halfwidth), _ptr(lo),
                                          _ptr(hi), _stream()))

    def pso_run_graph(self, sw, params: PsoParams, n_generations: int):
        _check(self.lib.ht_pso_run_graph(self.handle, C.byref(sw["_struct"]), C.byref(params),
                                         n_generations, _stream()))

    # -- tracing ------------------------------------------------------------------------
    def profile_begin(self):
        _check(self.lib.ht_profile_begin(self.handle))

    def profile_end(self) -> dict:
        """Per kernel kind: launches, particles and summed device milliseconds."""
        stats = (KernelStat * len(KERNEL_KINDS))()
        _check(self.lib.ht_profile_end(self.handle, stats))
        return {k: {"launches": s.launches, "particles": s.particles, "ms": s.total_ms}
                for k, s in zip(KERNEL_KINDS, stats)}

    def eval_counts(self, reset: bool = False) -> tuple[int, int]:
        """(forward, gradient) particle evaluations performed so far (synchronises)."""
        f, g = C.c_int64(), C.c_int64()
        _check(self.lib.ht_eval_counts(self.handle, C.byref(f), C.byref(g), int(reset)))
        return f.value, g.value

    def device_errors(self, reset: bool = False) -> int:
        """HT_DEVERR_* flags the device raised in enqueued work so far (synchronises)."""
        v = C.c_uint32()
        _check(self.lib.ht_device_errors(self.handle, C.byref(v), int(reset)))
        return v.value

    # -- launch shape -------------------------------------------------------------------
    def launch_config(self):
        lc = LaunchConfig()
        _check(self.lib.ht_get_launch_config(self.handle, C.byref(lc)))
        return lc.tiles_per_item, lc.groups_per_cu, lc.cull

    def set_launch_config(self, tiles_per_item: int, groups_per_cu: int, cull: int = 1):
        lc = LaunchConfig(tiles_per_item, groups_per_cu, cull)
        _check(self.lib.ht_set_launch_config(self.handle, C.byref(lc)))

    def autotune(self, poses, frame_slots, repeats: int = 5):
        import torch
        F, P, D = poses.shape
        cost = torch.empty((F, P), device=poses.device, dtype=torch.float32)
        lc = LaunchConfig()
        _check(self.lib.ht_autotune(self.handle, F, _ptr(frame_slots), P, _ptr(poses.contiguous()),
                                    _ptr(cost), repeats, C.byref(lc), _stream()))
        return lc.tiles_per_item, lc.groups_per_cu, lc.cull


def header_functions(header_path: str | None = None) -> list[str]:
    """Names of the functions declared in include/handtrack.h."""
    import re
    if header_path is None:
        header_path = os.path.join(os.path.dirname(HERE), "include", "handtrack.h")
    text = open(header_path).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ht_[a-z_]+)\s*\(", text)))
