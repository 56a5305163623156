"""Python binding of librlc (include/rlc.h): argument marshalling only.

Every function keeps the C name and takes torch tensors on the GPU (their
data_ptr() is passed as a device pointer) and the current torch stream.  All
computation happens in librlc's HIP kernels; there is no fallback: if the
library is not built, or no GPU is present, these calls raise.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "librlc.so")

RLC_OK = 0
RLC_EINVAL = -1
RLC_ENOMEM = -2
RLC_EHIP = -3
RLC_ECAPACITY = -4
RLC_ESTATE = -5
RLC_MMAX = 256

_ERRNAMES = {RLC_EINVAL: "RLC_EINVAL", RLC_ENOMEM: "RLC_ENOMEM", RLC_EHIP: "RLC_EHIP",
             RLC_ECAPACITY: "RLC_ECAPACITY", RLC_ESTATE: "RLC_ESTATE"}

# every entry point declared in include/rlc.h
EXPORTS = (
    "rlc_create", "rlc_destroy", "rlc_build_light_tree", "rlc_reset_cells", "rlc_set_emission",
    "rlc_set_occluders",
    "rlc_sample", "rlc_shade", "rlc_learn", "rlc_adapt_cuts", "rlc_frame", "rlc_frame_sub", "rlc_frame_sub_noalloc", "rlc_visible",
    "rlc_cell_keys", "rlc_image_error", "rlc_sync", "rlc_last_error", "rlc_num_cells", "rlc_meff",
    "rlc_dump_cells", "rlc_load_cells", "rlc_dump_tree", "rlc_get_light_order", "rlc_get_template",
    "rlc_set_timing", "rlc_get_timing",
    "rlc_batch_create", "rlc_batch_destroy", "rlc_batch_set_schedule", "rlc_batch_get_schedule",
    "rlc_batch_autotune", "rlc_batch_frame",
    "rlc_mlp_fixed_cut", "rlc_mlp_init", "rlc_mlp_set_params", "rlc_mlp_get_params", "rlc_mlp_copy_params",
    "rlc_mlp_forward",
    "rlc_mlp_grad", "rlc_mlp_train", "rlc_mlp_order", "rlc_set_mixture", "rlc_set_sample_log",
    "rlc_get_mlp_timing",
    "rlc_set_footprints",
)
RLC_MLP_PARAMS = 21760
RLC_MLP_NODES = 64


class RLCError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__("%s (%d): %s" % (_ERRNAMES.get(code, "RLC_ERROR"), code, msg))
        self.code = code


class rlc_config(ctypes.Structure):
    _fields_ = [
        ("M", ctypes.c_uint32),
        ("alpha", ctypes.c_float),
        ("T", ctypes.c_float),
        ("eps", ctypes.c_float),
        ("fx_shift", ctypes.c_uint32),
        ("reward_max", ctypes.c_float),
        ("t_lo", ctypes.c_float),
        ("reward_mode", ctypes.c_uint32),
        ("two_sided", ctypes.c_uint32),
        ("albedo", ctypes.c_float),
        ("grid_lo", ctypes.c_float * 3),
        ("grid_hi", ctypes.c_float * 3),
        ("grid_dims", ctypes.c_uint32 * 3),
        ("hashed", ctypes.c_uint32),
        ("capacity", ctypes.c_uint32),
        ("adapt", ctypes.c_uint32),
        ("temporal", ctypes.c_uint32),
        ("scene_id", ctypes.c_uint32),
        ("occ_grid_res", ctypes.c_uint32),
        ("split_steps", ctypes.c_uint32),
        ("seed", ctypes.c_uint64),
        ("normal_bits", ctypes.c_uint32),
        ("jitter", ctypes.c_float),
        ("footprint_levels", ctypes.c_uint32),
        ("footprint_tile", ctypes.c_float),
        ("max_cells", ctypes.c_uint32),
    ]


class rlc_samples(ctypes.Structure):
    _fields_ = [(n, ctypes.c_void_p) for n in
                ("d_key", "d_cell", "d_ready", "d_slot", "d_light", "d_inv_pdf", "d_y", "d_comp")]


class rlc_batch_scene(ctypes.Structure):
    _fields_ = [("ctx", ctypes.c_void_p), ("d_pos", ctypes.c_void_p), ("d_nrm", ctypes.c_void_p),
                ("d_radiance", ctypes.c_void_p), ("P", ctypes.c_uint32), ("spp", ctypes.c_uint32)]


class rlc_schedule(ctypes.Structure):
    _fields_ = [("tile", ctypes.c_uint32), ("blocks_per_cu", ctypes.c_uint32), ("dynamic", ctypes.c_uint32),
                ("cell_sorted", ctypes.c_uint32)]

    def as_dict(self):
        return {k: int(getattr(self, k)) for k, _ in self._fields_}


_vp = ctypes.c_void_p
_u32 = ctypes.c_uint32
_lib = None


def lib():
    """Load librlc.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("librlc.so is not built; run __graft_entry__.build() "
                              "(or python -m paper_1911_10217_amd.build)")
        L = ctypes.CDLL(LIB_PATH)
        _declare(L)
        _lib = L
    return _lib


def _declare(L):
    i = ctypes.c_int
    L.rlc_create.argtypes = [ctypes.POINTER(rlc_config), _vp, ctypes.POINTER(_vp)]
    L.rlc_destroy.argtypes = [_vp]
    L.rlc_build_light_tree.argtypes = [_vp, _vp, _vp, _u32]
    L.rlc_reset_cells.argtypes = [_vp]
    L.rlc_set_emission.argtypes = [_vp, _vp, _u32]
    L.rlc_set_occluders.argtypes = [_vp, _vp, _u32]
    L.rlc_sample.argtypes = [_vp, _vp, _vp, _u32, _u32, _u32, ctypes.POINTER(rlc_samples)]
    L.rlc_shade.argtypes = [_vp, _vp, _vp, _u32, _u32, ctypes.POINTER(rlc_samples), _vp, _vp, _vp]
    L.rlc_learn.argtypes = [_vp, ctypes.POINTER(rlc_samples), _vp, _u32]
    L.rlc_adapt_cuts.argtypes = [_vp]
    L.rlc_frame.argtypes = [_vp, _vp, _vp, _u32, _u32, _u32, _vp]
    L.rlc_frame_sub.argtypes = [_vp, _vp, _vp, _u32, _u32, _u32, _u32, _vp]
    L.rlc_frame_sub_noalloc.argtypes = [_vp, _vp, _vp, _u32, _u32, _u32, _u32, _vp]
    L.rlc_visible.argtypes = [_vp, _vp, _vp, _u32, _vp]
    L.rlc_cell_keys.argtypes = [_vp, _vp, _u32, _vp]
    L.rlc_image_error.argtypes = [_vp, _vp, _vp, _u32, _vp]
    L.rlc_sync.argtypes = [_vp]
    L.rlc_last_error.argtypes = [_vp]
    L.rlc_last_error.restype = ctypes.c_char_p
    L.rlc_num_cells.argtypes = [_vp, _vp]
    L.rlc_meff.argtypes = [_vp, _vp]
    L.rlc_dump_cells.argtypes = [_vp, _u32] + [_vp] * 9
    L.rlc_load_cells.argtypes = [_vp, _u32, _vp, _vp, _vp]
    L.rlc_dump_tree.argtypes = [_vp] + [_vp] * 7
    L.rlc_get_template.argtypes = [_vp, _vp, _vp, _vp]
    L.rlc_batch_create.argtypes = [ctypes.POINTER(rlc_batch_scene), _u32, _vp, ctypes.POINTER(_vp)]
    L.rlc_batch_destroy.argtypes = [_vp]
    L.rlc_batch_set_schedule.argtypes = [_vp, ctypes.POINTER(rlc_schedule)]
    L.rlc_batch_get_schedule.argtypes = [_vp, ctypes.POINTER(rlc_schedule)]
    L.rlc_batch_autotune.argtypes = [_vp, _u32, ctypes.POINTER(rlc_schedule), ctypes.POINTER(rlc_schedule),
                                     _vp, _vp]
    L.rlc_batch_frame.argtypes = [_vp, _u32]
    L.rlc_set_timing.argtypes = [_vp, i]
    L.rlc_get_timing.argtypes = [_vp, _vp, _vp, _vp]
    f = ctypes.c_float
    L.rlc_mlp_fixed_cut.argtypes = [_vp, _vp, _vp, _vp]
    L.rlc_mlp_init.argtypes = [_vp, ctypes.c_uint64]
    L.rlc_mlp_set_params.argtypes = [_vp, _vp]
    L.rlc_mlp_get_params.argtypes = [_vp, _vp]
    L.rlc_mlp_forward.argtypes = [_vp, _vp, _vp, _u32, _vp, _vp]
    L.rlc_mlp_grad.argtypes = [_vp, _vp, _vp, _u32, _vp, _vp, _vp, _u32, _vp, _vp]
    L.rlc_mlp_train.argtypes = [_vp, _vp, _vp, _u32, _vp, _vp, _vp, _u32, _u32, _u32, f, _vp]
    L.rlc_set_mixture.argtypes = [_vp, _vp, _u32, f]
    L.rlc_set_footprints.argtypes = [_vp, _vp, _u32]
    L.rlc_set_sample_log.argtypes = [_vp, _vp, _vp, _vp, ctypes.c_uint64]
    L.rlc_get_mlp_timing.argtypes = [_vp, _vp, _vp, _vp]
    L.rlc_mlp_order.argtypes = [_vp, _u32, _u32, _vp]
    L.rlc_get_light_order.argtypes = [_vp, _vp]
    L.rlc_mlp_copy_params.argtypes = [_vp, _vp]
    for name in EXPORTS:
        if name != "rlc_last_error":
            getattr(L, name).restype = i


def _ptr(t) -> Optional[int]:
    if t is None:
        return None
    if isinstance(t, np.ndarray):
        return t.ctypes.data
    return t.data_ptr()


def _dev(t, dtype, name):
    import torch
    if not isinstance(t, torch.Tensor) or t.device.type != "cuda":
        raise TypeError("%s must be a CUDA/HIP torch tensor" % name)
    if t.dtype != dtype:
        raise TypeError("%s must be %s, got %s" % (name, dtype, t.dtype))
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % name)
    return t


def _stream_handle():
    import torch
    return torch.cuda.current_stream().cuda_stream


def make_config(params: dict) -> rlc_config:
    c = rlc_config()
    c.M = int(params["M"])
    c.alpha = float(params["alpha"])
    c.T = float(params["T"])
    c.eps = float(params["eps"])
    c.fx_shift = int(params["fx_shift"])
    c.reward_max = float(params["reward_max"])
    c.t_lo = float(params["t_lo"])
    c.reward_mode = int(params["reward_mode"])
    c.two_sided = int(params["two_sided"])
    c.albedo = float(params["albedo"])
    for a in range(3):
        c.grid_lo[a] = float(params["grid_lo"][a])
        c.grid_hi[a] = float(params["grid_hi"][a])
        c.grid_dims[a] = int(params["grid_dims"][a])
    c.hashed = int(params.get("hashed", 0))
    c.capacity = int(params.get("capacity", 0))
    c.adapt = int(params["adapt"])
    c.temporal = int(params["temporal"])
    c.scene_id = int(params["scene_id"])
    c.occ_grid_res = int(params.get("occ_grid_res", 0))
    c.split_steps = int(params.get("split_steps", 1))
    c.seed = int(params["seed"])
    c.normal_bits = int(params.get("normal_bits", 0))
    c.jitter = float(params.get("jitter", 0.0))
    c.footprint_levels = int(params.get("footprint_levels", 0))
    c.footprint_tile = float(params.get("footprint_tile", 0.0))
    c.max_cells = int(params.get("max_cells", 0))
    return c


class Context:
    """An rlc_ctx bound to the torch stream current at creation."""

    def __init__(self, params: dict, stream=None):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("librlc needs a GPU (torch.cuda.is_available() is False)")
        L = lib()
        self.params = dict(params)
        self._cfg = make_config(params)
        self._stream = stream if stream is not None else _stream_handle()
        h = _vp()
        rc = L.rlc_create(ctypes.byref(self._cfg), _vp(self._stream), ctypes.byref(h))
        if rc != RLC_OK:
            raise RLCError(rc, "rlc_create rejected the configuration")
        self._h = h
        self.N = 0

    # -- helpers ---------------------------------------------------------------
    def _check(self, rc: int, what: str):
        if rc != RLC_OK:
            msg = lib().rlc_last_error(self._h)
            raise RLCError(rc, "%s: %s" % (what, msg.decode() if msg else ""))

    def close(self):
        """rlc_destroy; refused (RLCError, the context stays usable) while a
        batch refers to the context."""
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            self._check(lib().rlc_destroy(h), "rlc_destroy")
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- the method's calls --------------------------------------------------------
    def rlc_build_light_tree(self, tri, emit):
        import torch
        _dev(tri, torch.float32, "tri")
        _dev(emit, torch.float32, "emit")
        N = tri.numel() // 9
        if tri.numel() != 9 * N or emit.numel() != 3 * N:
            raise ValueError("tri must be N x 9 and emit N x 3")
        self._check(lib().rlc_build_light_tree(self._h, _ptr(tri), _ptr(emit), N), "rlc_build_light_tree")
        self.N = N

    def rlc_reset_cells(self):
        self._check(lib().rlc_reset_cells(self._h), "rlc_reset_cells")

    def rlc_set_emission(self, emit):
        import torch
        _dev(emit, torch.float32, "emit")
        self._check(lib().rlc_set_emission(self._h, _ptr(emit), emit.numel() // 3), "rlc_set_emission")

    def rlc_set_occluders(self, boxes):
        import torch
        K = 0 if boxes is None else boxes.numel() // 6
        if K:
            _dev(boxes, torch.float32, "boxes")
        self._check(lib().rlc_set_occluders(self._h, _ptr(boxes) if K else None, K), "rlc_set_occluders")

    def new_samples(self, n: int) -> dict:
        import torch
        dev = torch.device("cuda")
        return dict(key=torch.empty(n, dtype=torch.int64, device=dev),
                    cell=torch.empty(n, dtype=torch.int32, device=dev),
                    ready=torch.empty(n, dtype=torch.int32, device=dev),
                    slot=torch.empty(n, dtype=torch.int32, device=dev),
                    light=torch.empty(n, dtype=torch.int32, device=dev),
                    inv_pdf=torch.empty(n, dtype=torch.float32, device=dev),
                    y=torch.empty((n, 3), dtype=torch.float32, device=dev),
                    comp=torch.empty(n, dtype=torch.int32, device=dev))

    @staticmethod
    def _samples_struct(s: dict) -> rlc_samples:
        return rlc_samples(*[_ptr(s.get(k)) for k in ("key", "cell", "ready", "slot", "light", "inv_pdf", "y",
                                                      "comp")])

    def rlc_sample(self, pos, nrm, spp: int, frame: int, out: Optional[dict] = None) -> dict:
        import torch
        _dev(pos, torch.float32, "pos")
        P = pos.numel() // 3
        out = out if out is not None else self.new_samples(P * spp)
        st = self._samples_struct(out)
        self._check(lib().rlc_sample(self._h, _ptr(pos), _ptr(nrm), P, spp, frame, ctypes.byref(st)), "rlc_sample")
        return out

    def rlc_shade(self, pos, nrm, spp: int, samples: dict, radiance=None, contrib: bool = True):
        import torch
        _dev(pos, torch.float32, "pos")
        _dev(nrm, torch.float32, "nrm")
        P = pos.numel() // 3
        n = P * spp
        radiance = radiance if radiance is not None else torch.empty((P, 3), dtype=torch.float32, device="cuda")
        c = torch.empty((n, 3), dtype=torch.float32, device="cuda") if contrib else None
        reward = torch.empty(n, dtype=torch.float32, device="cuda")
        st = self._samples_struct(samples)
        self._check(lib().rlc_shade(self._h, _ptr(pos), _ptr(nrm), P, spp, ctypes.byref(st), _ptr(radiance),
                                    _ptr(c), _ptr(reward)), "rlc_shade")
        return radiance, c, reward

    def rlc_learn(self, samples: dict, reward):
        st = self._samples_struct(samples)
        self._check(lib().rlc_learn(self._h, ctypes.byref(st), _ptr(reward), reward.numel()), "rlc_learn")

    def rlc_adapt_cuts(self):
        self._check(lib().rlc_adapt_cuts(self._h), "rlc_adapt_cuts")

    def rlc_frame(self, pos, nrm, spp: int, frame: int, radiance=None):
        import torch
        _dev(pos, torch.float32, "pos")
        _dev(nrm, torch.float32, "nrm")
        P = pos.numel() // 3
        radiance = radiance if radiance is not None else torch.empty((P, 3), dtype=torch.float32, device="cuda")
        _dev(radiance, torch.float32, "radiance")
        self._check(lib().rlc_frame(self._h, _ptr(pos), _ptr(nrm), P, spp, frame, _ptr(radiance)), "rlc_frame")
        return radiance

    def rlc_frame_sub(self, pos, nrm, spp: int, n_sub: int, frame: int, radiance=None):
        import torch
        _dev(pos, torch.float32, "pos")
        _dev(nrm, torch.float32, "nrm")
        P = pos.numel() // 3
        radiance = radiance if radiance is not None else torch.empty((P, 3), dtype=torch.float32, device="cuda")
        _dev(radiance, torch.float32, "radiance")
        self._check(lib().rlc_frame_sub(self._h, _ptr(pos), _ptr(nrm), P, spp, n_sub, frame, _ptr(radiance)),
                    "rlc_frame_sub")
        return radiance

    def rlc_frame_sub_noalloc(self, pos, nrm, spp: int, n_sub: int, frame: int, radiance):
        """rlc_frame_sub through the entry point that allocates nothing; the
        caller passes the radiance tensor (P x 3)."""
        import torch
        _dev(pos, torch.float32, "pos")
        _dev(nrm, torch.float32, "nrm")
        _dev(radiance, torch.float32, "radiance")
        P = pos.numel() // 3
        self._check(lib().rlc_frame_sub_noalloc(self._h, _ptr(pos), _ptr(nrm), P, spp, n_sub, frame,
                                                _ptr(radiance)), "rlc_frame_sub_noalloc")
        return radiance

    def rlc_visible(self, x, y):
        import torch
        _dev(x, torch.float32, "x")
        _dev(y, torch.float32, "y")
        n = x.numel() // 3
        vis = torch.empty(n, dtype=torch.uint8, device="cuda")
        self._check(lib().rlc_visible(self._h, _ptr(x), _ptr(y), n, _ptr(vis)), "rlc_visible")
        return vis

    def rlc_cell_keys(self, pos):
        import torch
        _dev(pos, torch.float32, "pos")
        n = pos.numel() // 3
        keys = torch.empty(n, dtype=torch.int64, device="cuda")
        self._check(lib().rlc_cell_keys(self._h, _ptr(pos), n, _ptr(keys)), "rlc_cell_keys")
        return keys

    def rlc_image_error(self, img, ref) -> np.ndarray:
        out = np.zeros(5, np.float64)
        self._check(lib().rlc_image_error(self._h, _ptr(img), _ptr(ref), img.numel(), out.ctypes.data), "rlc_image_error")
        return out

    def rlc_sync(self):
        self._check(lib().rlc_sync(self._h), "rlc_sync")

    def rlc_num_cells(self) -> int:
        n = np.zeros(1, np.uint32)
        self._check(lib().rlc_num_cells(self._h, n.ctypes.data), "rlc_num_cells")
        return int(n[0])

    def rlc_meff(self) -> int:
        n = np.zeros(1, np.uint32)
        self._check(lib().rlc_meff(self._h, n.ctypes.data), "rlc_meff")
        return int(n[0])

    def rlc_dump_cells(self) -> dict:
        n = self.rlc_num_cells()
        m = self.rlc_meff()
        d = dict(key=np.zeros(n, np.uint64), ready=np.zeros(n, np.uint32),
                 node=np.zeros((n, m), np.uint32), end=np.zeros((n, m), np.uint32),
                 Q=np.zeros((n, m), np.float32), Qt=np.zeros((n, m), np.float32),
                 C=np.zeros((n, m), np.float32), sum=np.zeros((n, m), np.uint64),
                 cnt=np.zeros((n, m), np.uint32))
        if n:
            self._check(lib().rlc_dump_cells(self._h, n, *[d[k].ctypes.data for k in
                                                          ("key", "ready", "node", "end", "Q", "Qt", "C", "sum", "cnt")]),
                        "rlc_dump_cells")
        return d

    def rlc_load_cells(self, keys, node, Q):
        """Checkpoint load: keys (n,), node and Q (n, Meff), host arrays, as
        rlc_dump_cells gives them for ready cells."""
        keys = np.ascontiguousarray(keys, np.uint64).reshape(-1)
        n = keys.size
        m = self.rlc_meff()
        node = np.ascontiguousarray(node, np.uint32).reshape(n, m)
        Q = np.ascontiguousarray(Q, np.float32).reshape(n, m)
        self._check(lib().rlc_load_cells(self._h, n, keys.ctypes.data, node.ctypes.data, Q.ctypes.data),
                    "rlc_load_cells")

    def rlc_dump_tree(self) -> dict:
        N = self.N
        nn = 2 * N - 1
        d = dict(perm=np.zeros(N, np.uint32), left=np.zeros(max(N - 1, 1), np.uint32),
                 right=np.zeros(max(N - 1, 1), np.uint32), parent=np.zeros(nn, np.uint32),
                 first=np.zeros(nn, np.uint32), last=np.zeros(nn, np.uint32),
                 rec=np.zeros((N, 16), np.float32))
        self._check(lib().rlc_dump_tree(self._h, *[d[k].ctypes.data for k in
                                                   ("perm", "left", "right", "parent", "first", "last", "rec")]),
                    "rlc_dump_tree")
        d["left"] = d["left"][:N - 1]
        d["right"] = d["right"][:N - 1]
        return d

    def rlc_get_light_order(self, out=None):
        """Input index of the light at each tree position (device int32 tensor of N)."""
        import torch
        if out is None:
            out = torch.empty(self.N, dtype=torch.int32, device="cuda")
        self._check(lib().rlc_get_light_order(self._h, _ptr(out)), "rlc_get_light_order")
        return out

    def rlc_get_template(self):
        node = np.zeros(RLC_MMAX, np.uint32)
        end = np.zeros(RLC_MMAX, np.uint32)
        m = np.zeros(1, np.uint32)
        self._check(lib().rlc_get_template(self._h, node.ctypes.data, end.ctypes.data, m.ctypes.data),
                    "rlc_get_template")
        return node[:m[0]].copy(), end[:m[0]].copy()

    def rlc_set_timing(self, enable: bool):
        self._check(lib().rlc_set_timing(self._h, 1 if enable else 0), "rlc_set_timing")

    def rlc_get_timing(self):
        f = np.zeros(1, np.float64)
        a = np.zeros(1, np.float64)
        n = np.zeros(1, np.uint32)
        self._check(lib().rlc_get_timing(self._h, f.ctypes.data, a.ctypes.data, n.ctypes.data), "rlc_get_timing")
        return float(f[0]), float(a[0]), int(n[0])

    def rlc_get_mlp_timing(self):
        f = np.zeros(1, np.float64)
        u = np.zeros(1, np.float64)
        n = np.zeros(1, np.uint32)
        self._check(lib().rlc_get_mlp_timing(self._h, f.ctypes.data, u.ctypes.data, n.ctypes.data),
                    "rlc_get_mlp_timing")
        return float(f[0]), float(u[0]), int(n[0])

    # -- learned proposal ------------------------------------------------------------
    def rlc_mlp_order(self, n: int, epoch: int, out=None):
        """Tuple order of a training epoch (device uint32 tensor of n)."""
        import torch
        if out is None:
            out = torch.empty(n, dtype=torch.int32, device="cuda")
        self._check(lib().rlc_mlp_order(self._h, n, epoch, _ptr(out)), "rlc_mlp_order")
        return out

    def rlc_mlp_fixed_cut(self):
        node = np.zeros(RLC_MLP_NODES, np.uint32)
        end = np.zeros(RLC_MLP_NODES, np.uint32)
        m = np.zeros(1, np.uint32)
        self._check(lib().rlc_mlp_fixed_cut(self._h, node.ctypes.data, end.ctypes.data, m.ctypes.data),
                    "rlc_mlp_fixed_cut")
        return node[:m[0]].copy(), end[:m[0]].copy()

    def rlc_mlp_init(self, seed: int):
        self._check(lib().rlc_mlp_init(self._h, int(seed)), "rlc_mlp_init")

    def rlc_mlp_set_params(self, params):
        import torch
        _dev(params, torch.float32, "params")
        if params.numel() != RLC_MLP_PARAMS:
            raise ValueError("params must hold %d floats" % RLC_MLP_PARAMS)
        self._check(lib().rlc_mlp_set_params(self._h, _ptr(params)), "rlc_mlp_set_params")

    def rlc_mlp_get_params(self):
        import torch
        out = torch.empty(RLC_MLP_PARAMS, dtype=torch.float32, device="cuda")
        self._check(lib().rlc_mlp_get_params(self._h, _ptr(out)), "rlc_mlp_get_params")
        return out

    def rlc_mlp_copy_params(self, src: "Context"):
        """Take src's network weights on this context's stream, after the work
        enqueued so far on src's stream (no host synchronisation)."""
        self._check(lib().rlc_mlp_copy_params(self._h, src._h), "rlc_mlp_copy_params")

    def rlc_mlp_forward(self, pos, nrm, cdf=True, logits=False):
        """cdf / logits: True to allocate the output, a (P, 64) float32 tensor
        to write into, or False/None for none."""
        import torch
        _dev(pos, torch.float32, "pos")
        _dev(nrm, torch.float32, "nrm")
        P = pos.numel() // 3

        def out(spec, name):
            if spec is True:
                return torch.empty((P, RLC_MLP_NODES), dtype=torch.float32, device="cuda")
            if spec is None or spec is False:
                return None
            _dev(spec, torch.float32, name)
            if spec.numel() != P * RLC_MLP_NODES:
                raise ValueError("%s must be P x 64" % name)
            return spec
        c = out(cdf, "cdf")
        z = out(logits, "logits")
        self._check(lib().rlc_mlp_forward(self._h, _ptr(pos), _ptr(nrm), P, _ptr(c), _ptr(z)), "rlc_mlp_forward")
        return c, z

    @staticmethod
    def _tuples(pid, node, w):
        import torch
        _dev(pid, torch.int32, "pid")
        _dev(node, torch.int32, "node")
        _dev(w, torch.float32, "w")
        n = pid.numel()
        if node.numel() != n or w.numel() != n:
            raise ValueError("pid, node and w must have the same length")
        return n

    def rlc_mlp_grad(self, pos, nrm, pid, node, w):
        import torch
        n = self._tuples(pid, node, w)
        g = torch.empty(RLC_MLP_PARAMS, dtype=torch.float32, device="cuda")
        loss = np.zeros(1, np.float32)
        self._check(lib().rlc_mlp_grad(self._h, _ptr(pos), _ptr(nrm), pos.numel() // 3, _ptr(pid), _ptr(node),
                                       _ptr(w), n, _ptr(g), loss.ctypes.data), "rlc_mlp_grad")
        return float(loss[0]), g

    def rlc_mlp_train(self, pos, nrm, pid, node, w, epochs: int, batch: int, lr: float, sync: bool = True):
        """Returns the last batch's loss; with sync=False only enqueues and returns None."""
        n = self._tuples(pid, node, w)
        loss = np.zeros(1, np.float32)
        self._check(lib().rlc_mlp_train(self._h, _ptr(pos), _ptr(nrm), pos.numel() // 3, _ptr(pid), _ptr(node),
                                        _ptr(w), n, int(epochs), int(batch), float(lr),
                                        loss.ctypes.data if sync else None), "rlc_mlp_train")
        return float(loss[0]) if sync else None

    def rlc_set_mixture(self, cdf=None, w: float = 0.5):
        import torch
        if cdf is None:
            self._mix_keep = None
            self._check(lib().rlc_set_mixture(self._h, None, 0, 0.0), "rlc_set_mixture")
            return
        _dev(cdf, torch.float32, "cdf")
        rows = cdf.numel() // RLC_MLP_NODES
        self._mix_keep = cdf
        self._check(lib().rlc_set_mixture(self._h, _ptr(cdf), rows, float(w)), "rlc_set_mixture")

    def rlc_set_footprints(self, fp=None):
        """Per-point footprint sides (a float32 device tensor, one per point)
        for footprint-sized cells, or None for the finest level everywhere."""
        import torch
        if fp is None:
            self._fp_keep = None
            self._check(lib().rlc_set_footprints(self._h, None, 0), "rlc_set_footprints")
            return
        _dev(fp, torch.float32, "footprints")
        self._check(lib().rlc_set_footprints(self._h, _ptr(fp), fp.numel()), "rlc_set_footprints")
        self._fp_keep = fp

    def rlc_set_sample_log(self, pid=None, node=None, w=None):
        import torch
        if pid is None:
            self._log_keep = None
            self._check(lib().rlc_set_sample_log(self._h, None, None, None, 0), "rlc_set_sample_log")
            return
        n = self._tuples(pid, node, w)
        self._log_keep = (pid, node, w)
        self._check(lib().rlc_set_sample_log(self._h, _ptr(pid), _ptr(node), _ptr(w), n), "rlc_set_sample_log")



class Batch:
    """rlc_batch: one pass of several scenes per graph launch.

    scenes: list of (Context, pos, nrm, spp); radiance tensors are allocated
    here and returned by rlc_batch_frame.  All contexts must have been created
    on `stream` (a torch.cuda.Stream, not the default stream)."""

    def __init__(self, scenes, stream):
        import torch
        L = lib()
        self._keep = []
        self.radiance = []
        arr = (rlc_batch_scene * len(scenes))()
        for i, (ctx, pos, nrm, spp) in enumerate(scenes):
            _dev(pos, torch.float32, "pos")
            _dev(nrm, torch.float32, "nrm")
            P = pos.numel() // 3
            rad = torch.zeros((P, 3), dtype=torch.float32, device=pos.device)
            self.radiance.append(rad)
            self._keep += [ctx, pos, nrm, rad]
            arr[i] = rlc_batch_scene(ctx._h.value, _ptr(pos), _ptr(nrm), _ptr(rad), P, int(spp))
        self._ctx0 = scenes[0][0]
        h = _vp()
        rc = L.rlc_batch_create(arr, len(scenes), _vp(stream.cuda_stream), ctypes.byref(h))
        if rc != RLC_OK:
            msg = L.rlc_last_error(self._ctx0._h)
            raise RLCError(rc, "rlc_batch_create: %s" % (msg.decode() if msg else ""))
        self._h = h

    def _check(self, rc, what):
        if rc != RLC_OK:
            msg = lib().rlc_last_error(self._ctx0._h)
            raise RLCError(rc, "%s: %s" % (what, msg.decode() if msg else ""))

    def close(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            lib().rlc_batch_destroy(h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def rlc_batch_frame(self, frame: int):
        self._check(lib().rlc_batch_frame(self._h, int(frame)), "rlc_batch_frame")
        return self.radiance

    def rlc_batch_set_schedule(self, tile=512, blocks_per_cu=8, dynamic=1, cell_sorted=0):
        sc = rlc_schedule(tile, blocks_per_cu, dynamic, cell_sorted)
        self._check(lib().rlc_batch_set_schedule(self._h, ctypes.byref(sc)), "rlc_batch_set_schedule")

    def rlc_batch_get_schedule(self) -> dict:
        sc = rlc_schedule()
        self._check(lib().rlc_batch_get_schedule(self._h, ctypes.byref(sc)), "rlc_batch_get_schedule")
        return sc.as_dict()

    def rlc_batch_autotune(self, passes: int = 2):
        best = rlc_schedule()
        cap = 64
        cands = (rlc_schedule * cap)()
        ms = np.zeros(cap, np.float64)
        n = np.array([cap], np.uint32)
        self._check(lib().rlc_batch_autotune(self._h, int(passes), ctypes.byref(best), cands, ms.ctypes.data,
                                             n.ctypes.data), "rlc_batch_autotune")
        k = int(n[0])
        return best.as_dict(), [(cands[i].as_dict(), float(ms[i])) for i in range(min(k, cap))]
