"""CPU oracle for Reinforcement Lightcuts Learning -- test infrastructure only.

Only the test suite, the smoke check and the benchmark's CPU-baseline leg use
this package.  The product library never imports, links or calls it, and it
shares no code with the GPU path: the C source ``rlc_oracle.c`` is a separate,
plain, single-threaded implementation of the method written from the paper
(section 3 and Eqs. 1-2), plus FP64 "truth" integrators for the quantity the
method estimates.

``build()`` compiles ``rlc_oracle.c`` with gcc (``-ffp-contract=off``, no fast
math) into ``liboracle.so`` next to it.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "rlc_oracle.c")
_SRC_MLP = os.path.join(_HERE, "rlc_oracle_mlp.c")
_SO = os.path.join(_HERE, "liboracle.so")
# a prebuilt oracle library to load instead (the sanitizer test builds one
# with AddressSanitizer and UBSan and runs the oracle's pins against it)
_SO_OVERRIDE = os.environ.get("RLC_ORACLE_LIB")
_lib = None

MMAX = 256
MIX_M = 64


FLAGS = ["-std=c11", "-Wall", "-ffp-contract=off", "-fno-fast-math", "-fexcess-precision=standard", "-fPIC",
         "-shared"]


def build(force: bool = True, out: str = _SO, extra=("-O2",)) -> str:
    """Compile the oracle library (always recompiles when force is true)."""
    if force or not os.path.exists(out):
        tmp = out + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", *extra, *FLAGS, "-o", tmp, _SRC, _SRC_MLP, "-lm"])
        os.replace(tmp, out)
    return out


def lib():
    global _lib
    if _lib is None:
        if _SO_OVERRIDE:
            _lib = ctypes.CDLL(_SO_OVERRIDE)
            _declare(_lib)
            return _lib
        if not os.path.exists(_SO) or os.path.getmtime(_SO) < max(os.path.getmtime(_SRC),
                                                                    os.path.getmtime(_SRC_MLP)):
            build()
        _lib = ctypes.CDLL(_SO)
        _declare(_lib)
    return _lib


class OrcConfig(ctypes.Structure):
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
        ("adapt", ctypes.c_uint32),
        ("temporal", ctypes.c_uint32),
        ("scene_id", ctypes.c_uint32),
        ("split_steps", ctypes.c_uint32),
        ("seed", ctypes.c_uint64),
        ("normal_bits", ctypes.c_uint32),
        ("jitter", ctypes.c_float),
        ("footprint_levels", ctypes.c_uint32),
        ("footprint_tile", ctypes.c_float),
    ]


class OrcRecords(ctypes.Structure):
    _fields_ = [(n, ctypes.c_void_p) for n in
                ("key", "ready", "slot", "light", "inv_pdf", "y", "contrib", "reward", "fnode",
                 "weight", "comp")]


_vp = ctypes.c_void_p
_u32 = ctypes.c_uint32


def _declare(L):
    L.orc_philox.argtypes = [_vp, _vp, _vp, _u32]
    L.orc_create.restype = _vp
    L.orc_create.argtypes = [ctypes.POINTER(OrcConfig), _vp, _vp, _u32, _vp, _u32]
    L.orc_destroy.argtypes = [_vp]
    L.orc_set_emission.argtypes = [_vp, _vp]
    L.orc_get_tree.argtypes = [_vp] + [_vp] * 7
    L.orc_get_template.restype = _u32
    L.orc_get_template.argtypes = [_vp, _vp, _vp]
    L.orc_cell_keys.argtypes = [_vp, _vp, _u32, _vp]
    L.orc_visible.argtypes = [_vp, _vp, _vp, _u32, _vp]
    L.orc_frame.argtypes = [_vp, _vp, _vp, _vp, _u32, _u32, _u32, _vp, ctypes.POINTER(OrcRecords)]
    L.orc_ema.argtypes = [_vp, _vp, _vp, _u32, ctypes.c_float, _u32, _vp]
    L.orc_split_collapse.argtypes = [_vp, _vp, _vp, _u32, ctypes.c_float]
    L.orc_cdf.argtypes = [_vp, _u32, ctypes.c_float, _vp, _vp]
    L.orc_adapt.argtypes = [_vp]
    L.orc_num_cells.restype = _u32
    L.orc_num_cells.argtypes = [_vp]
    L.orc_meff.restype = _u32
    L.orc_meff.argtypes = [_vp]
    L.orc_dump_cells.argtypes = [_vp] + [_vp] * 9
    L.orc_load_cell.argtypes = [_vp, _u32, _vp, _vp]
    L.orc_set_footprints.argtypes = [_vp, _vp, _u32]
    L.orc_point_levels.argtypes = [_vp, _u32, _vp]
    L.orc_status.restype = _u32
    L.orc_status.argtypes = [_vp]
    L.orc_truth_unoccluded.argtypes = [_vp, _vp, _vp, _u32, _vp]
    L.orc_truth_mc.argtypes = [_vp, _vp, _vp, _vp, _u32, _u32, _u32, _vp]
    L.orc_fixed_cut.restype = _u32
    L.orc_fixed_cut.argtypes = [_vp, _vp, _vp]
    L.orc_set_mixture.argtypes = [_vp, _vp, _u32, ctypes.c_float]
    L.orc_mlp_nparam.restype = _u32
    L.orc_bf16_round.argtypes = [_vp, _u32, _vp]
    L.orc_mlp_encode.argtypes = [_vp, _vp, _u32, _vp, _vp, _vp]
    L.orc_mlp_forward.argtypes = [_vp, _vp, _u32, ctypes.c_int, _vp, _vp]
    L.orc_mlp_loss_grad.argtypes = [_vp, _vp, _vp, _vp, _u32, ctypes.c_int, _vp, _vp]
    _d = ctypes.c_double
    L.orc_mlp_adam.argtypes = [_vp, _vp, _vp, _vp, _u32, _u32, _d, _d, _d, _d]
    L.orc_mlp_shuffle.argtypes = [_u32, _u32, _u32, ctypes.c_uint64, _vp]
    L.orc_mlp_train.argtypes = [_vp, _vp, _vp, _vp, _vp, _u32, _vp, _vp, _vp, _u32, _u32, _u32, _d, _d, _d,
                                _d, _u32, ctypes.c_uint64, ctypes.c_int, _vp]


def _p(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _c(a, dt):
    return np.ascontiguousarray(np.asarray(a, dtype=dt))


def philox(ctr, key) -> np.ndarray:
    """Philox4x32-10 of an (n, 4) counter array under a 2-word key."""
    ctr = _c(ctr, np.uint32).reshape(-1, 4)
    key = _c(key, np.uint32).reshape(2)
    out = np.zeros_like(ctr)
    lib().orc_philox(_p(ctr), _p(key), _p(out), ctr.shape[0])
    return out


def make_config(params: dict) -> OrcConfig:
    c = OrcConfig()
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
    c.adapt = int(params["adapt"])
    c.temporal = int(params["temporal"])
    c.scene_id = int(params["scene_id"])
    c.split_steps = int(params.get("split_steps", 1))
    c.seed = int(params["seed"])
    c.normal_bits = int(params.get("normal_bits", 0))
    c.jitter = float(params.get("jitter", 0.0))
    c.footprint_levels = int(params.get("footprint_levels", 0))
    c.footprint_tile = float(params.get("footprint_tile", 0.0))
    return c


class Oracle:
    """One scene's oracle state: reference tree, initial cut, cells."""

    def __init__(self, params: dict, tri, emit, boxes=None):
        L = lib()
        self.params = dict(params)
        self._tri = _c(tri, np.float32).reshape(-1, 9)
        self._emit = _c(emit, np.float32).reshape(-1, 3)
        self._boxes = _c(boxes if boxes is not None else np.zeros((0, 6)), np.float32).reshape(-1, 6)
        self.N = self._tri.shape[0]
        self.K = self._boxes.shape[0]
        self._cfg = make_config(params)
        h = L.orc_create(ctypes.byref(self._cfg), _p(self._tri), _p(self._emit), self.N,
                         _p(self._boxes) if self.K else None, self.K)
        if not h:
            raise ValueError("oracle: invalid scene or parameters")
        self._h = h

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            lib().orc_destroy(h)
            self._h = None

    # -- tree ---------------------------------------------------------------
    def tree(self) -> dict:
        N = self.N
        nn = 2 * N - 1
        out = dict(perm=np.zeros(N, np.uint32), left=np.zeros(max(N - 1, 0), np.uint32),
                   right=np.zeros(max(N - 1, 0), np.uint32), parent=np.zeros(nn, np.uint32),
                   first=np.zeros(nn, np.uint32), last=np.zeros(nn, np.uint32),
                   rec=np.zeros((N, 16), np.float32))
        lib().orc_get_tree(self._h, _p(out["perm"]), _p(out["left"]) if N > 1 else None,
                           _p(out["right"]) if N > 1 else None, _p(out["parent"]), _p(out["first"]),
                           _p(out["last"]), _p(out["rec"]))
        return out

    def template(self):
        node = np.zeros(MMAX, np.uint32)
        end = np.zeros(MMAX, np.uint32)
        m = lib().orc_get_template(self._h, _p(node), _p(end))
        return node[:m].copy(), end[:m].copy()

    def fixed_cut(self):
        """The fixed breadth-first cut (up to 64 nodes) of the learned proposal."""
        node = np.zeros(MIX_M, np.uint32)
        end = np.zeros(MIX_M, np.uint32)
        m = lib().orc_fixed_cut(self._h, _p(node), _p(end))
        return node[:m].copy(), end[:m].copy()

    def set_mixture(self, cdf=None, w: float = 0.5):
        """Turn the mixture with a learned per-point cdf on (rows of 64
        inclusive running sums, indexed by point id; w is the network's
        share, 0.5 the 50/50 mixture), or off with None or w = 0."""
        if cdf is None:
            lib().orc_set_mixture(self._h, None, 0, 0.0)
            self._mix = None
            return
        self._mix = _c(cdf, np.float32).reshape(-1, MIX_M)
        if lib().orc_set_mixture(self._h, _p(self._mix), self._mix.shape[0], float(w)) != 0:
            raise ValueError("bad mixture")

    def set_footprints(self, fp=None):
        """Footprint sides per point id (footprint-sized cells), or None for
        the finest level everywhere."""
        if fp is None:
            lib().orc_set_footprints(self._h, None, 0)
            self._fp = None
            return
        self._fp = _c(fp, np.float32).reshape(-1)
        if lib().orc_set_footprints(self._h, _p(self._fp), self._fp.size) != 0:
            raise ValueError("bad footprints")

    def point_levels(self, n: int) -> np.ndarray:
        out = np.zeros(n, np.uint32)
        lib().orc_point_levels(self._h, n, _p(out))
        return out

    @property
    def Meff(self) -> int:
        return int(lib().orc_meff(self._h))

    # -- per-frame ------------------------------------------------------------
    def set_emission(self, emit):
        e = _c(emit, np.float32).reshape(self.N, 3)
        lib().orc_set_emission(self._h, _p(e))

    def cell_keys(self, pos) -> np.ndarray:
        pos = _c(pos, np.float32).reshape(-1, 3)
        out = np.zeros(pos.shape[0], np.uint64)
        lib().orc_cell_keys(self._h, _p(pos), pos.shape[0], _p(out))
        return out

    def visible(self, x, y) -> np.ndarray:
        x = _c(x, np.float32).reshape(-1, 3)
        y = _c(y, np.float32).reshape(-1, 3)
        out = np.zeros(x.shape[0], np.uint8)
        lib().orc_visible(self._h, _p(x), _p(y), x.shape[0], _p(out))
        return out

    def frame(self, pos, nrm, spp: int, frame: int, pid=None, records: bool = False):
        """One pass (sample + shade + learn) over the given points; no adapt.

        Returns (radiance (P, 3), records dict or None)."""
        pos = _c(pos, np.float32).reshape(-1, 3)
        nrm = _c(nrm, np.float32).reshape(-1, 3)
        P = pos.shape[0]
        pid_a = None if pid is None else _c(pid, np.uint32).reshape(P)
        rad = np.zeros((P, 3), np.float32)
        rec = None
        recs = None
        if records:
            n = P * spp
            rec = dict(key=np.zeros(n, np.uint64), ready=np.zeros(n, np.uint32),
                       slot=np.zeros(n, np.uint32), light=np.zeros(n, np.uint32),
                       inv_pdf=np.zeros(n, np.float32), y=np.zeros((n, 3), np.float32),
                       contrib=np.zeros((n, 3), np.float32), reward=np.zeros(n, np.float32),
                       fnode=np.zeros(n, np.uint32), weight=np.zeros(n, np.float32),
                       comp=np.zeros(n, np.uint32))
            recs = OrcRecords(*[_p(rec[k]) for k in ("key", "ready", "slot", "light", "inv_pdf",
                                                     "y", "contrib", "reward", "fnode", "weight",
                                                     "comp")])
        lib().orc_frame(self._h, _p(pos), _p(nrm), _p(pid_a), P, int(spp), int(frame), _p(rad),
                        ctypes.byref(recs) if recs is not None else None)
        return rad, rec

    def adapt(self):
        lib().orc_adapt(self._h)

    def frame_sub(self, pos, nrm, spp: int, n_sub: int, frame: int, pid=None):
        """One frame as n_sub passes (section 3: a frame split into
        sub-frames, the cuts adapted after each pass): pass j has spp / n_sub
        samples per point and pass index frame * n_sub + j.  Returns the
        passes' radiance summed in pass order, times 1 / n_sub, in FP32."""
        assert n_sub >= 1 and spp % n_sub == 0
        acc = None
        for j in range(n_sub):
            rad, _ = self.frame(pos, nrm, spp // n_sub, frame * n_sub + j, pid=pid)
            self.adapt()
            acc = rad if acc is None else (acc + rad).astype(np.float32)
        if n_sub > 1:
            acc = (acc * np.float32(np.float32(1.0) / np.float32(n_sub))).astype(np.float32)
        return acc

    def run(self, pos, nrm, spp: int, frames: int, pid=None, first_frame: int = 0,
            emission_at=None):
        """frames passes of frame + adapt; returns the per-frame radiance list."""
        out = []
        for f in range(first_frame, first_frame + frames):
            if emission_at is not None:
                self.set_emission(emission_at(f))
            rad, _ = self.frame(pos, nrm, spp, f, pid=pid)
            self.adapt()
            out.append(rad)
        return out

    # -- inspection -----------------------------------------------------------
    def status(self) -> int:
        """Status bits raised since the previous call (1: a fixed-point
        reward sum wrapped 64 bits), then cleared."""
        return int(lib().orc_status(self._h))

    def num_cells(self) -> int:
        return int(lib().orc_num_cells(self._h))

    def cells(self) -> dict:
        n = self.num_cells()
        m = self.Meff
        d = dict(key=np.zeros(n, np.uint64), ready=np.zeros(n, np.uint32),
                 node=np.zeros((n, m), np.uint32), end=np.zeros((n, m), np.uint32),
                 Q=np.zeros((n, m), np.float32), Qt=np.zeros((n, m), np.float32),
                 C=np.zeros((n, m), np.float32), sum=np.zeros((n, m), np.uint64),
                 cnt=np.zeros((n, m), np.uint32))
        lib().orc_dump_cells(self._h, *[_p(d[k]) for k in ("key", "ready", "node", "end", "Q", "Qt",
                                                           "C", "sum", "cnt")])
        return d

    def load_cell(self, lin: int, node, Q):
        node = _c(node, np.uint32)
        Q = _c(Q, np.float32)
        assert node.size == self.Meff and Q.size == self.Meff
        if lib().orc_load_cell(self._h, int(lin), _p(node), _p(Q)) != 0:
            raise ValueError("bad cell index")

    def split_collapse(self, node, Q, T=None):
        node = _c(node, np.uint32).copy()
        Q = _c(Q, np.float32).copy()
        changed = lib().orc_split_collapse(self._h, _p(node), _p(Q), node.size,
                                           float(self.params["T"] if T is None else T))
        return bool(changed), node, Q

    # -- truth ---------------------------------------------------------------
    def truth_unoccluded(self, pos, nrm) -> np.ndarray:
        pos = _c(pos, np.float32).reshape(-1, 3)
        nrm = _c(nrm, np.float32).reshape(-1, 3)
        out = np.zeros((pos.shape[0], 3), np.float64)
        lib().orc_truth_unoccluded(self._h, _p(pos), _p(nrm), pos.shape[0], _p(out))
        return out

    def truth_mc(self, pos, nrm, ks: int = 16, replica: int = 0, pid=None) -> np.ndarray:
        pos = _c(pos, np.float32).reshape(-1, 3)
        nrm = _c(nrm, np.float32).reshape(-1, 3)
        P = pos.shape[0]
        pid_a = None if pid is None else _c(pid, np.uint32).reshape(P)
        out = np.zeros((P, 3), np.float64)
        lib().orc_truth_mc(self._h, _p(pos), _p(nrm), _p(pid_a), P, int(ks), int(replica), _p(out))
        return out


def ema(Q, sums, cnts, alpha: float, fx_shift: int) -> np.ndarray:
    Q = _c(Q, np.float32)
    s = _c(sums, np.uint64)
    n = _c(cnts, np.uint32)
    out = np.zeros_like(Q)
    lib().orc_ema(_p(Q), _p(s), _p(n), Q.size, float(alpha), int(fx_shift), _p(out))
    return out


def cdf(Q, eps: float):
    Q = _c(Q, np.float32)
    Qt = np.zeros_like(Q)
    C = np.zeros_like(Q)
    lib().orc_cdf(_p(Q), Q.size, float(eps), _p(Qt), _p(C))
    return Qt, C


# -- learned proposal (rlc_oracle_mlp.c) ---------------------------------------
MLP_IN, MLP_H, MLP_OUT = 144, 64, 64


def mlp_nparam() -> int:
    return int(lib().orc_mlp_nparam())


def bf16_round(a) -> np.ndarray:
    a = _c(a, np.float64)
    out = np.zeros_like(a)
    lib().orc_bf16_round(_p(a), a.size, _p(out))
    return out


def mlp_encode(pos, nrm, lo, hi) -> np.ndarray:
    pos = _c(pos, np.float32).reshape(-1, 3)
    nrm = _c(nrm, np.float32).reshape(-1, 3)
    lo = _c(lo, np.float32).reshape(3)
    hi = _c(hi, np.float32).reshape(3)
    out = np.zeros((pos.shape[0], MLP_IN), np.float64)
    lib().orc_mlp_encode(_p(pos), _p(nrm), pos.shape[0], _p(lo), _p(hi), _p(out))
    return out


def mlp_forward(params, x, bf16: bool = False):
    """(logits, probabilities), each (n, 64)."""
    params = _c(params, np.float64)
    x = _c(x, np.float64).reshape(-1, MLP_IN)
    n = x.shape[0]
    z = np.zeros((n, MLP_OUT))
    q = np.zeros((n, MLP_OUT))
    lib().orc_mlp_forward(_p(params), _p(x), n, int(bf16), _p(z), _p(q))
    return z, q


def mlp_loss_grad(params, x, node, w, bf16: bool = False):
    params = _c(params, np.float64)
    x = _c(x, np.float64).reshape(-1, MLP_IN)
    node = _c(node, np.uint32)
    w = _c(w, np.float64)
    loss = np.zeros(1)
    g = np.zeros(mlp_nparam())
    if lib().orc_mlp_loss_grad(_p(params), _p(x), _p(node), _p(w), x.shape[0], int(bf16), _p(loss),
                               _p(g)) != 0:
        raise ValueError("bad tuple")
    return float(loss[0]), g


def mlp_adam(params, m, v, grad, step: int, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam step in place on float64 arrays."""
    lib().orc_mlp_adam(_p(params), _p(m), _p(v), _p(_c(grad, np.float64)), params.size, int(step), lr, beta1,
                       beta2, eps)


def mlp_shuffle(n: int, epoch: int, scene_id: int, seed: int) -> np.ndarray:
    out = np.zeros(n, np.uint32)
    lib().orc_mlp_shuffle(n, epoch, scene_id, seed, _p(out))
    return out


def mlp_train(params, m, v, step: int, xall, pid, node, w, epochs: int, batch: int, lr=1e-3, beta1=0.9,
              beta2=0.999, eps=1e-8, scene_id: int = 0, seed: int = 0, bf16: bool = False):
    """Minibatch Adam training in place; returns (new step count, last batch loss)."""
    xall = _c(xall, np.float64).reshape(-1, MLP_IN)
    pid = _c(pid, np.uint32)
    node = _c(node, np.uint32)
    w = _c(w, np.float64)
    st = np.array([step], np.uint32)
    loss = np.zeros(1)
    rc = lib().orc_mlp_train(_p(params), _p(m), _p(v), _p(st), _p(xall), xall.shape[0], _p(pid), _p(node), _p(w),
                             pid.size, epochs, batch, lr, beta1, beta2, eps, scene_id, seed, int(bf16), _p(loss))
    if rc != 0:
        raise ValueError("bad training input")
    return int(st[0]), float(loss[0])


def mlp_cdf(probs) -> np.ndarray:
    """Inclusive running sums in FP32, left to right, of FP32-rounded
    probabilities: the per-point table the mixture draws from."""
    q = np.asarray(probs, np.float64).astype(np.float32)
    out = np.zeros_like(q)
    acc = np.zeros(q.shape[0], np.float32)
    for k in range(q.shape[1]):
        acc = (acc + q[:, k]).astype(np.float32)
        out[:, k] = acc
    return out
