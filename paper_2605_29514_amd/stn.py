"""ctypes binding of libstn (include/stn.h).  Argument marshalling only:
every step of the simulation runs in the library's HIP kernels; PyTorch
provides device memory and the stream.  There is no CPU fallback: importing
works anywhere, but creating a Simulator without the built library or
without a GPU raises.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libstn.so")

STN_FP64, STN_FP32 = 0, 1
PROFILE_TIMING_ONLY = 0x80000000          # include/stn.h STN_PROFILE_TIMING_ONLY
GATE_KIND = {"H": 0, "S": 1, "SDG": 2, "X": 3, "Y": 4, "Z": 5, "CX": 6, "CY": 7, "CZ": 8}
STATUS = {0: "STN_OK", -1: "STN_EINVAL", -2: "STN_ENOMEM", -3: "STN_EDEVICE",
          -4: "STN_EZEROPROB", -5: "STN_ENUMERIC", -6: "STN_ESTATE"}
DEFAULT_EPS = {STN_FP64: 1e-14, STN_FP32: 1e-12}


class STNError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class StnConfig(ctypes.Structure):
    _fields_ = [("n_qubits", ctypes.c_int), ("n_shots", ctypes.c_int), ("chi_max", ctypes.c_int),
                ("precision", ctypes.c_int), ("eps_cut", ctypes.c_double), ("stream", ctypes.c_void_p)]


class StnGate(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("q0", ctypes.c_int32), ("q1", ctypes.c_int32)]


_lib = None
EXPORTS = ["stn_workspace_bytes", "stn_init", "stn_free", "stn_last_error", "stn_clifford",
           "stn_rotate", "stn_measure", "stn_logprob", "stn_sync", "stn_get_tableau",
           "stn_get_bonds", "stn_get_site", "stn_center", "stn_profile", "stn_profile_read",
           "stn_set_site", "stn_set_center", "stn_set_layer_mode", "stn_set_layer_threads", "stn_reset",
           "stn_tape_bytes", "stn_tape_begin", "stn_tape_end", "stn_adjoint_bytes", "stn_adjoint_init",
           "stn_adjoint_zero", "stn_backward", "stn_checkpoint_bytes", "stn_checkpoint_save",
           "stn_checkpoint_load", "stn_profile_phases", "stn_adjoint_truncated", "stn_profile_paths",
           "stn_set_layer_lds", "stn_tape_begin_static", "stn_spectrum",
           "stn_set_layer_env"]
K_CLASSES = ["tableau", "build", "qr", "gemm", "gram", "eigen", "select", "expect", "layer"]


def load(path: str = LIB_PATH):
    """Load libstn.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    # torch first: its HIP runtime must be the one the library binds to, or
    # the device memory torch hands over is foreign to the library's runtime.
    import torch  # noqa: F401
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with python -m paper_2605_29514_amd.build")
    lib = ctypes.CDLL(path)
    vp, i32, i64, dbl = ctypes.c_void_p, ctypes.c_int, ctypes.c_int64, ctypes.c_double
    lib.stn_workspace_bytes.restype = ctypes.c_size_t
    lib.stn_workspace_bytes.argtypes = [ctypes.POINTER(StnConfig)]
    lib.stn_init.restype = i32
    lib.stn_init.argtypes = [ctypes.POINTER(vp), ctypes.POINTER(StnConfig), vp, ctypes.c_size_t]
    lib.stn_free.restype = None
    lib.stn_free.argtypes = [vp]
    lib.stn_last_error.restype = ctypes.c_char_p
    lib.stn_last_error.argtypes = [vp]
    lib.stn_clifford.restype = i32
    lib.stn_clifford.argtypes = [vp, ctypes.POINTER(StnGate), i32, vp]
    lib.stn_rotate.restype = i32
    lib.stn_rotate.argtypes = [vp, vp, i32, vp, i64]
    lib.stn_measure.restype = i32
    lib.stn_measure.argtypes = [vp, vp, i32, i32, vp, vp, vp, vp]
    lib.stn_logprob.restype = i32
    lib.stn_logprob.argtypes = [vp, vp, vp]
    lib.stn_sync.restype = i32
    lib.stn_sync.argtypes = [vp]
    lib.stn_get_tableau.restype = i32
    lib.stn_get_tableau.argtypes = [vp, vp, vp, vp]
    lib.stn_get_bonds.restype = i32
    lib.stn_get_bonds.argtypes = [vp, vp]
    lib.stn_get_site.restype = i32
    lib.stn_get_site.argtypes = [vp, i32, i32, vp, ctypes.c_size_t, ctypes.POINTER(i32),
                                 ctypes.POINTER(i32)]
    lib.stn_center.restype = i32
    lib.stn_center.argtypes = [vp]
    lib.stn_set_site.restype = i32
    lib.stn_set_site.argtypes = [vp, i32, i32, vp, i32, i32]
    lib.stn_set_center.restype = i32
    lib.stn_set_center.argtypes = [vp, i32]
    lib.stn_profile.restype = i32
    lib.stn_profile.argtypes = [vp, ctypes.c_uint]
    lib.stn_profile_read.restype = i32
    lib.stn_profile_read.argtypes = [vp, vp, vp, vp, vp, vp, vp]
    lib.stn_set_layer_mode.restype = i32
    lib.stn_set_layer_mode.argtypes = [vp, i32]
    lib.stn_set_layer_threads.restype = i32
    lib.stn_reset.restype = i32
    lib.stn_reset.argtypes = [vp]
    lib.stn_tape_bytes.restype = ctypes.c_size_t
    lib.stn_tape_bytes.argtypes = [vp, i32]
    lib.stn_tape_begin.restype = i32
    lib.stn_tape_begin.argtypes = [vp, vp, ctypes.c_size_t, i32]
    lib.stn_set_layer_env.restype = i32
    lib.stn_set_layer_env.argtypes = [vp, i32]
    lib.stn_spectrum.restype = i32
    lib.stn_spectrum.argtypes = [vp, i32, vp, i32, vp]
    lib.stn_tape_begin_static.restype = i32
    lib.stn_tape_begin_static.argtypes = [vp, i32]
    lib.stn_tape_end.restype = i32
    lib.stn_tape_end.argtypes = [vp, ctypes.POINTER(i32)]
    lib.stn_adjoint_bytes.restype = ctypes.c_size_t
    lib.stn_adjoint_bytes.argtypes = [vp, i32]
    lib.stn_adjoint_init.restype = i32
    lib.stn_adjoint_init.argtypes = [vp, vp, ctypes.c_size_t, i32]
    lib.stn_adjoint_zero.restype = i32
    lib.stn_adjoint_zero.argtypes = [vp]
    lib.stn_backward.restype = i32
    lib.stn_backward.argtypes = [vp, vp, i64]
    lib.stn_adjoint_truncated.restype = i32
    lib.stn_adjoint_truncated.argtypes = [vp, vp]
    lib.stn_profile_phases.restype = i32
    lib.stn_profile_phases.argtypes = [vp, vp]
    lib.stn_set_layer_lds.restype = i32
    lib.stn_set_layer_lds.argtypes = [vp, i32]
    lib.stn_profile_paths.restype = i32
    lib.stn_profile_paths.argtypes = [vp, vp]
    lib.stn_checkpoint_bytes.restype = ctypes.c_size_t
    lib.stn_checkpoint_bytes.argtypes = [vp]
    lib.stn_checkpoint_save.restype = i32
    lib.stn_checkpoint_save.argtypes = [vp, vp]
    lib.stn_checkpoint_load.restype = i32
    lib.stn_checkpoint_load.argtypes = [vp, vp]
    lib.stn_set_layer_threads.argtypes = [vp, i32]
    _lib = lib
    return lib


def pack_shots(mask: np.ndarray) -> np.ndarray:
    """bool [S, n] -> uint64 sign words [n, ceil(S/64)] (bit s%64 of word s//64)."""
    S, n = mask.shape
    SW = (S + 63) // 64
    pad = np.zeros((SW * 64, n), dtype=np.uint64)
    pad[:S] = mask
    b = pad.reshape(SW, 64, n) << np.arange(64, dtype=np.uint64)[None, :, None]
    return np.bitwise_or.reduce(b, axis=1).T.copy()


def unpack_shots(words: np.ndarray, S: int) -> np.ndarray:
    """uint64 [..., SW] -> bool [..., S]."""
    bits = (words[..., :, None] >> np.arange(64, dtype=np.uint64)) & np.uint64(1)
    return bits.reshape(*words.shape[:-1], -1)[..., :S].astype(bool)


def unpack_bits(words: np.ndarray, n: int) -> np.ndarray:
    return unpack_shots(words, n)


class Simulator:
    """One libstn context on a CUDA (HIP) device with a torch-owned workspace."""

    def __init__(self, n_qubits: int, n_shots: int, chi_max: int, precision: str = "fp32",
                 eps_cut: Optional[float] = None, device: str = "cuda:0", poison: bool = False,
                 layer_mode: int = 0, layer_threads: int = 0, stream=None, layer_lds: int = 0):
        """stream: torch.cuda.Stream every launch goes to (default: the
        current stream); a side stream is needed to capture HIP graphs."""
        import torch
        self.torch = torch
        if not torch.cuda.is_available():
            raise RuntimeError("libstn needs a GPU; no device is visible")
        self.lib = load()
        self.device = torch.device(device)
        self.prec = STN_FP64 if precision == "fp64" else STN_FP32
        self.n, self.S, self.chi = n_qubits, n_shots, chi_max
        self.eps_cut = DEFAULT_EPS[self.prec] if eps_cut is None else eps_cut
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.cfg = StnConfig(n_qubits, n_shots, chi_max, self.prec, self.eps_cut,
                             ctypes.c_void_p(self.stream.cuda_stream))
        nbytes = self.lib.stn_workspace_bytes(ctypes.byref(self.cfg))
        if nbytes == 0:
            raise STNError(-1, "invalid configuration")
        self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        if poison:              # testing aid: NaN bytes expose reads of unwritten workspace
            self.workspace.fill_(0xFF)
        base = self.workspace.data_ptr()
        aligned = (base + 255) & ~255
        self.ctx = ctypes.c_void_p()
        st = self.lib.stn_init(ctypes.byref(self.ctx), ctypes.byref(self.cfg),
                               ctypes.c_void_p(aligned), nbytes)
        if st != 0:
            raise STNError(st, "stn_init failed")
        self.W = (n_qubits + 63) // 64
        self.SW = (n_shots + 63) // 64
        if layer_mode:
            self.set_layer_mode(layer_mode)
        if layer_threads:
            self.set_layer_threads(layer_threads)
        if layer_lds:
            self.set_layer_lds(layer_lds)

    def __del__(self):
        ctx = getattr(self, "ctx", None)
        if ctx is not None and ctx.value and getattr(self, "lib", None) is not None:
            self.lib.stn_free(ctx)
            self.ctx = None

    # ------------------------------------------------------------ helpers
    def _check(self, st: int):
        if st != 0:
            raise STNError(st, self.lib.stn_last_error(self.ctx).decode())

    def _dev(self, arr, dtype):
        t = self.torch
        if isinstance(arr, t.Tensor):
            return arr.to(self.device, dtype).contiguous()
        return t.as_tensor(np.ascontiguousarray(arr), dtype=dtype, device=self.device)

    # ------------------------------------------------------------ the ABI
    def clifford(self, gates, noise=None):
        """gates: list of (name, q0, q1); noise: device int64 tensor [2, n, SW] or None."""
        arr = (StnGate * max(1, len(gates)))()
        for i, (name, q0, q1) in enumerate(gates):
            arr[i] = StnGate(GATE_KIND[name], int(q0), int(q1))
        ptr = None if noise is None else ctypes.c_void_p(noise.data_ptr())
        self._check(self.lib.stn_clifford(self.ctx, arr, len(gates), ptr))

    def rotate(self, qubits: np.ndarray, theta, stride: int):
        q = np.ascontiguousarray(qubits, dtype=np.int32)
        self._check(self.lib.stn_rotate(self.ctx, q.ctypes.data_as(ctypes.c_void_p), len(q),
                                        ctypes.c_void_p(theta.data_ptr()), int(stride)))

    def measure(self, qubits: np.ndarray, reset: bool, u=None, forced=None, out=None, prob=None):
        q = np.ascontiguousarray(qubits, dtype=np.int32)
        M = len(q)
        t = self.torch
        if out is None:
            out = t.empty((self.S, M), dtype=t.uint8, device=self.device)
        if prob is None:
            prob = t.empty((self.S, M), dtype=t.float64, device=self.device)
        up = None if u is None else ctypes.c_void_p(u.data_ptr())
        fp = None if forced is None else ctypes.c_void_p(forced.data_ptr())
        self._check(self.lib.stn_measure(self.ctx, q.ctypes.data_as(ctypes.c_void_p), M, int(bool(reset)),
                                         up, fp, ctypes.c_void_p(out.data_ptr()),
                                         ctypes.c_void_p(prob.data_ptr())))
        return out, prob

    def logprob(self):
        t = self.torch
        lp = t.empty(self.S, dtype=t.float64, device=self.device)
        te = t.empty(self.S, dtype=t.float64, device=self.device)
        self._check(self.lib.stn_logprob(self.ctx, ctypes.c_void_p(lp.data_ptr()),
                                         ctypes.c_void_p(te.data_ptr())))
        return lp, te

    def sync(self):
        self._check(self.lib.stn_sync(self.ctx))

    def reset(self):
        """Initial state for every shot, by kernel launches only (capturable)."""
        self._check(self.lib.stn_reset(self.ctx))

    # ------------------------------------------------------------ gradients
    def _aligned(self, nbytes):
        t = self.torch.empty(nbytes + 256, dtype=self.torch.uint8, device=self.device)
        return t, (t.data_ptr() + 255) & ~255

    def tape_begin(self, max_steps: int):
        nb = self.lib.stn_tape_bytes(self.ctx, int(max_steps))
        if nb == 0:
            raise STNError(-1, "invalid tape size")
        self._tape, ptr = self._aligned(nb)
        self._check(self.lib.stn_tape_begin(self.ctx, ctypes.c_void_p(ptr), nb, int(max_steps)))

    def tape_begin_static(self, max_steps: int):
        """Records into the library's static per-GPU tape (no allocation)."""
        self._check(self.lib.stn_tape_begin_static(self.ctx, int(max_steps)))

    def tape_end(self) -> int:
        nr = ctypes.c_int(0)
        self._check(self.lib.stn_tape_end(self.ctx, ctypes.byref(nr)))
        return nr.value

    def adjoint_init(self, chi_adj: int):
        nb = self.lib.stn_adjoint_bytes(self.ctx, int(chi_adj))
        if nb == 0:
            raise STNError(-1, "invalid adjoint bond cap")
        self._adj, ptr = self._aligned(nb)
        self._check(self.lib.stn_adjoint_init(self.ctx, ctypes.c_void_p(ptr), nb, int(chi_adj)))

    def adjoint_zero(self):
        self._check(self.lib.stn_adjoint_zero(self.ctx))

    def adjoint_truncated(self) -> np.ndarray:
        """Per shot: did the adjoint state's bond cap drop weight?"""
        out = np.zeros(self.S, np.int32)
        self._check(self.lib.stn_adjoint_truncated(self.ctx, out.ctypes.data_as(ctypes.c_void_p)))
        return out.astype(bool)

    def backward(self, grad, col: int = 0):
        """grad: float64 device tensor [S, R]; the tape's rotations go to
        columns col, col + 1, ..."""
        assert grad.dtype == self.torch.float64 and grad.is_contiguous() and grad.dim() == 2
        ptr = grad.data_ptr() + 8 * int(col)
        self._check(self.lib.stn_backward(self.ctx, ctypes.c_void_p(ptr), grad.shape[1]))

    def checkpoint_save(self):
        nb = self.lib.stn_checkpoint_bytes(self.ctx)
        buf, ptr = self._aligned(nb)
        self._check(self.lib.stn_checkpoint_save(self.ctx, ctypes.c_void_p(ptr)))
        return (buf, ptr)

    def checkpoint_load(self, ck):
        self._check(self.lib.stn_checkpoint_load(self.ctx, ctypes.c_void_p(ck[1])))

    def tableau(self):
        """(x [2n, n] bool, z [2n, n] bool, sign [2n, S] bool)."""
        n = self.n
        hx = np.zeros((2 * n, self.W), np.uint64)
        hz = np.zeros((2 * n, self.W), np.uint64)
        hs = np.zeros((2 * n, self.SW), np.uint64)
        self._check(self.lib.stn_get_tableau(self.ctx, hx.ctypes.data_as(ctypes.c_void_p),
                                             hz.ctypes.data_as(ctypes.c_void_p),
                                             hs.ctypes.data_as(ctypes.c_void_p)))
        return unpack_bits(hx, n), unpack_bits(hz, n), unpack_shots(hs, self.S)

    def bonds(self) -> np.ndarray:
        b = np.zeros((self.S, self.n + 1), np.int32)
        self._check(self.lib.stn_get_bonds(self.ctx, b.ctypes.data_as(ctypes.c_void_p)))
        return b

    def site(self, shot: int, j: int) -> np.ndarray:
        cap = self.chi * 2 * self.chi
        ctype = np.complex128 if self.prec == STN_FP64 else np.complex64
        buf = np.zeros(cap, ctype)
        dl, dr = ctypes.c_int32(), ctypes.c_int32()
        self._check(self.lib.stn_get_site(self.ctx, shot, j, buf.ctypes.data_as(ctypes.c_void_p),
                                          buf.nbytes, ctypes.byref(dl), ctypes.byref(dr)))
        return buf[: dl.value * 2 * dr.value].reshape(dl.value, 2, dr.value).astype(np.complex128)

    def mps(self, shot: int):
        return [self.site(shot, j) for j in range(self.n)]

    def set_site(self, shot: int, j: int, t: np.ndarray):
        ctype = np.complex128 if self.prec == STN_FP64 else np.complex64
        a = np.ascontiguousarray(t, dtype=ctype)
        self._check(self.lib.stn_set_site(self.ctx, shot, j, a.ctypes.data_as(ctypes.c_void_p),
                                          a.shape[0], a.shape[2]))

    def set_mps(self, shot: int, tensors, center: int):
        for j, t in enumerate(tensors):
            self.set_site(shot, j, t)
        self._check(self.lib.stn_set_center(self.ctx, center))

    def spectrum(self, bond: int):
        """Squared Schmidt values across the cut between sites bond-1 and bond
        of every shot, computed on the device: (values [S, ld] descending,
        normalised to sum 1, zero past the bond; bond dimensions [S])."""
        t = self.torch
        ld = max(1, min(self.chi, 1 << min(bond, self.n - bond, 30)))
        out = t.empty((self.S, ld), dtype=t.float64, device=self.device)
        rank = t.empty(self.S, dtype=t.int32, device=self.device)
        self._check(self.lib.stn_spectrum(self.ctx, int(bond), ctypes.c_void_p(out.data_ptr()), ld,
                                          ctypes.c_void_p(rank.data_ptr())))
        return out, rank

    def center(self) -> int:
        return self.lib.stn_center(self.ctx)

    def profile(self, classes=None, counters: bool = True):
        """Start profiling the named kernel classes (None: all; []: stop).
        counters=False records only the launch events (the device work
        counters slow the kernels they count)."""
        if classes is None:
            classes = K_CLASSES
        mask = 0
        for c in classes:
            mask |= 1 << K_CLASSES.index(c)
        if mask and not counters:
            mask |= PROFILE_TIMING_ONLY
        self._check(self.lib.stn_profile(self.ctx, mask))

    def profile_read(self) -> dict:
        K = len(K_CLASSES)
        ms, fl, by = np.zeros(K), np.zeros(K), np.zeros(K)
        ln = np.zeros(K, np.int64)
        sw = np.zeros(1)
        f64 = np.zeros(1)
        self._check(self.lib.stn_profile_read(self.ctx, *(a.ctypes.data_as(ctypes.c_void_p) for a in (ms, fl, by, ln, sw, f64))))
        out = {c: {"ms": float(ms[i]), "flops": float(fl[i]), "bytes": float(by[i]),
                   "launches": int(ln[i])} for i, c in enumerate(K_CLASSES)}
        out["eigen_sweeps"] = float(sw[0])
        out["layer_fp64_flops"] = float(f64[0])
        return out

    def profile_phases(self) -> dict:
        """Fused-kernel phase cycle totals (see stn_profile_phases)."""
        out = np.zeros(8, np.float64)
        self._check(self.lib.stn_profile_phases(self.ctx, out.ctypes.data_as(ctypes.c_void_p)))
        names = ["angles_single", "moves", "build", "lr_qr", "lr_absorb", "gram", "eigen", "select_trunc"]
        return dict(zip(names, out.tolist()))

    def profile_paths(self) -> dict:
        """Fused-kernel branch counters (see stn_profile_paths)."""
        out = np.zeros(11, np.float64)
        self._check(self.lib.stn_profile_paths(self.ctx, out.ctypes.data_as(ctypes.c_void_p)))
        names = ["env_steps", "qr_steps", "eig_lds", "eig_global", "eig_global_gt128", "max_order",
                 "chol_cycles", "jacobi_global", "cholqr", "eig_nominal_flops", "eig_exec_flops"]
        return dict(zip(names, out.tolist()))

    def set_layer_mode(self, mode: int):
        """0 automatic, 1 per-step kernels, 2 fused per-shot layer kernel."""
        self._check(self.lib.stn_set_layer_mode(self.ctx, int(mode)))

    def set_layer_lds(self, order: int):
        """Eigen-solve order kept in LDS by the fused kernel (0 auto, 32, 64)."""
        self._check(self.lib.stn_set_layer_lds(self.ctx, int(order)))

    def set_layer_env(self, max_bond: int):
        """Largest doubled bond of the environment-Gram sweep (0: QR sweep only)."""
        self._check(self.lib.stn_set_layer_env(self.ctx, int(max_bond)))

    def set_layer_threads(self, threads: int):
        """Threads per shot of the fused layer kernel (64, 128, 256 or 512)."""
        self._check(self.lib.stn_set_layer_threads(self.ctx, int(threads)))


# ----------------------------------------------------------------- circuits
def prepare(circ, device="cuda:0", forced: Optional[np.ndarray] = None, per_shot_theta: bool = False):
    """Uploads every per-shot input of a workload Circuit to the device once
    (noise sign words, angles, measurement uniforms or forced outcomes).
    forced: uint8 [S, n_measurements] or None.  Angles shared by all shots
    are uploaded once (stride 0) unless per_shot_theta."""
    import torch
    dev = torch.device(device)
    ops = []
    mi = 0
    for op in circ.ops:
        k = op["op"]
        if k == "gates":
            ops.append(("gates", [(g[0], g[1], g[2]) for g in op["gates"]]))
        elif k == "noise":
            words = np.stack([pack_shots(op["x"]), pack_shots(op["z"])])
            ops.append(("noise", torch.from_numpy(words.view(np.int64)).to(dev)))
        elif k == "rotate":
            th = np.ascontiguousarray(op["theta"], dtype=np.float64)
            shared = not per_shot_theta and bool(np.all(th == th[:1]))
            tdev = torch.from_numpy(th[0].copy() if shared else th).to(dev)
            ops.append(("rotate", np.ascontiguousarray(op["paulis"], np.int32), tdev,
                        0 if shared else th.shape[1]))
        elif k == "measure":
            M = len(op["qubits"])
            u = torch.from_numpy(np.ascontiguousarray(op["u"], np.float64)).to(dev)
            f = None
            if forced is not None:
                f = torch.from_numpy(np.ascontiguousarray(forced[:, mi:mi + M], np.uint8)).to(dev)
            ops.append(("measure", np.ascontiguousarray(op["qubits"], np.int32), bool(op["reset"]), u, f))
            mi += M
    return ops


def run_prepared(sim: Simulator, ops, start: int = 0, stop: Optional[int] = None, records=None):
    """Runs prepared ops [start, stop) on a Simulator; returns the list of
    (outcomes, prob) device tensors of the measurement ops run."""
    res = [] if records is None else records
    for op in ops[start:stop]:
        k = op[0]
        if k == "gates":
            sim.clifford(op[1])
        elif k == "noise":
            sim.clifford([], op[1])
        elif k == "rotate":
            sim.rotate(op[1], op[2], op[3])
        elif k == "measure":
            res.append(sim.measure(op[1], op[2], u=None if op[4] is not None else op[3], forced=op[4]))
    return res


def capture(sim: Simulator, ops):
    """Captures stn_reset followed by every prepared op into a HIP graph on
    the Simulator's (side) stream.  Returns (graph, results): each
    graph.replay() re-runs the whole circuit for the current contents of the
    ops' device inputs and rewrites the captured (outcomes, prob) tensors."""
    import torch
    if sim.stream == torch.cuda.current_stream(sim.device) and sim.stream.cuda_stream == 0:
        raise ValueError("graph capture needs a Simulator created on a side stream")
    sim.stream.wait_stream(torch.cuda.current_stream(sim.device))
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=sim.stream):
        sim.reset()
        res = run_prepared(sim, ops)
    return g, res


def load_inputs(dst_ops, src_ops):
    """Copies the per-shot device inputs of src_ops into the tensors of
    dst_ops (same circuit structure), e.g. a new batch of shots for a
    captured graph.  Host-side parts (gates, Pauli lists) must agree."""
    for a, b in zip(dst_ops, src_ops):
        if a[0] != b[0]:
            raise ValueError("op sequences differ")
        if a[0] == "noise":
            a[1].copy_(b[1])
        elif a[0] == "rotate":
            if not np.array_equal(a[1], b[1]) or a[3] != b[3]:
                raise ValueError("rotation Paulis differ")
            a[2].copy_(b[2])
        elif a[0] == "measure":
            a[3].copy_(b[3])
            if a[4] is not None:
                a[4].copy_(b[4])
        elif a[0] == "gates" and a[1] != b[1]:
            raise ValueError("gate lists differ")


def run_circuit(circ, chi_max: int, precision: str = "fp32", eps_cut: Optional[float] = None,
                device: str = "cuda:0", forced: Optional[np.ndarray] = None, sim: Optional[Simulator] = None,
                layer_mode: int = 0, layer_threads: int = 0, layer_lds: int = 0):
    """Simulates every shot of a workload Circuit on the GPU.  Returns a dict
    with records [S, M] uint8, prob [S, M], logp [S], trunc_err [S] (numpy)
    and the Simulator (for tableau / MPS inspection)."""
    if sim is None:
        sim = Simulator(circ.n, circ.n_shots, chi_max, precision, eps_cut, device, layer_mode=layer_mode,
                        layer_threads=layer_threads, layer_lds=layer_lds)
    ops = prepare(circ, device, forced)
    res = run_prepared(sim, ops)
    lp, te = sim.logprob()
    import torch
    rec = torch.cat([r[0] for r in res], dim=1).cpu().numpy() if res else np.zeros((circ.n_shots, 0), np.uint8)
    prob = torch.cat([r[1] for r in res], dim=1).cpu().numpy() if res else np.zeros((circ.n_shots, 0))
    return {"records": rec, "prob": prob, "logp": lp.cpu().numpy(), "trunc_err": te.cpu().numpy(),
            "sim": sim}


def run_waves(circ, chi_max: int, wave: int, precision: str = "fp32", eps_cut: Optional[float] = None,
              device: str = "cuda:0", stop_op: Optional[int] = None, layer_mode: int = 0,
              layer_threads: int = 0, layer_lds: int = 0, use_graph: bool = True, log=None):
    """Simulates the shots of a workload Circuit in waves of `wave` shots on
    one context (the device memory of a context grows with its shot count:
    at large chi_max the whole batch does not fit).  With use_graph, stn_reset
    and the circuit's ops [0, stop_op) are captured once as a HIP graph on a
    side stream and replayed for every wave with that wave's inputs loaded
    into the captured buffers; otherwise each wave runs eagerly after
    stn_reset.  The last wave is padded with copies of its last shot
    (results dropped).  Returns records [S, M], prob [S, M], logp [S],
    trunc_err [S] and max_bond [S] (numpy; M counts the measurements run)."""
    import torch
    S = circ.n_shots
    wave = max(1, min(int(wave), S))
    per_shot = any(o["op"] == "rotate" and not np.all(o["theta"] == o["theta"][:1]) for o in circ.ops)
    stream = torch.cuda.Stream(device=device) if use_graph else None
    sim = Simulator(circ.n, wave, chi_max, precision, eps_cut, device, layer_mode=layer_mode,
                    layer_threads=layer_threads, layer_lds=layer_lds, stream=stream)
    out = {"records": [], "prob": [], "logp": [], "trunc_err": [], "max_bond": []}
    graph, gres, gops = None, None, None
    for w0 in range(0, S, wave):
        take = np.minimum(np.arange(w0, w0 + wave), S - 1)
        cw = circ.shot_select(take)
        ops = prepare(cw, device, per_shot_theta=per_shot)[:stop_op]
        if use_graph:
            if graph is None:
                gops = ops
                graph, gres = capture(sim, gops)
            else:
                load_inputs(gops, ops)
            # the replay goes to the current stream: make that the library's
            # stream, ordered after the input copies of load_inputs
            sim.stream.wait_stream(torch.cuda.current_stream(sim.device))
            with torch.cuda.stream(sim.stream):
                graph.replay()
            res = gres
        else:
            sim.reset()
            res = run_prepared(sim, ops)
        lp, te = sim.logprob()
        torch.cuda.current_stream(sim.device).wait_stream(sim.stream)
        keep = min(wave, S - w0)
        if res:
            out["records"].append(torch.cat([r[0] for r in res], dim=1)[:keep].cpu().numpy())
            out["prob"].append(torch.cat([r[1] for r in res], dim=1)[:keep].cpu().numpy())
        out["logp"].append(lp[:keep].cpu().numpy())
        out["trunc_err"].append(te[:keep].cpu().numpy())
        out["max_bond"].append(sim.bonds()[:keep].max(axis=1))
        if log:
            log(f"wave of shots {w0}..{w0 + keep - 1} done")
    res = {k: (np.concatenate(v) if v else None) for k, v in out.items()}
    res["sim"] = sim
    return res
