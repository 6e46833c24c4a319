"""Python face of the TTN trajectory engine.

A thin wrapper over the C ABI of include/ttn.h: PyTorch supplies device
memory and the HIP stream, every step of the simulation runs in the
library's HIP kernels.  There is no CPU path: constructing an engine without
the built library or without a GPU raises.
"""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass

import numpy as np
import torch

from . import _abi
from ._abi import check, lib

OP_COLS = 9


def _ptr(t) -> int | None:
    return None if t is None else int(t.data_ptr())


@dataclass
class RunResult:
    records: torch.Tensor     # [rows, n_rec] uint8
    branches: torch.Tensor    # [rows, n_ad] int8
    logp: torch.Tensor        # [rows] float64
    stats: dict


class OpList:
    """An op list uploaded to a context (see ttn_oplist_upload)."""

    def __init__(self, engine: "TTNEngine", ops: np.ndarray, n_loc: int, n_rec: int, n_draws: int):
        ops = np.ascontiguousarray(np.asarray(ops, dtype=np.int32).reshape(-1, OP_COLS))
        self.engine = engine
        self.n_ops = int(ops.shape[0])
        self.n_loc, self.n_rec, self.n_draws = int(n_loc), int(n_rec), int(n_draws)
        self.n_ad = int((ops[:, 0] == 3).sum())
        h = C.c_void_p()
        check(lib().ttn_oplist_upload(engine._ctx, ops.ctypes.data, self.n_ops, self.n_loc,
                                      self.n_rec, self.n_draws, C.byref(h)), engine._ctx)
        self._h = h

    def free(self):
        if self._h:
            lib().ttn_oplist_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


class TTNEngine:
    """B trajectories of an N-qubit binary tree tensor network on one GPU."""

    def __init__(self, n_qubits: int, batch: int, leaf_of_qubit=None, chi_max: int = 64,
                 cutoff: float = 1e-10, dtype: str = "c64", seed: int = 0, device: str = "cuda:0",
                 ad_mode: str = "kraus"):
        if not torch.cuda.is_available():
            raise RuntimeError("TTNEngine needs a ROCm GPU (torch.cuda.is_available() is False)")
        self.device = torch.device(device)
        self.n_qubits = int(n_qubits)
        self.batch = int(batch)
        if leaf_of_qubit is None:
            leaf_of_qubit = np.arange(n_qubits)
        self.leaf_of_qubit = np.ascontiguousarray(np.asarray(leaf_of_qubit, dtype=np.int32))
        self.dtype = dtype
        self.seed = int(seed)
        self.stream = torch.cuda.current_stream(self.device)
        cfg = _abi.Config()
        cfg.n_qubits = self.n_qubits
        cfg.leaf_of_qubit = self.leaf_of_qubit.ctypes.data_as(C.POINTER(C.c_int32))
        cfg.chi_max = int(chi_max)
        cfg.cutoff = float(cutoff)
        cfg.dtype = {"c64": _abi.TTN_C64, "c128": _abi.TTN_C128}[dtype]
        cfg.ad_mode = {"kraus": _abi.TTN_AD_KRAUS, "trotter": _abi.TTN_AD_TROTTER}[ad_mode]
        self.ad_mode = ad_mode
        cfg.batch = self.batch
        cfg.seed = self.seed
        cfg.stream = C.c_void_p(self.stream.cuda_stream)
        h = C.c_void_p()
        with torch.cuda.device(self.device):
            code = lib().ttn_create(C.byref(cfg), C.byref(h))
        if code != 0:
            raise _abi.TTNError(code, "ttn_create failed")
        self._ctx = h

    # ---------------------------------------------------------------------
    def close(self):
        if getattr(self, "_ctx", None):
            lib().ttn_destroy(self._ctx)
            self._ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _dev(self, x, dtype):
        return torch.as_tensor(x, dtype=dtype, device=self.device).contiguous()

    # ------------------------------------------------------------ state ----
    def init_product(self, basis=None):
        b = None if basis is None else np.ascontiguousarray(np.asarray(basis, dtype=np.uint8))
        check(lib().ttn_init_product(self._ctx, None if b is None else b.ctypes.data), self._ctx)
        self._keep = b

    def apply_1q(self, q: int, u):
        """u: [2,2] or [rows,2,2] complex matrix (numpy or torch)."""
        m = torch.view_as_real(torch.as_tensor(np.asarray(u, dtype=np.complex128) if not torch.is_tensor(u)
                                               else u.to(torch.complex128)).contiguous())
        m = m.to(self.device).contiguous()
        stride = 0 if m.dim() == 3 else 8
        check(lib().ttn_apply_1q(self._ctx, int(q), _ptr(m), stride), self._ctx)
        self.stream.synchronize()

    def apply_2q(self, q0: int, q1: int, g):
        g = np.ascontiguousarray(np.stack([np.real(g), np.imag(g)], axis=-1).astype(np.float64))
        check(lib().ttn_apply_2q(self._ctx, int(q0), int(q1), g.ctypes.data), self._ctx)

    def measure(self, q: int, basis: int = 0, draw: int = 0, traj_offset: int = 0, forced=None, logp=None):
        bits = torch.zeros(self.batch, dtype=torch.uint8, device=self.device)
        if logp is None:
            logp = torch.zeros(self.batch, dtype=torch.float64, device=self.device)
        f = None if forced is None else self._dev(forced, torch.uint8)
        check(lib().ttn_measure_project(self._ctx, int(q), int(basis), _ptr(f), _ptr(bits), _ptr(logp),
                                        int(traj_offset), int(draw)), self._ctx)
        return bits, logp

    def kraus_jump(self, q: int, k0, k1, draw: int = 0, traj_offset: int = 0, forced=None, logp=None):
        k = np.stack([np.asarray(k0, dtype=np.complex128), np.asarray(k1, dtype=np.complex128)])
        kt = torch.view_as_real(torch.as_tensor(k)).contiguous().to(self.device)
        br = torch.zeros(self.batch, dtype=torch.int8, device=self.device)
        if logp is None:
            logp = torch.zeros(self.batch, dtype=torch.float64, device=self.device)
        f = None if forced is None else self._dev(forced, torch.int8)
        check(lib().ttn_kraus_jump(self._ctx, int(q), _ptr(kt), 0, _ptr(f), _ptr(br), _ptr(logp),
                                   int(traj_offset), int(draw)), self._ctx)
        return br, logp

    # ---------------------------------------------------------- circuits ----
    def upload(self, circuit) -> OpList:
        return OpList(self, circuit.ops, circuit.n_loc, circuit.n_rec, circuit.n_draws)

    def _params(self, ol: OpList, theta, gamma):
        def prep(x):
            if x is None:
                return torch.zeros(1, max(ol.n_loc, 1), dtype=torch.float64, device=self.device)
            t = torch.as_tensor(x, dtype=torch.float64)
            if t.dim() == 0:
                t = t.reshape(1, 1).expand(1, max(ol.n_loc, 1))
            if t.dim() == 1:
                t = t.reshape(1, -1)
            return t.to(self.device).contiguous()
        th, ga = prep(theta), prep(gamma)
        if th.shape[0] != ga.shape[0]:
            if th.shape[0] == 1:
                th = th.expand(ga.shape[0], -1).contiguous()
            elif ga.shape[0] == 1:
                ga = ga.expand(th.shape[0], -1).contiguous()
        rows = th.shape[0]
        if rows not in (1, self.batch):
            raise ValueError("parameters must have 1 or `batch` rows")
        if th.shape[1] < ol.n_loc or ga.shape[1] < ol.n_loc:
            raise ValueError("parameters need n_loc columns")
        stride = 0 if rows == 1 else th.shape[1]
        if rows > 1 and th.shape[1] != ga.shape[1]:
            raise ValueError("theta and gamma must have the same column count")
        return th, ga, stride

    def outputs(self, ol: OpList) -> tuple:
        """Record, branch and log P buffers for run_circuit(out=...): a graph
        captured in "graph" mode is replayed only while the same buffers (and
        parameter tensors) are passed."""
        return (torch.zeros(self.batch, max(ol.n_rec, 1), dtype=torch.uint8, device=self.device),
                torch.zeros(self.batch, max(ol.n_ad, 1), dtype=torch.int8, device=self.device),
                torch.zeros(self.batch, dtype=torch.float64, device=self.device))

    def run_circuit(self, ol: OpList, theta=None, gamma=None, traj_offset: int = 0,
                    stats: bool = True, out=None) -> RunResult:
        th, ga, stride = self._params(ol, theta, gamma)
        rec, br, logp = self.outputs(ol) if out is None else out
        st = _abi.Stats()
        code = lib().ttn_batch_run_circuit(self._ctx, ol._h, _ptr(th), _ptr(ga), stride, int(traj_offset),
                                           _ptr(rec), _ptr(br), _ptr(logp), C.byref(st) if stats else None)
        if code not in (0, _abi.TTN_ENONFINITE):
            check(code, self._ctx)
        self._hold = (th, ga)
        return RunResult(rec[:, :ol.n_rec], br[:, :ol.n_ad], logp, st.as_dict() if stats else {})

    def log_prob(self, ol: OpList, records, branches=None, theta=None, gamma=None):
        th, ga, stride = self._params(ol, theta, gamma)
        rec = self._dev(records, torch.uint8)
        br = None if branches is None or ol.n_ad == 0 else self._dev(branches, torch.int8)
        logp = torch.zeros(self.batch, dtype=torch.float64, device=self.device)
        st = _abi.Stats()
        code = lib().ttn_log_prob(self._ctx, ol._h, _ptr(rec), _ptr(br), _ptr(th), _ptr(ga), stride,
                                  _ptr(logp), C.byref(st))
        if code not in (0, _abi.TTN_EPROB):
            check(code, self._ctx)
        return logp, st.as_dict()

    def log_prob_grad(self, ol: OpList, records, branches=None, theta=None, gamma=None):
        """log P of the records and d log P / d(theta_l, gamma_l) per row (ttn_log_prob_grad).

        Returns (logp [rows], dtheta [rows, n_loc], dgamma [rows, n_loc], stats)."""
        th, ga, stride = self._params(ol, theta, gamma)
        rec = self._dev(records, torch.uint8)
        br = None if branches is None or ol.n_ad == 0 else self._dev(branches, torch.int8)
        logp = torch.zeros(self.batch, dtype=torch.float64, device=self.device)
        n_loc = max(ol.n_loc, 1)
        dth = torch.zeros(self.batch, n_loc, dtype=torch.float64, device=self.device)
        dga = torch.zeros(self.batch, n_loc, dtype=torch.float64, device=self.device)
        st = _abi.Stats()
        code = lib().ttn_log_prob_grad(self._ctx, ol._h, _ptr(rec), _ptr(br), _ptr(th), _ptr(ga), stride,
                                       _ptr(logp), _ptr(dth), _ptr(dga), C.byref(st))
        if code not in (0, _abi.TTN_EPROB):
            check(code, self._ctx)
        return logp, dth[:, :ol.n_loc], dga[:, :ol.n_loc], st.as_dict()

    def run_mode(self, mode: str) -> tuple:
        """"dynamic" (default), "static" or "graph" (see ttn_set_run_mode).
        Returns (graph captures, graph replays) so far."""
        modes = {"dynamic": _abi.TTN_RUN_DYNAMIC, "static": _abi.TTN_RUN_STATIC, "graph": _abi.TTN_RUN_GRAPH}
        if mode not in modes:
            raise ValueError(f"run mode must be one of {sorted(modes)}")
        m = modes[mode]
        cap, rep = C.c_int64(0), C.c_int64(0)
        check(lib().ttn_set_run_mode(self._ctx, m, C.byref(cap), C.byref(rep)), self._ctx)
        return cap.value, rep.value

    def trace_probs(self, probs: torch.Tensor | None):
        """Record the probability of every sampled event of later runs into
        probs [rows, n_draws] (float64, on the device); None stops it."""
        if probs is None:
            check(lib().ttn_trace_probs(self._ctx, None, 0), self._ctx)
            self._trace = None
            return
        if probs.dtype != torch.float64 or probs.dim() != 2 or probs.shape[0] != self.batch or \
                not probs.is_contiguous() or probs.device != self.device:
            raise ValueError("probs must be a contiguous float64 [batch, n] tensor on the engine's device")
        check(lib().ttn_trace_probs(self._ctx, _ptr(probs), int(probs.shape[1])), self._ctx)
        self._trace = probs

    def decode(self, records: torch.Tensor, data_rec, checks) -> torch.Tensor:
        data_rec = np.ascontiguousarray(np.asarray(data_rec, dtype=np.int32))
        checks = np.ascontiguousarray(np.asarray(checks, dtype=np.uint8))
        rec = records.contiguous()
        fail = torch.zeros(self.batch, dtype=torch.uint8, device=self.device)
        check(lib().ttn_decode(self._ctx, _ptr(rec), int(rec.shape[1]), data_rec.ctypes.data,
                               int(data_rec.size), checks.ctypes.data, int(checks.shape[0]), _ptr(fail)),
              self._ctx)
        return fail

    # ---------------------------------------------------------- profiling ----
    def profile(self, on: bool = True):
        check(lib().ttn_profile_enable(self._ctx, 1 if on else 0), self._ctx)

    def autotune(self, on, force_cfg=None) -> tuple:
        """Tile-shape tuning of the GEMM launches: True measures new shapes,
        False keeps the measured choices, None forgets them; force_cfg = c
        (0..5) runs every launch in tile shape c instead (testing).  Returns
        (shapes measured, shapes whose choice differs from the fixed rule)."""
        shapes, changed = C.c_int64(0), C.c_int64(0)
        mode = -1 if on is None else (1 if on else 0)
        if force_cfg is not None:
            mode = 2 + int(force_cfg)
        check(lib().ttn_autotune(self._ctx, mode, C.byref(shapes), C.byref(changed)), self._ctx)
        return shapes.value, changed.value

    def profile_read(self) -> dict:
        out = {}
        for name, cls in _abi.CLASSES.items():
            ms, n, fl, by = C.c_double(), C.c_int64(), C.c_double(), C.c_double()
            check(lib().ttn_profile_read(self._ctx, cls, C.byref(ms), C.byref(n), C.byref(fl), C.byref(by)),
                  self._ctx)
            out[name] = {"ms": ms.value, "launches": n.value, "alg_flops": fl.value, "alg_bytes": by.value}
        return out

    # ------------------------------------------------------------ exports ----
    def compress(self):
        check(lib().ttn_compress(self._ctx), self._ctx)

    def statevector(self, row: int = 0) -> np.ndarray:
        amp = torch.zeros(2 ** self.n_qubits, 2, dtype=torch.float64, device=self.device)
        check(lib().ttn_to_statevector(self._ctx, int(row), _ptr(amp)), self._ctx)
        a = amp.cpu().numpy()
        return a[:, 0] + 1j * a[:, 1]

    def bond_dims(self, row: int = 0) -> np.ndarray:
        L = 2
        while L < self.n_qubits:
            L *= 2
        out = np.zeros(L, dtype=np.int32)
        check(lib().ttn_bond_dims(self._ctx, int(row), out.ctypes.data), self._ctx)
        return out

    def uniforms(self, traj_offset: int, rows: int, n_draws: int) -> np.ndarray:
        out = torch.zeros(rows, n_draws, dtype=torch.float64, device=self.device)
        check(lib().ttn_uniforms(self._ctx, int(traj_offset), int(rows), int(n_draws), _ptr(out)), self._ctx)
        return out.cpu().numpy()


def philox_uniform_host(seed: int, traj: int, draw: int) -> float:
    """The engine's counter-based draw evaluated on the host (no GPU needed)."""
    return float(lib().ttn_philox_uniform_host(int(seed), int(traj), int(draw)))


def version() -> str:
    return lib().ttn_version().decode()
