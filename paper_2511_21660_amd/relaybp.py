"""ctypes binding of the Relay-BP C ABI (``include/relaybp.h``).

Argument marshalling only: every step of decoding runs in the HIP kernels of
``librelaybp.so``.  Device buffers are torch CUDA (HIP) tensors; the stream is
torch's current stream of the tensor's device.  There is no CPU fallback: if
the library is not built, or no GPU is present, calls raise.
"""
from __future__ import annotations

import ctypes
import os
import re

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "librelaybp.so")
HEADER_PATH = os.path.join(os.path.dirname(_HERE), "include", "relaybp.h")

STATUS = {
    0: "RB_OK", 1: "RB_E_INVALID_ARG", 2: "RB_E_SHAPE", 3: "RB_E_DUPLICATE_ENTRY",
    4: "RB_E_PRIOR_RANGE", 5: "RB_E_DEVICE", 6: "RB_E_OOM", 7: "RB_E_WORKSPACE",
    8: "RB_E_UNSUPPORTED", 9: "RB_E_NONFINITE", 10: "RB_E_INTERNAL",
}
ANCHOR_CHAIN, ANCHOR_PRIOR = 0, 1
IO_BYTES, IO_BITS32 = 0, 1
PREC_F32, PREC_F16 = 0, 1


def pack_bits(a) -> np.ndarray:
    """uint8 0/1 array [B, K] -> int32 words [B, ceil(K / 32)], entry k in bit
    k % 32 of word k // 32 (the RB_IO_BITS32 layout)."""
    a = np.ascontiguousarray(np.asarray(a) != 0)
    b, k = a.shape
    w = (k + 31) // 32
    pad = np.zeros((b, 32 * w), dtype=bool)
    pad[:, :k] = a
    by = np.packbits(pad, axis=1, bitorder="little")          # [B, 4w] bytes, little-endian bits
    return np.ascontiguousarray(by).view("<u4").astype(np.uint32).view(np.int32).reshape(b, w)


def unpack_bits(words, k: int) -> np.ndarray:
    """Inverse of pack_bits: int32 / uint32 words [B, W] -> uint8 0/1 [B, k]."""
    w = np.ascontiguousarray(np.asarray(words)).astype(np.uint32).astype("<u4")
    by = w.view(np.uint8).reshape(w.shape[0], -1)
    return np.unpackbits(by, axis=1, bitorder="little")[:, :k].astype(np.uint8)


class RelayError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS.get(status, status)}: {message}")
        self.status = status


class RBParams(ctypes.Structure):
    _fields_ = [
        ("num_legs", ctypes.c_int32),
        ("iters_first", ctypes.c_int32),
        ("iters_leg", ctypes.c_int32),
        ("num_solutions", ctypes.c_int32),
        ("gamma_first", ctypes.c_float),
        ("gamma_lo", ctypes.c_float),
        ("gamma_hi", ctypes.c_float),
        ("llr_clip", ctypes.c_float),
        ("seed", ctypes.c_uint64),
        ("anchor", ctypes.c_int32),
        ("max_total_iters", ctypes.c_int32),
        ("io_layout", ctypes.c_int32),
        ("precision", ctypes.c_int32),
    ]


class RBInfo(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int32) for n in ("M", "N")] + [("num_edges", ctypes.c_int64)] + [
        (n, ctypes.c_int32) for n in (
            "max_row_degree", "max_col_degree", "variant", "lanes_per_shot", "checks_per_lane",
            "row_slots", "cols_per_lane", "col_slots", "shots_per_block", "threads_per_block",
            "waves_per_simd_target", "lds_bytes_per_block", "blocks_per_cu", "grid_blocks",
            "num_variants")]


class RBPlanReport(ctypes.Structure):
    _fields_ = [("variant", ctypes.c_int32), ("block_kernel", ctypes.c_int32), ("lds_bytes", ctypes.c_int32),
                ("check_gathers", ctypes.c_int64), ("check_bank_cycles", ctypes.c_int64),
                ("fault_gathers", ctypes.c_int64), ("fault_bank_cycles", ctypes.c_int64)]


class RBCodeDesc(ctypes.Structure):
    _fields_ = [("M", ctypes.c_int32), ("N", ctypes.c_int32), ("nnz", ctypes.c_int64),
                ("rows", ctypes.c_void_p), ("cols", ctypes.c_void_p), ("prior_p", ctypes.c_void_p)]


_lib = None


def load_library():
    """Loads librelaybp.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built; run paper_2511_21660_amd.build.build()")
    L = ctypes.CDLL(LIB_PATH)
    P, i32, i64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
    L.rb_params_default.argtypes = [ctypes.POINTER(RBParams)]
    L.rb_create.argtypes = [ctypes.POINTER(P), i32, i32, i64, P, P, P, ctypes.POINTER(RBParams), i32]
    L.rb_destroy.argtypes = [P]
    L.rb_destroy.restype = None
    L.rb_decode.argtypes = [P, i64, P, P, P, P, P, P, P, P]
    L.rb_trace.argtypes = [P, i64, P, P, ctypes.c_float, i32, P, P]
    L.rb_get_llr.argtypes = [P, P]
    L.rb_get_gamma_table.argtypes = [P, P]
    L.rb_get_info.argtypes = [P, ctypes.POINTER(RBInfo)]
    L.rb_set_variant.argtypes = [P, i32]
    L.rb_set_leg_gamma.argtypes = [P, i32, P]
    L.rb_set_prior_scale.argtypes = [P, ctypes.c_float]
    L.rb_sync_status.argtypes = [P]
    L.rb_autotune.argtypes = [P, i64, P, i32, ctypes.POINTER(i32), ctypes.POINTER(ctypes.c_float)]
    L.rb_reserve.argtypes = [P, i64]
    L.rb_workspace_size.argtypes = [P, i64]
    L.rb_workspace_size.restype = ctypes.c_size_t
    L.rb_create_multi.argtypes = [ctypes.POINTER(P), i32, ctypes.POINTER(RBCodeDesc),
                                  ctypes.POINTER(RBParams), i32]
    L.rb_decode_multi.argtypes = [P, i64, P, P, P, P, P, P, P, P, P, ctypes.c_size_t, P]
    L.rb_decode_multi_noalloc.argtypes = [P, i64, P, P, P, P, P, P, P, P, P]
    L.rb_noalloc_max_batch.argtypes = [P]
    L.rb_noalloc_max_batch.restype = i64
    L.rb_autotune_multi.argtypes = [P, ctypes.POINTER(i64), ctypes.POINTER(P), i32,
                                    ctypes.POINTER(i32)]
    L.rb_set_code_variant.argtypes = [P, i32, i32]
    L.rb_train_tape_size.argtypes = [P, i64, i32, i32]
    L.rb_train_tape_size.restype = ctypes.c_size_t
    L.rb_forward_train.argtypes = [P, i64, P, P, P, i32, i32, P, P, ctypes.c_size_t, P]
    L.rb_backward.argtypes = [P, i64, P, P, P, i32, i32, P, ctypes.c_size_t, P, P, P, P]
    L.rb_plan_check.argtypes = [i32, i32, i64, P, P, i32, ctypes.POINTER(RBPlanReport)]
    L.rb_syndrome.argtypes = [P, i64, P, P, P, P]
    L.rb_status_string.argtypes = [ctypes.c_int]
    L.rb_status_string.restype = ctypes.c_char_p
    L.rb_last_error_message.argtypes = []
    L.rb_last_error_message.restype = ctypes.c_char_p
    for name in ("rb_params_default", "rb_create", "rb_decode", "rb_trace", "rb_get_llr",
                 "rb_get_gamma_table", "rb_get_info", "rb_set_variant", "rb_sync_status",
                 "rb_autotune", "rb_reserve", "rb_create_multi", "rb_decode_multi", "rb_decode_multi_noalloc",
                 "rb_autotune_multi", "rb_set_code_variant", "rb_forward_train", "rb_backward", "rb_set_leg_gamma",
                 "rb_set_prior_scale", "rb_plan_check", "rb_syndrome"):
        getattr(L, name).restype = ctypes.c_int
    _lib = L
    return L


def header_functions(path: str = HEADER_PATH):
    """Names of the functions declared in the public header."""
    text = open(path).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(rb_[a-z_]+)\s*\(", text)))


def _check(status: int):
    if status != 0:
        L = load_library()
        raise RelayError(status, L.rb_last_error_message().decode())


def default_params(**overrides) -> RBParams:
    p = RBParams()
    _check(load_library().rb_params_default(ctypes.byref(p)))
    for k, v in overrides.items():
        setattr(p, k, v)
    return p


def bp_params(rounds=25, **overrides) -> dict:
    """Decoder parameters for plain min-sum BP as a special case of Relay: one
    leg of `rounds` iterations with gamma = 0, so the memory term
    (1 - gamma) lambda(0) + gamma Lambda(t-1) is the prior itself (paper Sec.
    2.3 with gamma = 0).  The paper hands the next decoding stage the LLRs of
    25 such rounds when the memory-BP pre-decoder fails (Sec. 7.1); decode
    with want_llr=True returns them (after `rounds` iterations, or at
    convergence if plain BP converges earlier)."""
    p = dict(num_legs=1, iters_first=rounds, iters_leg=rounds, num_solutions=1, gamma_first=0.0,
             gamma_lo=0.0, gamma_hi=0.0, llr_clip=2.0 ** 64, seed=0, anchor=ANCHOR_CHAIN, max_total_iters=0)
    p.update(overrides)
    return p


def plan_check(m: int, n: int, rows, cols, variant: int = -1) -> dict:
    """Host-only check of the LDS gather tables for H (rows, cols: COO) on
    configuration `variant` (-1: the automatic choice); raises RelayError
    (RB_E_INTERNAL) if a table is inconsistent with H.  Returns the report:
    configuration, LDS bytes, and the number and modelled bank cost of the
    table-driven gathers of one iteration (2 per gather is conflict-free)."""
    L = load_library()
    rows = np.ascontiguousarray(rows, np.int32)
    cols = np.ascontiguousarray(cols, np.int32)
    rep = RBPlanReport()
    _check(L.rb_plan_check(m, n, rows.size, rows.ctypes.data_as(ctypes.c_void_p),
                           cols.ctypes.data_as(ctypes.c_void_p), variant, ctypes.byref(rep)))
    return {f: getattr(rep, f) for f, _ in RBPlanReport._fields_}


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _stream(device):
    import torch

    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


class Decoder:
    """Relay-BP decoder for one check matrix and prior vector on one GPU."""

    def __init__(self, m, n, rows, cols, prior, params=None, device=0, **overrides):
        L = load_library()
        self.m, self.n = int(m), int(n)
        self.device = int(device)
        if params is None:
            params = default_params(**overrides)
        elif isinstance(params, dict):
            params = default_params(**params, **overrides)
        self.params = params
        self.bits = params.io_layout == IO_BITS32
        self.wm, self.wn = (self.m + 31) // 32, (self.n + 31) // 32
        rows = np.ascontiguousarray(rows, dtype=np.int32)
        cols = np.ascontiguousarray(cols, dtype=np.int32)
        prior = np.ascontiguousarray(np.broadcast_to(np.asarray(prior, np.float64), (self.n,)))
        h = ctypes.c_void_p()
        _check(L.rb_create(ctypes.byref(h), self.m, self.n, rows.size,
                           rows.ctypes.data_as(ctypes.c_void_p), cols.ctypes.data_as(ctypes.c_void_p),
                           prior.ctypes.data_as(ctypes.c_void_p), ctypes.byref(params), self.device))
        self._h = h

    @classmethod
    def from_problem(cls, problem, device=0, **params):
        return cls(problem.m, problem.n, problem.rows, problem.cols, problem.prior,
                   device=device, **params)

    def close(self):
        if getattr(self, "_h", None):
            load_library().rb_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _dev(self):
        import torch

        return torch.device("cuda", self.device)

    def _io(self):
        """(dtype, syndrome row length, correction row length) of the context's layout."""
        import torch

        return (torch.int32, self.wm, self.wn) if self.bits else (torch.uint8, self.m, self.n)

    def decode(self, syndromes, want_weight=True, want_llr=False, out=None):
        """syndromes: uint8 CUDA tensor [B, M] (bit-packed layout: int32 [B, ceil(M/32)]).
        Returns a dict of CUDA tensors corr [B, N] u8 (bit-packed: int32 [B, ceil(N/32)]),
        conv [B] u8, legs [B] i32, iters [B] i32, and optionally weight [B] f64 and
        llr [B, N] f32.  Work is enqueued on the current stream."""
        import torch

        dt, sw, cw = self._io()
        if syndromes.dtype != dt or syndromes.dim() != 2 or syndromes.shape[1] != sw:
            raise ValueError(f"syndromes must be {dt} [B, {sw}]")
        if not syndromes.is_cuda:
            raise ValueError("syndromes must be a CUDA (HIP) tensor")
        syndromes = syndromes.contiguous()
        b = syndromes.shape[0]
        dev = syndromes.device
        if out is None:
            out = {
                "corr": torch.empty((b, cw), dtype=dt, device=dev),
                "conv": torch.empty(b, dtype=torch.uint8, device=dev),
                "legs": torch.empty(b, dtype=torch.int32, device=dev),
                "iters": torch.empty(b, dtype=torch.int32, device=dev),
            }
            if want_weight:
                out["weight"] = torch.empty(b, dtype=torch.float64, device=dev)
            if want_llr:
                out["llr"] = torch.empty((b, self.n), dtype=torch.float32, device=dev)
        _check(load_library().rb_decode(self._h, b, _ptr(syndromes), _ptr(out["corr"]),
                                        _ptr(out["conv"]), _ptr(out["legs"]), _ptr(out["iters"]),
                                        _ptr(out.get("weight")), _ptr(out.get("llr")),
                                        _stream(dev)))
        return out

    def syndrome(self, corr, syn_in=None, out=None):
        """(syn_in XOR H corr) mod 2 for corr uint8 [B, N] on the device: uint8 [B, M]
        (bit-packed layout: int32 [B, ceil(N/32)] -> int32 [B, ceil(M/32)]; syn_in None
        reads as zero; out may be syn_in).  Enqueued on the current stream."""
        import torch

        dt, sw, cw = self._io()
        if corr.dtype != dt or corr.dim() != 2 or corr.shape[1] != cw or not corr.is_cuda:
            raise ValueError(f"corr must be a {dt} CUDA tensor [B, {cw}]")
        corr = corr.contiguous()
        b = corr.shape[0]
        if syn_in is not None and (syn_in.dtype != dt or tuple(syn_in.shape) != (b, sw)
                                   or not syn_in.is_contiguous()):
            raise ValueError(f"syn_in must be a contiguous {dt} CUDA tensor [{b}, {sw}]")
        if out is None:
            out = torch.empty((b, sw), dtype=dt, device=corr.device)
        _check(load_library().rb_syndrome(self._h, b, _ptr(corr), _ptr(syn_in), _ptr(out), _stream(corr.device)))
        return out

    def trace(self, syndromes, gamma, t_iters, scale=1.0):
        """Marginals Lambda(t), t = 0..T, of one leg with per-column gamma: [B, T+1, N]."""
        import torch

        syndromes = syndromes.contiguous()
        gamma = gamma.to(device=syndromes.device, dtype=torch.float32).contiguous()
        b = syndromes.shape[0]
        tr = torch.empty((b, t_iters + 1, self.n), dtype=torch.float32, device=syndromes.device)
        _check(load_library().rb_trace(self._h, b, _ptr(syndromes), _ptr(gamma), float(scale),
                                       int(t_iters), _ptr(tr), _stream(syndromes.device)))
        return tr

    def llr(self) -> np.ndarray:
        w = np.zeros(self.n, np.float32)
        _check(load_library().rb_get_llr(self._h, w.ctypes.data_as(ctypes.c_void_p)))
        return w

    def gamma_table(self) -> np.ndarray:
        g = np.zeros((self.params.num_legs, self.n), np.float32)
        _check(load_library().rb_get_gamma_table(self._h, g.ctypes.data_as(ctypes.c_void_p)))
        return g

    def info(self) -> dict:
        inf = RBInfo()
        _check(load_library().rb_get_info(self._h, ctypes.byref(inf)))
        return {k: getattr(inf, k) for k, _ in RBInfo._fields_}

    def set_variant(self, v: int):
        _check(load_library().rb_set_variant(self._h, int(v)))

    def set_leg_gamma(self, leg: int, gamma):
        """Replaces leg `leg`'s memory strengths (float [N]) for later decodes
        (e.g. a learned first leg).  Synchronises the device."""
        g = np.ascontiguousarray(np.asarray(gamma, dtype=np.float32))
        if g.shape != (self.n,):
            raise ValueError(f"gamma must be float [{self.n}]")
        _check(load_library().rb_set_leg_gamma(self._h, int(leg), g.ctypes.data_as(ctypes.c_void_p)))

    def set_prior_scale(self, scale: float):
        """Sets s in Lambda(0) = s * w for later decodes.  Synchronises the device."""
        _check(load_library().rb_set_prior_scale(self._h, float(scale)))

    def tape_bytes(self, b: int, t_iters: int, ckpt_every: int) -> int:
        return int(load_library().rb_train_tape_size(self._h, int(b), int(t_iters), int(ckpt_every)))

    def forward_train(self, syndromes, gamma, scale, t_iters, ckpt_every, tape, llr_out):
        _check(load_library().rb_forward_train(
            self._h, syndromes.shape[0], _ptr(syndromes), _ptr(gamma), _ptr(scale), int(t_iters),
            int(ckpt_every), _ptr(llr_out), _ptr(tape), tape.numel(), _stream(syndromes.device)))

    def backward_train(self, syndromes, gamma, scale, t_iters, ckpt_every, tape, dllr, dgamma,
                       dscale):
        _check(load_library().rb_backward(
            self._h, syndromes.shape[0], _ptr(syndromes), _ptr(gamma), _ptr(scale), int(t_iters),
            int(ckpt_every), _ptr(tape), tape.numel(), _ptr(dllr), _ptr(dgamma), _ptr(dscale),
            _stream(syndromes.device)))

    def reserve(self, max_batch: int):
        """Enables longest-first scheduling for batches of up to max_batch syndromes
        (allocates a device workspace once; synchronises the device)."""
        _check(load_library().rb_reserve(self._h, int(max_batch)))

    def autotune(self, syndromes, reps: int = 3):
        """Times every fitting kernel configuration on these syndromes and keeps
        the fastest; returns (variant, ms per decode).  Synchronises the device."""
        syndromes = syndromes.contiguous()
        v = ctypes.c_int32()
        ms = ctypes.c_float()
        _check(load_library().rb_autotune(self._h, syndromes.shape[0], _ptr(syndromes), int(reps),
                                          ctypes.byref(v), ctypes.byref(ms)))
        return v.value, ms.value

    def sync(self):
        _check(load_library().rb_sync_status(self._h))


class MultiDecoder:
    """One persistent launch over syndromes of several codes (rb_decode_multi)."""

    def __init__(self, problems, params=None, device=0, **overrides):
        L = load_library()
        self.device = int(device)
        if params is None:
            params = default_params(**overrides)
        elif isinstance(params, dict):
            params = default_params(**params, **overrides)
        self.params = params
        self.bits = params.io_layout == IO_BITS32
        self.ms = [int(p.m) for p in problems]
        self.ns = [int(p.n) for p in problems]
        self.m_max, self.n_max = max(self.ms), max(self.ns)
        keep = []
        descs = (RBCodeDesc * len(problems))()
        for k, p in enumerate(problems):
            rows = np.ascontiguousarray(p.rows, dtype=np.int32)
            cols = np.ascontiguousarray(p.cols, dtype=np.int32)
            prior = np.ascontiguousarray(np.broadcast_to(np.asarray(p.prior, np.float64), (p.n,)))
            keep += [rows, cols, prior]
            descs[k] = RBCodeDesc(p.m, p.n, rows.size, rows.ctypes.data_as(ctypes.c_void_p),
                                  cols.ctypes.data_as(ctypes.c_void_p),
                                  prior.ctypes.data_as(ctypes.c_void_p))
        h = ctypes.c_void_p()
        _check(L.rb_create_multi(ctypes.byref(h), len(problems), descs, ctypes.byref(params),
                                 self.device))
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            load_library().rb_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def workspace_bytes(self, b: int) -> int:
        return int(load_library().rb_workspace_size(self._h, int(b)))

    def alloc(self, b: int, want_weight=True, want_llr=False):
        """Output buffers and workspace for a batch of b syndromes (reusable, e.g.
        across hipGraph replays)."""
        import torch

        dev = torch.device("cuda", self.device)
        dt, _, cw = self._io()
        out = {
            "corr": torch.empty((b, cw), dtype=dt, device=dev),
            "conv": torch.empty(b, dtype=torch.uint8, device=dev),
            "legs": torch.empty(b, dtype=torch.int32, device=dev),
            "iters": torch.empty(b, dtype=torch.int32, device=dev),
            "workspace": torch.empty(max(1, self.workspace_bytes(b)), dtype=torch.uint8,
                                     device=dev),
        }
        if want_weight:
            out["weight"] = torch.empty(b, dtype=torch.float64, device=dev)
        if want_llr:
            out["llr"] = torch.empty((b, self.n_max), dtype=torch.float32, device=dev)
        return out

    def _io(self):
        import torch

        if self.bits:
            return torch.int32, (self.m_max + 31) // 32, (self.n_max + 31) // 32
        return torch.uint8, self.m_max, self.n_max

    def decode(self, code_id, syndromes, out=None, want_weight=True, want_llr=False):
        """code_id int32 [B], syndromes uint8 [B, M_max] (bit-packed layout: int32
        [B, ceil(M_max/32)]; CUDA).  Enqueues on the current stream; returns the dict
        of output tensors."""
        import torch

        dt, sw, _ = self._io()
        if syndromes.dtype != dt or syndromes.shape[1] != sw:
            raise ValueError(f"syndromes must be {dt} [B, {sw}]")
        if code_id.dtype != torch.int32 or code_id.shape[0] != syndromes.shape[0]:
            raise ValueError("code_id must be int32 [B]")
        b = syndromes.shape[0]
        if out is None:
            out = self.alloc(b, want_weight, want_llr)
        ws = out["workspace"]
        _check(load_library().rb_decode_multi(
            self._h, b, _ptr(code_id), _ptr(syndromes), _ptr(out["corr"]), _ptr(out["conv"]),
            _ptr(out["legs"]), _ptr(out["iters"]), _ptr(out.get("weight")), _ptr(out.get("llr")),
            _ptr(ws), ws.numel(), _stream(syndromes.device)))
        return out

    def noalloc_max_batch(self) -> int:
        return int(load_library().rb_noalloc_max_batch(self._h))

    def decode_noalloc(self, code_id, syndromes, out):
        """rb_decode_multi_noalloc: the same decode with the library's static
        scratch instead of a workspace (``out`` from alloc(); its workspace
        is not used).  Enqueues on the current stream."""
        import torch

        dt, sw, _ = self._io()
        if syndromes.dtype != dt or syndromes.shape[1] != sw:
            raise ValueError(f"syndromes must be {dt} [B, {sw}]")
        if code_id.dtype != torch.int32 or code_id.shape[0] != syndromes.shape[0]:
            raise ValueError("code_id must be int32 [B]")
        _check(load_library().rb_decode_multi_noalloc(
            self._h, syndromes.shape[0], _ptr(code_id), _ptr(syndromes), _ptr(out["corr"]),
            _ptr(out["conv"]), _ptr(out["legs"]), _ptr(out["iters"]), _ptr(out.get("weight")),
            _ptr(out.get("llr")), _stream(syndromes.device)))
        return out

    def autotune(self, samples, reps: int = 3):
        """samples: list (one per code) of uint8 CUDA tensors [b_k, M_k] (or None)."""
        k = len(self.ms)
        bs = (ctypes.c_int64 * k)(*[0 if s is None else s.shape[0] for s in samples])
        ptrs = (ctypes.c_void_p * k)(*[None if s is None else s.data_ptr() for s in samples])
        chosen = (ctypes.c_int32 * k)()
        _check(load_library().rb_autotune_multi(self._h, bs, ptrs, int(reps), chosen))
        return list(chosen)

    def set_code_variant(self, k: int, variant: int):
        """Decode code k with the mixed-kernel tile `variant` (rb_set_code_variant)."""
        _check(load_library().rb_set_code_variant(self._h, int(k), int(variant)))
