"""ctypes front end of the C oracle (test infrastructure only).

The C source ``relay_oracle.c`` is compiled with gcc (-O2, -ffp-contract=off,
no fast-math) into ``liboracle_relay.so`` next to this file.  Decoding is split
into shot chunks run on a thread pool; ctypes releases the GIL during each call,
so the chunks run in parallel on the host cores.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from concurrent.futures import ThreadPoolExecutor

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "relay_oracle.c")
_SO = os.path.join(_HERE, "liboracle_relay.so")

_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle shared library (gcc, canonical FP: no contraction)."""
    if force or not os.path.exists(_SO):
        tmp = _SO + ".tmp"
        cmd = ["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fPIC",
               "-shared", "-Wall", "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True, cwd=_HERE)
        os.replace(tmp, _SO)
    return _SO


class OracleParams(ctypes.Structure):
    _fields_ = [
        ("num_legs", ctypes.c_int32),
        ("iters_first", ctypes.c_int32),
        ("iters_leg", ctypes.c_int32),
        ("num_solutions", ctypes.c_int32),
        ("gamma_first", ctypes.c_float),
        ("gamma_lo", ctypes.c_float),
        ("gamma_hi", ctypes.c_float),
        ("llr_clip", ctypes.c_double),
        ("seed", ctypes.c_uint64),
        ("anchor", ctypes.c_int32),
        ("max_total_iters", ctypes.c_int32),
    ]


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build(force=True)
        L = ctypes.CDLL(_SO)
        P = ctypes.c_void_p
        i32, i64 = ctypes.c_int, ctypes.c_long
        L.ro_philox4x32_10.argtypes = [P, P, P]
        L.ro_philox4x32_10.restype = None
        L.ro_gamma_f32.argtypes = [ctypes.c_uint64, i32, i32, ctypes.c_float, ctypes.c_float]
        L.ro_gamma_f32.restype = ctypes.c_float
        for sfx in ("f32", "f64"):
            f = getattr(L, f"ro_decode_{sfx}")
            f.argtypes = [i32, i32, i64, P, P, P, ctypes.POINTER(OracleParams), P, ctypes.c_double,
                          i64, P, P, P, P, P, P, P]
            f.restype = i32
            f = getattr(L, f"ro_trace_{sfx}")
            f.argtypes = [i32, i32, i64, P, P, P, ctypes.c_double, P, i32, ctypes.c_double, i64, P, P]
            f.restype = i32
            f = getattr(L, f"ro_minsum_trace_{sfx}")
            f.argtypes = [i32, i32, i64, P, P, P, i32, i64, P, P]
            f.restype = i32
        L.ro_sumproduct_trace.argtypes = [i32, i32, i64, P, P, P, i32, i64, P, P]
        L.ro_sumproduct_trace.restype = i32
        L.ro_round_h16.argtypes = [ctypes.c_double]
        L.ro_round_h16.restype = ctypes.c_double
        L.ro_decode_h16.argtypes = [i32, i32, i64, P, P, P, ctypes.POINTER(OracleParams), P, i64, P, P,
                                    P, P, P, P, P]
        L.ro_decode_h16.restype = i32
        L.ro_trace_h16.argtypes = [i32, i32, i64, P, P, P, P, i32, ctypes.c_double, i64, P, P]
        L.ro_trace_h16.restype = i32
        L.ro_tangent_f32.argtypes = [i32, i32, i64, P, P, P, ctypes.c_float, P, i32, ctypes.c_double, i64,
                                     P, P, ctypes.c_double, P, P, P]
        L.ro_tangent_f32.restype = i32
        _lib = L
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def philox4x32_10(key, ctr):
    k = np.asarray(key, dtype=np.uint32)
    c = np.asarray(ctr, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    lib().ro_philox4x32_10(_ptr(k), _ptr(c), _ptr(out))
    return out


def gamma_f32(seed, leg, j, lo, hi) -> np.float32:
    return np.float32(lib().ro_gamma_f32(int(seed), int(leg), int(j), float(lo), float(hi)))


def _coo(rows, cols):
    return (np.ascontiguousarray(rows, dtype=np.int32), np.ascontiguousarray(cols, dtype=np.int32))


def round_h16(x: float) -> float:
    """Nearest IEEE binary16 value (ties to even) of x, as the oracle's
    binary16 mode rounds."""
    return float(lib().ro_round_h16(float(x)))


def decode(m, n, rows, cols, prior, params: dict, syn, precision="f32", threads=None,
           chunk=None, want_llr=False, gamma1=None, scale=1.0):
    """Relay-decode syndromes [B, M]; returns dict of corr/conv/legs/iters/weight
    (and final marginals ``llr`` [B, N] when ``want_llr``).  ``gamma1`` [N]
    replaces leg 1's uniform memory strength per column and ``scale``
    multiplies the initial channel LLRs (a learned first leg); the defaults are
    the paper's decoder.  precision: "f32" (the decoder's arithmetic), "f64"
    (its twin) or "h16" (binary16 messages and marginals; no scale; llr is
    returned as float32)."""
    rows, cols = _coo(rows, cols)
    prior = np.ascontiguousarray(prior, dtype=np.float64)
    syn = np.ascontiguousarray(syn, dtype=np.uint8)
    b = syn.shape[0]
    p = OracleParams(**params)
    corr = np.zeros((b, n), np.uint8)
    conv = np.zeros(b, np.uint8)
    legs = np.zeros(b, np.int32)
    iters = np.zeros(b, np.int32)
    weight = np.zeros(b, np.float64)
    llr = np.zeros((b, n), np.float64 if precision == "f64" else np.float32) if want_llr else None
    fn = getattr(lib(), f"ro_decode_{precision}")
    g1 = None
    if gamma1 is not None:
        g1 = np.ascontiguousarray(gamma1, dtype=np.float64 if precision == "f64" else np.float32)
        if g1.shape != (n,):
            raise ValueError("gamma1 must have one entry per column")
    if precision == "h16" and scale != 1.0:
        raise ValueError("the binary16 mode has no prior scale")
    threads = threads or os.cpu_count() or 1
    chunk = chunk or max(1, min(256, (b + threads - 1) // max(threads, 1)))

    def run(s0):
        s1 = min(b, s0 + chunk)
        lead = (m, n, rows.size, _ptr(rows), _ptr(cols), _ptr(prior), ctypes.byref(p),
                _ptr(g1) if g1 is not None else None)
        if precision != "h16":
            lead = lead + (float(scale),)
        rc = fn(*lead, s1 - s0,
                _ptr(syn[s0:s1]), _ptr(corr[s0:s1]), _ptr(conv[s0:s1]), _ptr(legs[s0:s1]),
                _ptr(iters[s0:s1]), _ptr(weight[s0:s1]),
                _ptr(llr[s0:s1]) if want_llr else None)
        if rc != 0:
            raise ValueError(f"oracle decode failed with code {rc}")

    starts = list(range(0, b, chunk))
    if threads == 1 or len(starts) <= 1:
        for s in starts:
            run(s)
    else:
        with ThreadPoolExecutor(max_workers=threads) as ex:
            list(ex.map(run, starts))
    out = {"corr": corr, "conv": conv, "legs": legs, "iters": iters, "weight": weight}
    if want_llr:
        out["llr"] = llr
    return out


def trace(m, n, rows, cols, prior, gamma, t_iters, syn, scale=1.0, precision="f32",
          llr_clip=2.0 ** 64):
    """Marginal trace [B, T+1, N] of one leg with per-column gamma, no early stop
    (precision "f32", "f64" or "h16")."""
    rows, cols = _coo(rows, cols)
    prior = np.ascontiguousarray(prior, dtype=np.float64)
    dt = np.float64 if precision == "f64" else np.float32
    gamma = np.ascontiguousarray(np.broadcast_to(np.asarray(gamma, dtype=dt), (n,)))
    syn = np.ascontiguousarray(syn, dtype=np.uint8)
    b = syn.shape[0]
    out = np.zeros((b, t_iters + 1, n), dt)
    if precision == "h16":
        if scale != 1.0:
            raise ValueError("the binary16 mode has no prior scale")
        rc = lib().ro_trace_h16(m, n, rows.size, _ptr(rows), _ptr(cols), _ptr(prior), _ptr(gamma),
                                int(t_iters), float(llr_clip), b, _ptr(syn), _ptr(out))
        if rc != 0:
            raise ValueError(f"oracle trace failed with code {rc}")
        return out
    rc = getattr(lib(), f"ro_trace_{precision}")(m, n, rows.size, _ptr(rows), _ptr(cols),
                                                 _ptr(prior), float(scale), _ptr(gamma),
                                                 int(t_iters), float(llr_clip), b, _ptr(syn),
                                                 _ptr(out))
    if rc != 0:
        raise ValueError(f"oracle trace failed with code {rc}")
    return out


def tangent(m, n, rows, cols, prior, gamma, t_iters, syn, dgamma, dscale=0.0, scale=1.0,
            llr_clip=2.0 ** 64, dwprime=None):
    """Forward-mode derivative of one leg's Lambda(T) along its FP32 trajectory.

    The leg is the one ``trace`` runs (FP32, per-column gamma, channel LLRs
    w' = scale * w, no early stop); the direction is (dgamma [N], dscale), plus
    dwprime [N] on w' itself if given.  Returns
    (Lambda(T) float32 [B, N], dLambda(T) float64 [B, N]).
    """
    rows, cols = _coo(rows, cols)
    prior = np.ascontiguousarray(prior, dtype=np.float64)
    gamma = np.ascontiguousarray(np.broadcast_to(np.asarray(gamma, dtype=np.float32), (n,)))
    dgamma = np.ascontiguousarray(np.broadcast_to(np.asarray(dgamma, dtype=np.float64), (n,)))
    syn = np.ascontiguousarray(syn, dtype=np.uint8)
    b = syn.shape[0]
    lam = np.zeros((b, n), np.float32)
    dlam = np.zeros((b, n), np.float64)
    dwp = None if dwprime is None else np.ascontiguousarray(np.broadcast_to(
        np.asarray(dwprime, dtype=np.float64), (n,)))
    rc = lib().ro_tangent_f32(m, n, rows.size, _ptr(rows), _ptr(cols), _ptr(prior), float(scale),
                              _ptr(gamma), int(t_iters), float(llr_clip), b, _ptr(syn), _ptr(dgamma),
                              float(dscale), None if dwp is None else _ptr(dwp), _ptr(lam), _ptr(dlam))
    if rc != 0:
        raise ValueError(f"oracle tangent failed with code {rc}")
    return lam, dlam


def minsum_trace(m, n, rows, cols, llr, t_iters, syn, precision="f32"):
    rows, cols = _coo(rows, cols)
    dt = np.float32 if precision == "f32" else np.float64
    llr = np.ascontiguousarray(llr, dtype=dt)
    syn = np.ascontiguousarray(syn, dtype=np.uint8)
    b = syn.shape[0]
    out = np.zeros((b, t_iters + 1, n), dt)
    rc = getattr(lib(), f"ro_minsum_trace_{precision}")(m, n, rows.size, _ptr(rows), _ptr(cols),
                                                        _ptr(llr), int(t_iters), b, _ptr(syn),
                                                        _ptr(out))
    if rc != 0:
        raise ValueError(f"oracle minsum failed with code {rc}")
    return out


def sumproduct_trace(m, n, rows, cols, llr, t_iters, syn):
    rows, cols = _coo(rows, cols)
    llr = np.ascontiguousarray(llr, dtype=np.float64)
    syn = np.ascontiguousarray(syn, dtype=np.uint8)
    b = syn.shape[0]
    out = np.zeros((b, t_iters + 1, n), np.float64)
    rc = lib().ro_sumproduct_trace(m, n, rows.size, _ptr(rows), _ptr(cols), _ptr(llr),
                                   int(t_iters), b, _ptr(syn), _ptr(out))
    if rc != 0:
        raise ValueError(f"oracle sum-product failed with code {rc}")
    return out


def decode_windowed(m, n, rows, cols, prior, params: dict, syn, band, first_round, t_commit, t_overlap,
                    threads=None):
    """Windowed Relay decoding over detector rounds (the overlapping windows of
    T_commit + T_overlap rounds of the caveat in Sec. 7.3), written from
    the definition with boolean masks:

      rounds R = ceil(m / band); window k covers detector rounds
      [s, e) = [k*Tc, min(k*Tc + Tc + To, R)) and decodes the faults whose
      first detector round lies in [s, e), on the rows of those rounds, with
      the residual syndrome sigma + H F (F = the faults committed so far);
      it commits the faults whose first round lies in [s, s + Tc), or every
      fault of the window if e = R (the last window).

    Columns may be in any order.  Returns corr [B, N] and per-window conv and
    iters [W, B]."""
    rows = np.asarray(rows, np.int64)
    cols = np.asarray(cols, np.int64)
    first_round = np.asarray(first_round, np.int64)
    syn = np.ascontiguousarray(syn, dtype=np.uint8)
    h = np.zeros((m, n), dtype=np.uint8)
    h[rows, cols] = 1
    n_rounds = -(-m // band)
    b = syn.shape[0]
    corr = np.zeros((b, n), np.uint8)
    convs, iters = [], []
    s = 0
    while True:
        e = min(s + t_commit + t_overlap, n_rounds)
        row_in = (np.arange(m) // band >= s) & (np.arange(m) // band < e)
        col_in = (first_round >= s) & (first_round < e)
        commit = col_in if e == n_rounds else (first_round >= s) & (first_round < s + t_commit)
        residual = (syn.astype(np.int64) + corr.astype(np.int64) @ h.T.astype(np.int64)) % 2
        ri, ci = np.nonzero(row_in)[0], np.nonzero(col_in)[0]
        sub = h[np.ix_(ri, ci)]
        sr, sc = np.nonzero(sub)
        out = decode(ri.size, ci.size, sr, sc, np.asarray(prior)[ci], params,
                     residual[:, ri].astype(np.uint8), threads=threads)
        keep = commit[ci]
        corr[:, ci[keep]] = out["corr"][:, keep]
        convs.append(out["conv"])
        iters.append(out["iters"])
        if e == n_rounds:
            break
        s += t_commit
    return {"corr": corr, "conv": np.stack(convs), "iters": np.stack(iters)}
