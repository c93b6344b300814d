"""ctypes wrapper of the C oracle (test infrastructure only).

The circuit is marshalled from ``workloads.circuit.Circuit`` into this
oracle's own flat tape; nothing here is shared with the GPU library.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from typing import Dict

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "symft_oracle.c")
LIB = os.path.join(HERE, "libsymft_oracle.so")

_KIND = {
    "H": 1, "S": 2, "S_DAG": 3, "X": 4, "Y": 5, "Z": 6, "CX": 7, "CZ": 8, "SWAP": 9,
    "R": 10, "M": 11, "MR": 12, "X_ERROR": 13, "DEPOLARIZE1": 14, "DEPOLARIZE2": 15,
    "PAULI_CHANNEL": 16, "ROT": 17, "MPP": 18, "FEEDBACK": 19, "DETECTOR": 20,
    "OBSERVABLE_INCLUDE": 21, "TICK": 22,
}
_LET = {"I": 0, "X": 1, "Y": 2, "Z": 3}


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (OpenMP over 64-shot words)."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + ".tmp"
        cmd = ["gcc", "-O2", "-std=gnu11", "-fPIC", "-shared", "-fopenmp", SRC, "-o", tmp, "-lm"]
        subprocess.check_call(cmd)
        os.replace(tmp, LIB)
    return LIB


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build(force=True)
        lib = C.CDLL(LIB)
        lib.orc_circuit_new.restype = C.c_void_p
        lib.orc_circuit_new.argtypes = [C.c_int, C.POINTER(C.c_int64), C.POINTER(C.c_double)]
        lib.orc_circuit_free.argtypes = [C.c_void_p]
        lib.orc_circuit_info.argtypes = [C.c_void_p, C.POINTER(C.c_int64)]
        lib.orc_channel_info.argtypes = [C.c_void_p] + [C.POINTER(C.c_int64)] * 2 + [C.POINTER(C.c_uint64)]
        lib.orc_sample.restype = C.c_int
        lib.orc_sample.argtypes = [C.c_void_p, C.c_uint64, C.c_uint64, C.c_uint64, C.POINTER(C.c_uint64),
                                   C.c_int64, C.c_int]
        lib.orc_trace.argtypes = [C.c_void_p, C.c_uint64, C.c_uint64, C.POINTER(C.c_int8), C.POINTER(C.c_uint8),
                                  C.POINTER(C.c_double), C.POINTER(C.c_int8), C.POINTER(C.c_int16),
                                  C.POINTER(C.c_int16)]
        lib.orc_noise_counts.argtypes = [C.c_void_p, C.c_uint64, C.c_uint64, C.c_uint64, C.POINTER(C.c_uint64),
                                         C.POINTER(C.c_uint64)]
        lib.orc_final_state.argtypes = [C.c_void_p, C.c_uint64, C.c_uint64, C.POINTER(C.c_int),
                                        C.POINTER(C.c_double), C.POINTER(C.c_uint64), C.POINTER(C.c_uint64),
                                        C.POINTER(C.c_int)]
        lib.orc_philox.argtypes = [C.POINTER(C.c_uint32), C.POINTER(C.c_uint32), C.POINTER(C.c_uint32)]
        lib.orc_rmeas_bit.restype = C.c_int
        lib.orc_rmeas_bit.argtypes = [C.c_uint64, C.c_uint64, C.c_uint64]
        lib.orc_active_u.restype = C.c_double
        lib.orc_active_u.argtypes = [C.c_uint64, C.c_uint64, C.c_uint64]
        lib.orc_gap_table.argtypes = [C.c_uint64, C.POINTER(C.c_uint64)]
        lib.orc_conjugate.argtypes = [C.c_int, C.c_int, C.c_int, C.POINTER(C.c_uint64), C.POINTER(C.c_uint64),
                                      C.POINTER(C.c_int)]
        _lib = lib
    return _lib


def _ptr(a: np.ndarray, ct):
    return a.ctypes.data_as(C.POINTER(ct))


def philox(ctr, key):
    lib = _load()
    c = np.asarray(ctr, dtype=np.uint32)
    k = np.asarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    lib.orc_philox(_ptr(c, C.c_uint32), _ptr(k, C.c_uint32), _ptr(out, C.c_uint32))
    return out


def rmeas_bit(seed: int, t: int, s: int) -> int:
    return _load().orc_rmeas_bit(seed, t, s)


def active_u(seed: int, t: int, s: int) -> float:
    return _load().orc_active_u(seed, t, s)


def gap_table(p32: int) -> np.ndarray:
    q = np.zeros(4097, dtype=np.uint64)
    _load().orc_gap_table(p32, _ptr(q, C.c_uint64))
    return q


def conjugate(gate: str, qa: int, qb: int, x: int, z: int, e: int):
    """U P U^dagger for P = i^e X^x Z^z on <= 64 qubits (bit masks); returns (x, z, e)."""
    xa = np.array([x], dtype=np.uint64)
    za = np.array([z], dtype=np.uint64)
    ea = C.c_int(e)
    _load().orc_conjugate(_KIND[gate], qa, qb, _ptr(xa, C.c_uint64), _ptr(za, C.c_uint64), C.byref(ea))
    return int(xa[0]), int(za[0]), ea.value


def _marshal(circ):
    tape = [len(circ.ops)]
    dargs = []
    for o in circ.ops:
        k = _KIND[o.name]
        if o.name in ("ROT", "MPP", "FEEDBACK"):
            qs = [q for q, _ in o.pauli]
            lets = [_LET[s] for _, s in o.pauli]
        else:
            qs = list(o.targets)
            lets = []
        tape += [k, len(qs)] + qs + [1 if o.negate else 0, len(lets)] + lets
        tape += [len(o.recs)] + list(o.recs) + [o.obs]
        tape += [len(o.branches)]
        for _, s in o.branches:
            if len(s) != len(qs):
                raise ValueError("PAULI_CHANNEL branch length must match its targets")
            tape += [_LET[ch] for ch in s]
        dargs.append(float(o.arg))
        dargs += [float(p) for p, _ in o.branches]
    return np.asarray(tape, dtype=np.int64), np.asarray(dargs + [0.0], dtype=np.float64)


class OracleCircuit:
    """One circuit loaded into the C oracle."""

    def __init__(self, circ):
        circ.validate()
        self.circuit = circ
        lib = _load()
        self._tape, self._dargs = _marshal(circ)
        self._h = lib.orc_circuit_new(circ.n_qubits, _ptr(self._tape, C.c_int64), _ptr(self._dargs, C.c_double))
        if not self._h:
            raise ValueError(f"oracle rejects the circuit: {circ.n_qubits} qubits (1 .. 4096) or a qubit out of range")
        info = np.zeros(8, dtype=np.int64)
        lib.orc_circuit_info(self._h, _ptr(info, C.c_int64))
        self.n_meas, self.n_rec, self.n_det, self.n_obs, self.n_chan, self.n_cls = (int(v) for v in info[:6])
        self.n_rows = self.n_rec + self.n_det + self.n_obs

    def __del__(self):
        h = getattr(self, "_h", None)
        if h and _lib is not None:
            _lib.orc_circuit_free(h)
            self._h = None

    def sample(self, seed: int, shots: int, shot_begin: int = 0, threads: int = 0) -> np.ndarray:
        """Records [rows, ceil(shots/64)] uint64, bit s%64 of word s//64 (relative to shot_begin)."""
        if shot_begin % 64:
            raise ValueError("shot_begin must be a multiple of 64")
        words = (shots + 63) // 64
        out = np.zeros((self.n_rows, max(words, 1)), dtype=np.uint64)
        if shots == 0:
            return out[:, :0]
        rc = _load().orc_sample(self._h, seed, shot_begin, shots, _ptr(out, C.c_uint64), out.shape[1], threads)
        if rc != 0:
            raise RuntimeError("oracle sample failed")
        return out

    def sample_words(self, seed: int, words, threads: int = 0) -> np.ndarray:
        """Records for a list of 64-shot words: [rows, len(words)]."""
        cols = [self.sample(seed, 64, shot_begin=64 * int(w), threads=threads)[:, 0] for w in words]
        return np.stack(cols, axis=1) if cols else np.zeros((self.n_rows, 0), dtype=np.uint64)

    def trace(self, seed: int, shot: int) -> Dict[str, np.ndarray]:
        lib = _load()
        n_ops = len(self.circuit.ops)
        kind = np.zeros(max(self.n_meas, 1), dtype=np.int8)
        m = np.zeros(max(self.n_meas, 1), dtype=np.uint8)
        p0 = np.zeros(max(self.n_meas, 1), dtype=np.float64)
        rot = np.zeros(max(n_ops, 1), dtype=np.int8)
        kk = np.zeros(max(n_ops, 1), dtype=np.int16)
        fired = np.zeros(max(self.n_chan, 1), dtype=np.int16)
        lib.orc_trace(self._h, seed, shot, _ptr(kind, C.c_int8), _ptr(m, C.c_uint8), _ptr(p0, C.c_double),
                      _ptr(rot, C.c_int8), _ptr(kk, C.c_int16), _ptr(fired, C.c_int16))
        return {
            "meas_kind": kind[: self.n_meas], "m": m[: self.n_meas], "p0": p0[: self.n_meas],
            "rot_kind": rot[:n_ops], "k": kk[:n_ops], "fired": fired[: self.n_chan],
        }

    def final_state(self, seed: int, shot: int) -> Dict[str, np.ndarray]:
        """Active vector alpha (complex, 2^k) after the last op, and the signed
        tableau: rows 0..n-1 Zbar_j, n..2n-1 Xbar_j as integer bit masks x, z
        and phase exponents e (row = i^e X^x Z^z)."""
        lib = _load()
        n = self.circuit.n_qubits
        W = (n + 63) // 64
        k = C.c_int(0)
        lib.orc_final_state(self._h, seed, shot, C.byref(k), None, None, None, None)
        amp = np.zeros(2 << k.value, dtype=np.float64)
        tx = np.zeros(2 * n * W, dtype=np.uint64)
        tz = np.zeros(2 * n * W, dtype=np.uint64)
        te = np.zeros(2 * n, dtype=np.int32)
        lib.orc_final_state(self._h, seed, shot, C.byref(k), _ptr(amp, C.c_double), _ptr(tx, C.c_uint64),
                            _ptr(tz, C.c_uint64), _ptr(te, C.c_int))

        def rows(t):
            return [sum(int(t[r * W + i]) << (64 * i) for i in range(W)) for r in range(2 * n)]

        return {"k": k.value, "alpha": amp[0::2] + 1j * amp[1::2], "x": rows(tx), "z": rows(tz), "e": te}

    def channel_info(self):
        lib = _load()
        cls = np.zeros(max(self.n_chan, 1), dtype=np.int64)
        rank = np.zeros(max(self.n_chan, 1), dtype=np.int64)
        p32 = np.zeros(max(self.n_chan, 1), dtype=np.uint64)
        lib.orc_channel_info(self._h, _ptr(cls, C.c_int64), _ptr(rank, C.c_int64), _ptr(p32, C.c_uint64))
        return cls[: self.n_chan], rank[: self.n_chan], p32[: self.n_chan]

    def noise_counts(self, seed: int, word_begin: int, n_words: int):
        counts = np.zeros(max(self.n_chan, 1), dtype=np.uint64)
        br = np.zeros(max(self.n_chan, 1) * 16, dtype=np.uint64)
        _load().orc_noise_counts(self._h, seed, word_begin, n_words, _ptr(counts, C.c_uint64), _ptr(br, C.c_uint64))
        return counts[: self.n_chan], br.reshape(-1, 16)[: self.n_chan]

    def k_trajectory(self) -> np.ndarray:
        """Active width after every op (shot-independent)."""
        return self.trace(0, 0)["k"]
