"""Python binding of the SymFT MI355X sampling library (libsymft.so).

Argument marshalling only: every step of the sampling path runs in the HIP
kernels behind the C ABI declared in include/symft.h.  PyTorch supplies
device memory and the current stream.  There is no CPU fallback: if the
library is missing the import of this module fails.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Dict, List, Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "libsymft.so")

if not os.path.exists(LIB):
    raise ImportError(f"{LIB} is not built; run `python paper_2607_28600_amd/build.py`")

# PyTorch ships its own HIP runtime under the same soname.  Loading it first
# makes the library bind to that one runtime; loaded the other way round, the
# process would hold two HIP runtimes, and the library's would find no device.
import torch  # noqa: E402,F401

_lib = C.CDLL(LIB)

OK = 0
ERRORS = {-1: "EINVAL", -2: "ENONHERMITIAN", -3: "EACAUSAL", -4: "EPROB", -5: "ECAPACITY", -6: "ENOMEM", -7: "EHIP"}

OP = {
    "H": 1, "S": 2, "S_DAG": 3, "X": 4, "Y": 5, "Z": 6, "CX": 7, "CZ": 8, "SWAP": 9,
    "R": 10, "M": 11, "MR": 12, "X_ERROR": 13, "DEPOLARIZE1": 14, "DEPOLARIZE2": 15,
    "PAULI_CHANNEL": 16, "ROT": 17, "MPP": 18, "FEEDBACK": 19, "DETECTOR": 20,
    "OBSERVABLE_INCLUDE": 21, "TICK": 22,
}
LETTER = {"I": 0, "X": 1, "Y": 2, "Z": 3}
INSTR_NAMES = {1: "PromoteRot", 2: "ActiveDiagRot", 3: "ActivePairRot", 4: "RandomMeas", 5: "DetMeas",
               6: "ActiveDiagMeas", 7: "ActivePairMeas"}


class symft_op(C.Structure):
    _fields_ = [
        ("kind", C.c_uint32), ("n", C.c_uint32), ("qubits", C.POINTER(C.c_uint32)),
        ("paulis", C.POINTER(C.c_uint8)), ("negate", C.c_uint32), ("arg", C.c_double),
        ("n_branches", C.c_uint32), ("probs", C.POINTER(C.c_double)), ("branch_paulis", C.POINTER(C.c_uint8)),
        ("n_recs", C.c_uint32), ("recs", C.POINTER(C.c_int64)), ("obs_id", C.c_uint32),
    ]


class symft_info(C.Structure):
    _fields_ = [
        ("n_qubits", C.c_uint32), ("k_max", C.c_uint32), ("n_ops", C.c_uint64), ("n_measurements", C.c_uint64),
        ("n_records", C.c_uint64), ("n_detectors", C.c_uint64), ("n_observables", C.c_uint64),
        ("n_rows", C.c_uint64), ("n_instr", C.c_uint64 * 8), ("n_channels", C.c_uint64),
        ("n_classes", C.c_uint64), ("n_noise_symbols", C.c_uint64), ("expr_noise_nnz", C.c_uint64),
        ("expr_meas_nnz", C.c_uint64), ("dense_flops_per_shot", C.c_double), ("dense_bytes_per_shot", C.c_double),
        ("frame_steps", C.c_uint64), ("frame_noise_steps", C.c_uint64), ("frame_slots", C.c_uint64),
        ("frame_max_level", C.c_uint64), ("frame_pushes", C.c_uint64), ("frame_noise_consumers", C.c_uint64),
        ("rotations_removed", C.c_uint64), ("frame_kernel", C.c_uint64), ("frame_wave_batches", C.c_uint64),
        ("frame_wave_flushes", C.c_uint64), ("product_selected", C.c_uint64), ("product_components", C.c_uint64),
        ("product_merges", C.c_uint64), ("product_vector_amplitudes", C.c_uint64),
        ("product_flops_per_shot", C.c_double), ("frame_small_words", C.c_uint64),
    ]


class symft_compile_opts(C.Structure):
    _fields_ = [("simplify", C.c_uint32), ("components", C.c_uint32), ("reserved", C.c_uint32 * 2)]


class symft_sample_opts(C.Structure):
    _fields_ = [("shot_offset", C.c_uint64), ("precision", C.c_uint32), ("sections", C.c_uint32),
                ("row_stride_words", C.c_uint64), ("frame_entry_cap", C.c_uint32), ("frame_tile_words", C.c_uint32),
                ("frame_kernel", C.c_uint32), ("active_kernel", C.c_uint32)]


class symft_count_opts(C.Structure):
    _fields_ = [("shot_offset", C.c_uint64), ("precision", C.c_uint32), ("n_post", C.c_uint32),
                ("post", C.c_void_p), ("obs_expected", C.c_void_p), ("threads_per_shot", C.c_uint32),
                ("mode", C.c_uint32), ("frame_kernel", C.c_uint32)]


_lib.symft_compile.restype = C.c_int32
_lib.symft_compile.argtypes = [C.c_uint32, C.POINTER(symft_op), C.c_size_t, C.c_void_p, C.POINTER(C.c_void_p)]
_lib.symft_program_info.restype = C.c_int32
_lib.symft_program_info.argtypes = [C.c_void_p, C.POINTER(symft_info)]
_lib.symft_program_plan.restype = C.c_int32
_lib.symft_program_plan.argtypes = [C.c_void_p, C.POINTER(C.c_int16), C.POINTER(C.c_int8), C.POINTER(C.c_int8)]
_lib.symft_sample.restype = C.c_int32
_lib.symft_sample.argtypes = [C.c_void_p, C.c_uint64, C.c_uint64, C.c_void_p, C.c_void_p]
_lib.symft_sample_ex.restype = C.c_int32
_lib.symft_sample_ex.argtypes = [C.c_void_p, C.POINTER(symft_sample_opts), C.c_uint64, C.c_uint64, C.c_void_p,
                                 C.c_void_p]
_lib.symft_sample_noalloc.restype = C.c_int32
_lib.symft_sample_noalloc.argtypes = [C.c_void_p, C.POINTER(symft_sample_opts), C.c_uint64, C.c_uint64, C.c_void_p,
                                      C.c_void_p]
_lib.symft_sample_counts.restype = C.c_int32
_lib.symft_sample_counts.argtypes = [C.c_void_p, C.POINTER(symft_count_opts), C.c_uint64, C.c_uint64, C.c_void_p,
                                     C.c_void_p, C.c_void_p]
_lib.symft_autotune_counts.restype = C.c_int32
_lib.symft_autotune_counts.argtypes = [C.c_void_p, C.POINTER(symft_count_opts), C.POINTER(C.c_uint32)]
_lib.symft_sample_batch.restype = C.c_int32
_lib.symft_sample_batch.argtypes = [C.POINTER(C.c_void_p), C.POINTER(C.c_uint64), C.POINTER(C.c_uint64),
                                    C.POINTER(C.c_void_p), C.c_size_t, C.c_uint32, C.c_uint32, C.c_void_p]
_lib.symft_sample_counts_batch.restype = C.c_int32
_lib.symft_sample_counts_batch.argtypes = [C.POINTER(C.c_void_p), C.POINTER(C.c_uint64), C.POINTER(C.c_uint64),
                                           C.POINTER(symft_count_opts), C.POINTER(C.c_void_p), C.c_void_p, C.c_size_t,
                                           C.c_uint32, C.c_uint32, C.c_void_p]
_lib.symft_autotune.restype = C.c_int32
_lib.symft_autotune.argtypes = [C.c_void_p, C.c_uint32, C.POINTER(C.c_uint32)]
_lib.symft_gap_check.restype = C.c_int32
_lib.symft_gap_check.argtypes = [C.c_uint64, C.c_void_p, C.c_void_p, C.c_uint64, C.c_void_p]
_lib.symft_probe.restype = C.c_int32
_lib.symft_probe.argtypes = [C.c_void_p, C.c_uint64, C.c_uint32, C.c_uint64, C.c_uint32, C.POINTER(C.c_double)]
_lib.symft_probe_amplitudes.restype = C.c_int32
_lib.symft_probe_amplitudes.argtypes = [C.c_void_p, C.c_uint64, C.c_uint32, C.c_uint64, C.c_uint32, C.c_void_p,
                                        C.POINTER(C.c_uint32)]
_lib.symft_program_export.restype = C.c_int32
_lib.symft_program_export.argtypes = [C.c_void_p, C.POINTER(C.c_uint64), C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                      C.c_void_p, C.c_void_p]
_lib.symft_program_free.argtypes = [C.c_void_p]
_lib.symft_last_error.restype = C.c_char_p

EXPORTED = ["symft_compile", "symft_program_info", "symft_program_plan", "symft_program_export",
            "symft_sample", "symft_sample_ex", "symft_sample_counts", "symft_autotune_counts",
            "symft_sample_noalloc", "symft_sample_batch", "symft_sample_counts_batch", "symft_autotune", "symft_probe", "symft_probe_amplitudes", "symft_gap_check", "symft_program_free",
            "symft_last_error"]


class SymftError(RuntimeError):
    def __init__(self, code: int, what: str):
        msg = _lib.symft_last_error().decode(errors="replace")
        super().__init__(f"{what}: {ERRORS.get(code, code)}: {msg}")
        self.code = code


def _check(rc: int, what: str):
    if rc != OK:
        raise SymftError(rc, what)


def _marshal(circ):
    """Circuit -> (symft_op array, keep-alive list)."""
    keep: List = []
    arr = (symft_op * max(1, len(circ.ops)))()
    for i, o in enumerate(circ.ops):
        s = arr[i]
        s.kind = OP[o.name]
        if o.name in ("ROT", "MPP", "FEEDBACK"):
            qs = [q for q, _ in o.pauli]
            lets = [LETTER[l] for _, l in o.pauli]
        else:
            qs = list(o.targets)
            lets = []
        qa = (C.c_uint32 * max(1, len(qs)))(*qs)
        keep.append(qa)
        s.n = len(qs)
        s.qubits = C.cast(qa, C.POINTER(C.c_uint32))
        if lets:
            la = (C.c_uint8 * len(lets))(*lets)
            keep.append(la)
            s.paulis = C.cast(la, C.POINTER(C.c_uint8))
        s.negate = 1 if o.negate else 0
        s.arg = float(o.arg)
        if o.branches:
            pr = (C.c_double * len(o.branches))(*[float(p) for p, _ in o.branches])
            bl = (C.c_uint8 * (len(o.branches) * len(qs)))(*[LETTER[ch] for _, st in o.branches for ch in st])
            keep += [pr, bl]
            s.n_branches = len(o.branches)
            s.probs = C.cast(pr, C.POINTER(C.c_double))
            s.branch_paulis = C.cast(bl, C.POINTER(C.c_uint8))
        if o.recs:
            ra = (C.c_int64 * len(o.recs))(*o.recs)
            keep.append(ra)
            s.n_recs = len(o.recs)
            s.recs = C.cast(ra, C.POINTER(C.c_int64))
        s.obs_id = o.obs
    return arr, keep


class Program:
    """A compiled SymFT sampling program (owned by the C library)."""

    def __init__(self, circ, simplify: bool = False, components: str = "auto"):
        """simplify: fuse and cancel rotations with the same Pauli body across ops on other qubits
        (symft_compile_opts.simplify).  components: "auto", "off" or "on" (symft_compile_opts.components,
        the product-component representation)."""
        arr, keep = _marshal(circ)
        h = C.c_void_p()
        opts = symft_compile_opts(simplify=1 if simplify else 0, components={"auto": 0, "off": 1, "on": 2}[components])
        _check(_lib.symft_compile(circ.n_qubits, arr, len(circ.ops), C.cast(C.pointer(opts), C.c_void_p), C.byref(h)),
               "symft_compile")
        self._h = h
        self.n_ops = len(circ.ops)
        info = self.info()
        self.n_rows = int(info["n_rows"])
        self.n_meas = int(info["n_measurements"])
        self.n_rec = int(info["n_records"])
        self.n_det = int(info["n_detectors"])
        self.n_obs = int(info["n_observables"])
        self.k_max = int(info["k_max"])

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value and _lib is not None:  # the library may be gone at interpreter exit
            _lib.symft_program_free(h)
            self._h = None

    @property
    def handle(self):
        return self._h

    def info(self) -> Dict:
        s = symft_info()
        _check(_lib.symft_program_info(self._h, C.byref(s)), "symft_program_info")
        d = {name: getattr(s, name) for name, _ in s._fields_}
        d["n_instr"] = {INSTR_NAMES[i]: int(s.n_instr[i]) for i in range(1, 8)}
        return d

    def plan(self):
        k = np.zeros(max(1, self.n_ops), dtype=np.int16)
        mk = np.zeros(max(1, self.n_meas), dtype=np.int8)
        rk = np.zeros(max(1, self.n_ops), dtype=np.int8)
        _check(_lib.symft_program_plan(self._h, k.ctypes.data_as(C.POINTER(C.c_int16)),
                                       mk.ctypes.data_as(C.POINTER(C.c_int8)),
                                       rk.ctypes.data_as(C.POINTER(C.c_int8))), "symft_program_plan")
        return {"k": k[: self.n_ops], "meas_kind": mk[: self.n_meas], "rot_kind": rk[: self.n_ops]}

    def export(self) -> Dict[str, np.ndarray]:
        """The compiled instruction stream and channel symbol masks (host copy)."""
        cnt = np.zeros(5, dtype=np.uint64)
        _check(_lib.symft_program_export(self._h, cnt.ctypes.data_as(C.POINTER(C.c_uint64)), None, None, None,
                                         None, None, None), "symft_program_export")
        ni, nn, nm, nc, nb = (int(v) for v in cnt)
        instr = np.zeros((max(ni, 1), 13), dtype=np.int64)
        theta = np.zeros(max(ni, 1), dtype=np.float64)
        noise = np.zeros(max(nn, 1), dtype=np.uint32)
        meas = np.zeros(max(nm, 1), dtype=np.uint32)
        chan = np.zeros((max(nc, 1), 4), dtype=np.int64)
        bm = np.zeros(max(nb, 1), dtype=np.uint32)
        _check(_lib.symft_program_export(self._h, cnt.ctypes.data_as(C.POINTER(C.c_uint64)), instr.ctypes.data,
                                         theta.ctypes.data, noise.ctypes.data, meas.ctypes.data, chan.ctypes.data,
                                         bm.ctypes.data), "symft_program_export")
        return {"instr": instr[:ni], "theta": theta[:ni], "noise": noise[:nn], "meas": meas[:nm],
                "chan": chan[:nc], "bmask": bm[:nb]}

    # -- sampling (device) ------------------------------------------------
    def sample_into(self, out, shots: int, seed: int, shot_offset: int = 0, precision: str = "fp64",
                    sections: int = 0, row_stride_words: int = 0, stream=None, frame_entry_cap: int = 0,
                    frame_tile_words: int = 0, frame_kernel: int = 0, active_kernel: int = 0) -> None:
        """out: a device tensor / pointer holding n_rows x stride uint64 words."""
        import torch
        ptr = out.data_ptr() if hasattr(out, "data_ptr") else int(out)
        if stream is None:
            stream = torch.cuda.current_stream().cuda_stream
        o = symft_sample_opts(shot_offset, 0 if precision == "fp64" else 1, sections, row_stride_words,
                              frame_entry_cap, frame_tile_words, frame_kernel, active_kernel)
        _check(_lib.symft_sample_ex(self._h, C.byref(o), shots, seed, C.c_void_p(ptr), C.c_void_p(stream)),
               "symft_sample_ex")

    def sample_noalloc_into(self, out, shots: int, seed: int, shot_offset: int = 0, precision: str = "fp64",
                            sections: int = 0, row_stride_words: int = 0, stream=None, frame_kernel: int = 0,
                            active_kernel: int = 0) -> None:
        """symft_sample_noalloc: as sample_into, with the kernels' scratch in the library's fixed device array
        (the program must have been sampled once on this device)."""
        import torch
        ptr = out.data_ptr() if hasattr(out, "data_ptr") else int(out)
        if stream is None:
            stream = torch.cuda.current_stream().cuda_stream
        o = symft_sample_opts(shot_offset, 0 if precision == "fp64" else 1, sections, row_stride_words, 0, 0,
                              frame_kernel, active_kernel)
        _check(_lib.symft_sample_noalloc(self._h, C.byref(o), shots, seed, C.c_void_p(ptr), C.c_void_p(stream)),
               "symft_sample_noalloc")

    def sample(self, shots: int, seed: int, shot_offset: int = 0, precision: str = "fp64", device="cuda",
               frame_entry_cap: int = 0, frame_tile_words: int = 0, frame_kernel: int = 0, active_kernel: int = 0):
        """Returns a [n_rows, ceil(shots/64)] int64 tensor on the GPU (uint64 bit patterns)."""
        import torch
        words = (shots + 63) // 64
        out = torch.zeros((max(self.n_rows, 1), max(words, 1)), dtype=torch.int64, device=device)
        if shots:
            self.sample_into(out, shots, seed, shot_offset=shot_offset, precision=precision,
                             frame_entry_cap=frame_entry_cap, frame_tile_words=frame_tile_words,
                             frame_kernel=frame_kernel, active_kernel=active_kernel)
        return out[: self.n_rows, :words]

    def _count_opts(self, post, obs_expected, shot_offset, precision, threads_per_shot, mode=0, frame_kernel=0):
        post = np.ascontiguousarray(np.asarray(post, dtype=np.uint32).reshape(-1))
        exp = None
        if obs_expected is not None:
            exp = np.ascontiguousarray(np.asarray(obs_expected, dtype=np.uint8).reshape(-1))
            if exp.size != self.n_obs:
                raise ValueError("obs_expected needs one value per observable")
        o = symft_count_opts(shot_offset, 0 if precision == "fp64" else 1, post.size,
                             post.ctypes.data if post.size else None, exp.ctypes.data if exp is not None else None,
                             threads_per_shot, mode, frame_kernel)
        return o, (post, exp)  # the arrays must outlive the call

    def sample_counts_into(self, flags, counts, shots: int, seed: int, post=(), obs_expected=None,
                           shot_offset: int = 0, precision: str = "fp64", stream=None,
                           threads_per_shot: int = 0, mode: int = 0, frame_kernel: int = 0) -> None:
        """Aggregate counts: flags (device [2, ceil(shots/64)] words, or None) receives the discarded and
        logical-error flags; counts (device [2] uint64, or None) has the two totals added to it."""
        import torch
        o, keep = self._count_opts(post, obs_expected, shot_offset, precision, threads_per_shot, mode, frame_kernel)
        if stream is None:
            stream = torch.cuda.current_stream().cuda_stream
        fp = None if flags is None else (flags.data_ptr() if hasattr(flags, "data_ptr") else int(flags))
        cp = None if counts is None else (counts.data_ptr() if hasattr(counts, "data_ptr") else int(counts))
        _check(_lib.symft_sample_counts(self._h, C.byref(o), shots, seed, C.c_void_p(fp), C.c_void_p(cp),
                                        C.c_void_p(stream)), "symft_sample_counts")

    def sample_counts(self, shots: int, seed: int, post=(), obs_expected=None, shot_offset: int = 0,
                      precision: str = "fp64", device="cuda", threads_per_shot: int = 0, mode: int = 0,
                      frame_kernel: int = 0):
        """Returns (flags [2, ceil(shots/64)] int64 tensor, counts [2] int64 tensor) on the GPU."""
        import torch
        words = (shots + 63) // 64
        flags = torch.zeros((2, max(words, 1)), dtype=torch.int64, device=device)
        counts = torch.zeros(2, dtype=torch.int64, device=device)
        self.sample_counts_into(flags, counts, shots, seed, post=post, obs_expected=obs_expected,
                                shot_offset=shot_offset, precision=precision, threads_per_shot=threads_per_shot,
                                mode=mode, frame_kernel=frame_kernel)
        return flags[:, :words], counts

    def autotune_counts(self, post=(), obs_expected=None, precision: str = "fp32") -> int:
        """Run the aggregate-count autotuner for this program, postselection set and precision."""
        o, keep = self._count_opts(post, obs_expected, 0, precision, 0)
        v = C.c_uint32(0)
        _check(_lib.symft_autotune_counts(self._h, C.byref(o), C.byref(v)), "symft_autotune_counts")
        return int(v.value)

    def autotune(self, precision: str = "fp32") -> int:
        """Run the autotuner for this program's (k_max, precision); returns threads per shot."""
        v = C.c_uint32(0)
        _check(_lib.symft_autotune(self._h, 0 if precision == "fp64" else 1, C.byref(v)), "symft_autotune")
        return int(v.value)

    def probe(self, shot_begin: int, n_shots: int, seed: int, precision: str = "fp64") -> np.ndarray:
        """Pr(m = 0) of every measurement of shots [shot_begin, +n_shots) from the GPU kernels."""
        p0 = np.zeros((n_shots, max(1, self.n_meas)), dtype=np.float64)
        _check(_lib.symft_probe(self._h, shot_begin, n_shots, seed, 0 if precision == "fp64" else 1,
                                p0.ctypes.data_as(C.POINTER(C.c_double))), "symft_probe")
        return p0[:, : self.n_meas]


def _probe_amplitudes(prog, shot_begin: int, n_shots: int, seed: int, precision: str = "fp64") -> np.ndarray:
    """Final active vector of shots [shot_begin, +n_shots) from the GPU kernels: [n_shots, 2^k_end] complex128."""
    k = C.c_uint32(0)
    _check(_lib.symft_probe_amplitudes(prog._h, shot_begin, 0, seed, 0, None, C.byref(k)), "symft_probe_amplitudes")
    amp = np.zeros((n_shots, (1 << k.value) * 2), dtype=np.float64)
    _check(_lib.symft_probe_amplitudes(prog._h, shot_begin, n_shots, seed, 0 if precision == "fp64" else 1,
                                       amp.ctypes.data, C.byref(k)), "symft_probe_amplitudes")
    return amp[:, 0::2] + 1j * amp[:, 1::2]


Program.probe_amplitudes = _probe_amplitudes


def compile(circ) -> Program:  # noqa: A001 - mirrors symft_compile
    return Program(circ)


def gap_check(p32: int, v, stream=None):
    """Geometric gaps of the noise draw contract for uint32 draws `v` (a CUDA int32 tensor
    holding the bit patterns), decided as the sampling kernels decide them."""
    import torch
    g = torch.empty_like(v)
    if stream is None:
        stream = torch.cuda.current_stream().cuda_stream
    _check(_lib.symft_gap_check(int(p32), C.c_void_p(v.data_ptr()), C.c_void_p(g.data_ptr()), v.numel(),
                                C.c_void_p(stream)), "symft_gap_check")
    return g


def sample_batch(programs: Sequence[Program], shots: Sequence[int], seeds: Sequence[int], outs,
                 precision: str = "fp32", graph: bool = True, stream=None) -> None:
    import torch
    n = len(programs)
    hs = (C.c_void_p * n)(*[p.handle.value for p in programs])
    sh = (C.c_uint64 * n)(*[int(s) for s in shots])
    sd = (C.c_uint64 * n)(*[int(s) for s in seeds])
    op = (C.c_void_p * n)(*[o.data_ptr() for o in outs])
    if stream is None:
        stream = torch.cuda.current_stream().cuda_stream
    _check(_lib.symft_sample_batch(hs, sh, sd, op, n, 0 if precision == "fp64" else 1, 1 if graph else 0,
                                   C.c_void_p(stream)), "symft_sample_batch")


def sample_counts_batch(programs: Sequence[Program], shots: Sequence[int], seeds: Sequence[int], posts, flags,
                        counts, obs_expected=None, shot_offsets=None, precision: str = "fp32", graph: bool = False,
                        stream=None) -> None:
    """symft_sample_counts_batch: posts[i] (detector indices) and obs_expected[i] (or None) per program; flags
    (list of device [2, ceil(shots[i]/64)] tensors or None) and counts (device [2n] int64 tensor or None)."""
    import torch
    n = len(programs)
    hs = (C.c_void_p * n)(*[p.handle.value for p in programs])
    sh = (C.c_uint64 * n)(*[int(s) for s in shots])
    sd = (C.c_uint64 * n)(*[int(s) for s in seeds])
    opts = (symft_count_opts * n)()
    keep = []
    for i, p in enumerate(programs):
        o, k = p._count_opts(posts[i], None if obs_expected is None else obs_expected[i],
                             0 if shot_offsets is None else int(shot_offsets[i]), precision, 0)
        opts[i] = o
        keep.append(k)
    fp = None
    if flags is not None:
        fp = (C.c_void_p * n)(*[None if f is None else f.data_ptr() for f in flags])
    cp = None if counts is None else counts.data_ptr()
    if stream is None:
        stream = torch.cuda.current_stream().cuda_stream
    _check(_lib.symft_sample_counts_batch(hs, sh, sd, opts, fp, C.c_void_p(cp), n, 0 if precision == "fp64" else 1,
                                          1 if graph else 0, C.c_void_p(stream)), "symft_sample_counts_batch")


def bits_to_numpy(t) -> np.ndarray:
    """int64 device tensor -> uint64 numpy array."""
    return t.cpu().numpy().view(np.uint64)
