"""Plain circuit descriptions shared by the oracle and the GPU library's binding.

This module holds no arithmetic of the sampling method: an operation is a
record of its name, targets and arguments, in the vocabulary of the paper's
noisy circuit model (Sec. 2): Clifford gates, Pauli rotations
R_P(theta) = exp(-i theta P / 2), Pauli-product measurements (outcome 0 for
the +1 eigenvalue), stochastic Pauli channels and Pauli feedback controlled
by the parity of earlier measurement records.  Resets and detector /
observable annotations are included because the benchmark circuits use them.

Records are referenced by absolute index in circuit order (visible
measurements only); a reset's internal measurement is not a record.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Sequence, Tuple

GATES_1Q = ("H", "S", "S_DAG", "X", "Y", "Z")
GATES_2Q = ("CX", "CZ", "SWAP")
NOISE = ("X_ERROR", "DEPOLARIZE1", "DEPOLARIZE2", "PAULI_CHANNEL")
MEAS_Z = ("R", "M", "MR")
PAULI_OPS = ("ROT", "MPP", "FEEDBACK")
ANNOT = ("DETECTOR", "OBSERVABLE_INCLUDE", "TICK")
ALL = GATES_1Q + GATES_2Q + NOISE + MEAS_Z + PAULI_OPS + ANNOT

LETTER = {"X": 1, "Y": 2, "Z": 3}


@dataclass(frozen=True)
class Op:
    name: str
    targets: Tuple[int, ...] = ()
    # ROT / MPP / FEEDBACK: the Pauli as ((qubit, letter), ...) with letter in "XYZ"
    pauli: Tuple[Tuple[int, str], ...] = ()
    negate: bool = False
    # ROT: angle theta; X_ERROR / DEPOLARIZE1 / DEPOLARIZE2: probability p;
    # M / MR / MPP: readout-flip probability (the recorded bit is complemented)
    arg: float = 0.0
    # FEEDBACK / DETECTOR / OBSERVABLE_INCLUDE: absolute record ids
    recs: Tuple[int, ...] = ()
    obs: int = 0
    # PAULI_CHANNEL on `targets`: ((prob, "letters over targets, I/X/Y/Z"), ...)
    branches: Tuple[Tuple[float, str], ...] = ()


@dataclass
class Circuit:
    n_qubits: int
    ops: List[Op] = field(default_factory=list)

    # -- builders -------------------------------------------------------
    def append(self, name: str, targets: Sequence[int] = (), **kw) -> "Circuit":
        if name not in ALL:
            raise ValueError(f"unknown op {name}")
        self.ops.append(Op(name, tuple(int(t) for t in targets), **kw))
        return self

    def rot(self, pauli: Sequence[Tuple[int, str]], theta: float, negate: bool = False) -> "Circuit":
        self.ops.append(Op("ROT", pauli=tuple((int(q), s) for q, s in pauli), arg=float(theta), negate=negate))
        return self

    def mpp(self, pauli: Sequence[Tuple[int, str]], negate: bool = False, p_flip: float = 0.0) -> int:
        self.ops.append(Op("MPP", pauli=tuple((int(q), s) for q, s in pauli), negate=negate, arg=float(p_flip)))
        return self.num_records - 1

    def feedback(self, pauli: Sequence[Tuple[int, str]], recs: Sequence[int]) -> "Circuit":
        self.ops.append(Op("FEEDBACK", pauli=tuple((int(q), s) for q, s in pauli), recs=tuple(int(r) for r in recs)))
        return self

    def detector(self, recs: Sequence[int]) -> "Circuit":
        self.ops.append(Op("DETECTOR", recs=tuple(int(r) for r in recs)))
        return self

    def observable(self, obs: int, recs: Sequence[int]) -> "Circuit":
        self.ops.append(Op("OBSERVABLE_INCLUDE", recs=tuple(int(r) for r in recs), obs=int(obs)))
        return self

    # -- counts (plain bookkeeping) --------------------------------------
    @property
    def num_records(self) -> int:
        n = 0
        for o in self.ops:
            if o.name in ("M", "MR"):
                n += len(o.targets)
            elif o.name == "MPP":
                n += 1
        return n

    @property
    def num_measurements(self) -> int:
        """All measurements, including the unrecorded ones inside resets."""
        n = 0
        for o in self.ops:
            if o.name in MEAS_Z:
                n += len(o.targets)
            elif o.name == "MPP":
                n += 1
        return n

    @property
    def num_detectors(self) -> int:
        return sum(1 for o in self.ops if o.name == "DETECTOR")

    @property
    def num_observables(self) -> int:
        ids = [o.obs for o in self.ops if o.name == "OBSERVABLE_INCLUDE"]
        return (max(ids) + 1) if ids else 0

    @property
    def num_rows(self) -> int:
        return self.num_records + self.num_detectors + self.num_observables

    def validate(self) -> None:
        """Structural checks only (qubit ranges, record causality)."""
        recs = 0
        for o in self.ops:
            for q in o.targets:
                if not 0 <= q < self.n_qubits:
                    raise ValueError(f"{o.name}: qubit {q} out of range")
            for q, s in o.pauli:
                if not 0 <= q < self.n_qubits or s not in LETTER:
                    raise ValueError(f"{o.name}: bad Pauli term {(q, s)}")
            for r in o.recs:
                if not 0 <= r < recs:
                    raise ValueError(f"{o.name}: record {r} not yet measured")
            if o.name in ("M", "MR"):
                recs += len(o.targets)
            elif o.name == "MPP":
                recs += 1
