"""FP64 oracle of the approximate (SDRP) mode of Sec. III (test infrastructure).

The ket is kept as a tensor product of kets on disjoint qubit sets (Sec. II-A,
factorized form). A subsystem is (ordered qubit list, complex128 amplitudes);
list position t is bit t of the subsystem's index.

Steps, in the paper's order (Sec. III-A):
  1. Bloch vector of qubit q from the ket: r = (<X>, <Y>, <Z>) of rho_q.
  2. epsilon = (1 - |r|)/2; no rounding when epsilon > p/2.
  3./4. Rotate r to the |0> pole, post-select |0>, rotate back. This is the
     projection of q onto the dominant eigenvector phi of rho_q, leaving the
     normalized remainder <phi|_q psi on the other qubits (Eq. sdrp).
Every rounding multiplies the fidelity estimate by (1 - epsilon) (Sec. III-B,
Eq. fid_model).

Readings (each also listed with the design notes):
  * Eq. schmidt prints the leading coefficient as (1 - sqrt(eps)); it is read
    as sqrt(1 - eps), the normalized form consistent with eps = (1-|r|)/2 and
    with the per-rounding fidelity 1 - eps.
  * The rounding condition is the inclusive eps <= p/2 of Eq. sdrp (not the
    eps_j <= p written in Sec. III-B, nor the strict inequality of Fig. 2's
    caption). Sec. III-A treats eps as zero to within rounding, which adds a
    tolerance tau: round when eps <= p/2 + tau (tau = 1e-12 here).
  * When and in what order the test runs is not stated (Table I says only that
    the state is decomposed both ahead of need and on demand). Only a two-qubit gate's operands and the remaining
    members of a subsystem that just lost a qubit can have a changed reduced
    state, so after every multi-qubit gate those qubits are marked dirty and
    the lowest-numbered dirty qubit is tested until none is left.
  * The phase of phi is fixed by phi_0 real and >= 0; at |r| = 0, phi = |0>.
  * A merge of subsystems A (first operand's) and B is kron(b, a): A's qubits
    keep their bit positions and B's follow.

Two-qubit rounding. The paper states only that the technique generalizes to
(at least) two-qubit subsystems (Sec. III-A, after Fig. 2); it gives no rule
or schedule. Reading used here (an opt-in policy; the benchmarks use the
one-qubit form):
  * For a pair B = {a, b} of one subsystem S with at least three qubits, rho_B
    is the 4x4 reduced density matrix; its largest eigenvalue lambda is the
    weight of the dominant Schmidt term, and eps_B = 1 - lambda (for a single
    qubit this is exactly (1 - |r|)/2). The pair is rounded when
    eps_B <= p/2 + tau: S is projected on the dominant eigenvector phi of
    rho_B, the pair becomes its own subsystem [a, b] with amplitudes phi
    (index bit 0 = a, bit 1 = b), the normalized remainder <phi| psi stays in
    S, and F is multiplied by 1 - eps_B.
  * Schedule: after a two-qubit gate on (a, b) and the one-qubit tests it
    causes, if a and b still share a subsystem of at least three qubits, the
    pair is tested once; a rounding makes the rest of S dirty, whose one-qubit
    tests then run.
  * The phase of phi is fixed by its first component of magnitude above 1e-9
    being real and positive; the expanded ket does not depend on it.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

from . import dense

C128 = np.complex128
TAU = 1e-12


class CapacityError(RuntimeError):
    """A merge would exceed the amplitude cap; the state is left unchanged."""


@dataclass
class Attempt:
    qubit: int
    n_sub: int
    eps: float
    rounded: bool
    pair: int = -1  # the second qubit of a two-qubit attempt
    gates: int = 0  # multi-qubit gates applied before this attempt


@dataclass
class Sub:
    qubits: list
    amps: np.ndarray


def bloch(amps: np.ndarray, nq: int, t: int) -> np.ndarray:
    """r = (<X>, <Y>, <Z>) of the qubit at bit t (Sec. III-A, step 1).

    With a0 / a1 the amplitudes whose bit t is 0 / 1:
    <X> = 2 Re sum conj(a0) a1, <Y> = 2 Im sum conj(a0) a1,
    <Z> = sum |a0|^2 - sum |a1|^2, all divided by the squared norm.
    """
    v = amps.reshape(2 ** (nq - t - 1), 2, 2 ** t)
    a0, a1 = v[:, 0, :], v[:, 1, :]
    s = np.sum(a0.conj() * a1)
    z = np.sum(np.abs(a0) ** 2) - np.sum(np.abs(a1) ** 2)
    nrm = np.sum(np.abs(amps) ** 2)
    return np.array([2.0 * s.real, 2.0 * s.imag, z]) / nrm


def epsilon(r: np.ndarray) -> float:
    """eps = (1 - |r|)/2 (Sec. III-A, step 2), clipped to [0, 1/2]."""
    return float(min(max((1.0 - np.linalg.norm(r)) / 2.0, 0.0), 0.5))


def dominant_state(r: np.ndarray) -> np.ndarray:
    """The single-qubit state phi whose Bloch vector points along r: the
    eigenvector of rho_q = (I + r.sigma)/2 with the larger eigenvalue.
    phi = (cos(theta/2), e^{i varphi} sin(theta/2)), theta the polar and
    varphi the azimuthal angle of r; phi = |0> when r = 0."""
    rn = float(np.linalg.norm(r))
    if rn == 0.0:
        return np.array([1.0, 0.0], dtype=C128)
    theta = math.acos(max(-1.0, min(1.0, r[2] / rn)))
    varphi = math.atan2(r[1], r[0])
    return np.array([math.cos(theta / 2.0),
                     np.exp(1j * varphi) * math.sin(theta / 2.0)], dtype=C128)


def project_out(amps: np.ndarray, nq: int, t: int, phi: np.ndarray) -> np.ndarray:
    """Remainder <phi|_q psi on the other nq-1 qubits, normalized (Sec. III-A,
    steps 3-4). Its index is the subsystem index with bit t removed."""
    v = amps.reshape(2 ** (nq - t - 1), 2, 2 ** t)
    b = (np.conj(phi[0]) * v[:, 0, :] + np.conj(phi[1]) * v[:, 1, :]).reshape(-1)
    return b / math.sqrt(float(np.vdot(b, b).real))


def pair_density(amps: np.ndarray, nq: int, t1: int, t2: int) -> np.ndarray:
    """Reduced density matrix of the qubits at bits t1, t2 (t1 != t2): row and
    column index m = bit t1 + 2 bit t2; rho[m, m'] = sum over the other bits of
    a[.., m] conj(a[.., m']), divided by the squared norm."""
    v = amps.reshape([2] * nq)  # axis k is bit nq - 1 - k
    ax1, ax2 = nq - 1 - t1, nq - 1 - t2
    # move bit t2 then bit t1 to the last two axes: flattened index 2 b2 + b1
    v = np.moveaxis(v, [ax2, ax1], [nq - 2, nq - 1]).reshape(-1, 4)
    rho = v.T @ v.conj()
    return rho / np.trace(rho).real


def pair_dominant(rho: np.ndarray) -> tuple:
    """(eps_B, phi): eps_B = 1 - the largest eigenvalue of rho (clipped to
    [0, 3/4]) and phi its unit eigenvector, phase-fixed as in the module
    notes (numpy's Hermitian eigensolver)."""
    w, vecs = np.linalg.eigh(rho)
    phi = vecs[:, -1].astype(C128)
    big = np.abs(phi) > 1e-9 * np.abs(phi).max()
    k = int(np.argmax(big))
    phi = phi * (abs(phi[k]) / phi[k])
    return float(min(max(1.0 - w[-1], 0.0), 0.75)), phi


def project_out_pair(amps: np.ndarray, nq: int, t1: int, t2: int,
                     phi: np.ndarray) -> np.ndarray:
    """Remainder <phi|_B psi on the other nq-2 qubits, normalized; its index is
    the subsystem index with bits t1 and t2 removed (in order)."""
    v = amps.reshape([2] * nq)
    ax1, ax2 = nq - 1 - t1, nq - 1 - t2
    v = np.moveaxis(v, [ax2, ax1], [nq - 2, nq - 1]).reshape(-1, 4)
    b = v @ phi.conj()
    return b / math.sqrt(float(np.vdot(b, b).real))


@dataclass
class FactorizedState:
    """n qubits, each starting as its own |0> subsystem."""
    n: int
    max_amps: int = 2 ** 30
    tau: float = TAU
    subs: list = field(default_factory=list)
    F: float = 1.0
    log: list = field(default_factory=list)
    dirty: set = field(default_factory=set)
    # optional decision hook decide(qubit, n_sub, eps, rule) -> bool, called
    # with the rule's own decision; used to replay another run's decisions
    # where eps lies within rounding distance of the threshold
    decide: object = None
    gates_applied: int = 0  # multi-qubit gates applied so far

    def __post_init__(self):
        if not self.subs:
            self.subs = [Sub([q], np.array([1.0, 0.0], dtype=C128)) for q in range(self.n)]

    # -------------------------------------------------------------- lookup
    def where(self, q: int) -> tuple:
        for si, s in enumerate(self.subs):
            if q in s.qubits:
                return si, s.qubits.index(q)
        raise KeyError(q)

    def sizes(self) -> list:
        return sorted(len(s.qubits) for s in self.subs)

    # -------------------------------------------------------------- merge
    def merge(self, qa: int, qb: int) -> int:
        """Make qa and qb members of one subsystem; returns its index.

        c[i_A + 2^{n_A} i_B] = a[i_A] b[i_B], i.e. kron(b, a) (Sec. II-A)."""
        ia, _ = self.where(qa)
        ib, _ = self.where(qb)
        if ia == ib:
            return ia
        A, B = self.subs[ia], self.subs[ib]
        if 2 ** (len(A.qubits) + len(B.qubits)) > self.max_amps:
            raise CapacityError(f"merge of {len(A.qubits)}+{len(B.qubits)} qubits exceeds cap")
        merged = Sub(A.qubits + B.qubits, np.kron(B.amps, A.amps))
        keep = [s for k, s in enumerate(self.subs) if k not in (ia, ib)]
        keep.append(merged)
        self.subs = keep
        return len(keep) - 1

    # -------------------------------------------------------------- gates
    def apply(self, qubits, m: np.ndarray):
        """Apply a gate on global qubits (merging their subsystems first)."""
        qubits = list(qubits)
        # capacity check before any change, so that failure leaves the state as is
        seen, total = set(), 0
        for q in qubits:
            si, _ = self.where(q)
            if si not in seen:
                seen.add(si)
                total += len(self.subs[si].qubits)
        if 2 ** total > self.max_amps:
            raise CapacityError(f"gate needs a {total}-qubit subsystem")
        si = self.where(qubits[0])[0]
        for q in qubits[1:]:
            si = self.merge(qubits[0], q)
        si = self.where(qubits[0])[0]
        S = self.subs[si]
        local = [S.qubits.index(q) for q in qubits]
        S.amps = dense.apply_matrix(S.amps, len(S.qubits), local, m)

    def apply_gate(self, g):
        qubits, m = dense.gate_matrix(g)
        self.apply(qubits, m)
        if len(qubits) >= 2:
            self.gates_applied += 1
            self.dirty.update(qubits)

    # -------------------------------------------------------------- SDRP
    def test_qubit(self, q: int, p: float) -> bool:
        """One separability attempt on q (Eq. sdrp). Returns True if rounded."""
        si, t = self.where(q)
        S = self.subs[si]
        nq = len(S.qubits)
        self.dirty.discard(q)
        if nq == 1:
            return False
        r = bloch(S.amps, nq, t)
        eps = epsilon(r)
        rounds = eps <= p / 2.0 + self.tau
        if self.decide is not None:
            rounds = bool(self.decide(q, nq, eps, rounds))
        if rounds:
            phi = dominant_state(r)
            rest = project_out(S.amps, nq, t, phi)
            others = [x for x in S.qubits if x != q]
            S.qubits, S.amps = others, rest
            self.subs.append(Sub([q], phi))
            self.F *= (1.0 - eps)
            self.log.append(Attempt(q, nq, eps, True, gates=self.gates_applied))
            self.dirty.update(others)
            return True
        self.log.append(Attempt(q, nq, eps, False, gates=self.gates_applied))
        return False

    def test_pair(self, qa: int, qb: int, p: float) -> bool:
        """One two-qubit attempt on (qa, qb) (the reading in the module notes).
        Returns True if the pair was rounded into its own subsystem."""
        sa, ta = self.where(qa)
        sb, tb = self.where(qb)
        if sa != sb or qa == qb:
            return False
        S = self.subs[sa]
        nq = len(S.qubits)
        if nq < 3:
            return False
        eps, phi = pair_dominant(pair_density(S.amps, nq, ta, tb))
        rounds = eps <= p / 2.0 + self.tau
        if self.decide is not None:
            rounds = bool(self.decide(qa, nq, eps, rounds))
        self.log.append(Attempt(qa, nq, eps, rounds, pair=qb, gates=self.gates_applied))
        if not rounds:
            return False
        rest = project_out_pair(S.amps, nq, ta, tb, phi)
        others = [x for x in S.qubits if x not in (qa, qb)]
        S.qubits, S.amps = others, rest
        self.subs.append(Sub([qa, qb], phi))
        self.F *= (1.0 - eps)
        self.dirty.update(others)
        return True

    def try_separate(self, p: float) -> int:
        """Test dirty qubits, lowest index first, until none is dirty."""
        count = 0
        while self.dirty:
            q = min(self.dirty)
            count += int(self.test_qubit(q, p))
        return count

    def run(self, gates, p: float, pairs: bool = False):
        """Apply a gate list, testing separability after every multi-qubit gate
        (and, with pairs=True, the two-qubit rounding after two-qubit gates)."""
        for g in gates:
            self.apply_gate(g)
            qubits = dense.gate_matrix(g)[0]
            if len(qubits) >= 2:
                self.try_separate(p)
                if pairs and len(qubits) == 2 and self.test_pair(qubits[0], qubits[1], p):
                    self.try_separate(p)
        return self

    def run_tests_as_logged(self, gates, p: float, tests):
        """Apply a gate list, making exactly the one-qubit attempts listed in
        `tests`, in their order: (k, q) tests qubit q after the k-th
        multi-qubit gate of the list and before the next one. This replays
        another schedule (such as a learned proposal's, which tests some
        dirty qubits, skips others and tests those later) with this oracle's
        own arithmetic; the decision on each attempt is the rounding rule's
        (or the decide hook's). The dirty set is kept but not consulted."""
        tests = list(tests)
        pos = 0

        def due(k):
            nonlocal pos
            while pos < len(tests) and tests[pos][0] == k:
                self.test_qubit(tests[pos][1], p)
                pos += 1

        due(self.gates_applied)
        for g in gates:
            self.apply_gate(g)
            if len(dense.gate_matrix(g)[0]) >= 2:
                due(self.gates_applied)
        if pos != len(tests):
            raise ValueError(f"attempt {pos} of {len(tests)} is not at a multi-qubit gate "
                             f"boundary of the list")
        return self

    # -------------------------------------------------------------- readout
    def expand(self) -> np.ndarray:
        """Full 2^n ket: amplitude(x) = prod_S a_S[x restricted to S]."""
        x = np.arange(2 ** self.n, dtype=np.int64)
        out = np.ones(2 ** self.n, dtype=C128)
        for S in self.subs:
            loc = np.zeros_like(x)
            for t, q in enumerate(S.qubits):
                loc |= ((x >> q) & 1) << t
            out *= S.amps[loc]
        return out

    def amplitude(self, x: int) -> complex:
        val = 1.0 + 0j
        for S in self.subs:
            loc = 0
            for t, q in enumerate(S.qubits):
                loc |= ((x >> q) & 1) << t
            val *= S.amps[loc]
        return complex(val)
