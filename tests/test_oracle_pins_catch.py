"""Plant plausible mistakes in the oracle (on the CPU) and check that the pins
catch each one: a pin that cannot fail does not pin anything."""
import math

import numpy as np
import pytest

from oracle import dense, factor, mlp
import test_oracle_dense as td
import test_oracle_factor as tf
import test_oracle_mlp as tm


def _fails(fn, *args):
    with pytest.raises(AssertionError):
        fn(*args)


def test_transposed_u3_is_caught(monkeypatch):
    good = dense.u3
    monkeypatch.setattr(dense, "u3", lambda t, p, l: good(t, p, l).T)
    _fails(td.test_u3_special_cases)


def test_wrong_sign_qft_phase_is_caught(monkeypatch):
    good = dense.qft_gates

    def bad(n, start=0, length=None, inverse=False):
        return [(g[0], g[1], g[2], -g[3]) if g[0] == "cp" else g
                for g in good(n, start, length, inverse)]
    monkeypatch.setattr(dense, "qft_gates", bad)
    _fails(td.test_qft_equals_inverse_fft, 5)


def test_missing_bit_reversal_is_caught(monkeypatch):
    good = dense.qft_gates
    monkeypatch.setattr(dense, "qft_gates",
                        lambda *a, **k: [g for g in good(*a, **k) if g[0] != "swap"])
    _fails(td.test_qft_basis_state_closed_form, 3)


def test_off_by_one_phase_index_is_caught(monkeypatch):
    good = dense.qft_gates

    def bad(n, start=0, length=None, inverse=False):
        return [(g[0], g[1], g[2], g[3] / 2) if g[0] == "cp" else g
                for g in good(n, start, length, inverse)]
    monkeypatch.setattr(dense, "qft_gates", bad)
    _fails(td.test_qft_ghz_closed_form, 3)


def test_reversed_qubit_axes_are_caught(monkeypatch):
    good = dense.apply_matrix
    monkeypatch.setattr(dense, "apply_matrix",
                        lambda a, n, qubits, m: good(a, n, list(qubits)[::-1], m))
    _fails(td.test_apply_matrix_matches_brute_force, 4, 2)


def test_swapped_control_value_is_caught(monkeypatch):
    good = dense.controlled_matrix
    monkeypatch.setattr(dense, "controlled_matrix",
                        lambda nc, cv, m: good(nc, cv ^ 1, m))
    _fails(td.test_controlled_gate_by_index_loop)


def test_bloch_missing_factor_two_is_caught(monkeypatch):
    good = factor.bloch

    def bad(amps, nq, t):
        r = good(amps, nq, t)
        return np.array([r[0] / 2, r[1] / 2, r[2]])
    monkeypatch.setattr(factor, "bloch", bad)
    _fails(tf.test_bloch_vector_is_pauli_expectation, 4)


def test_unconjugated_projection_is_caught(monkeypatch):
    def bad(amps, nq, t, phi):
        v = amps.reshape(2 ** (nq - t - 1), 2, 2 ** t)
        b = (phi[0] * v[:, 0, :] + phi[1] * v[:, 1, :]).reshape(-1)
        return b / math.sqrt(float(np.vdot(b, b).real))
    monkeypatch.setattr(factor, "project_out", bad)
    _fails(tf.test_projection_fidelity_is_one_minus_eps)


def test_flipped_threshold_is_caught(monkeypatch):
    def bad_test(self, q, p):
        # rounds when eps <= p instead of p/2
        si, t = self.where(q)
        S = self.subs[si]
        nq = len(S.qubits)
        self.dirty.discard(q)
        if nq == 1:
            return False
        r = factor.bloch(S.amps, nq, t)
        eps = factor.epsilon(r)
        ok = eps <= p
        self.log.append(factor.Attempt(q, nq, eps, ok))
        if ok:
            phi = factor.dominant_state(r)
            S.amps = factor.project_out(S.amps, nq, t, phi)
            S.qubits = [x for x in S.qubits if x != q]
            self.subs.append(factor.Sub([q], phi))
            self.F *= 1 - eps
        return ok
    monkeypatch.setattr(factor.FactorizedState, "test_qubit", bad_test)
    _fails(tf.test_golden_weakly_entangled_pair)


def test_merge_operand_order_is_caught(monkeypatch):
    def bad_merge(self, qa, qb):
        ia, _ = self.where(qa)
        ib, _ = self.where(qb)
        if ia == ib:
            return ia
        A, B = self.subs[ia], self.subs[ib]
        merged = factor.Sub(A.qubits + B.qubits, np.kron(A.amps, B.amps))
        self.subs = [s for k, s in enumerate(self.subs) if k not in (ia, ib)] + [merged]
        return len(self.subs) - 1
    monkeypatch.setattr(factor.FactorizedState, "merge", bad_merge)
    _fails(tf.test_merge_is_kron_and_keeps_reduced_states)


def test_dropped_tanh_derivative_is_caught(monkeypatch):
    good = mlp.backward

    def bad(params, x, y):
        f = mlp.forward(params, x)
        y = np.asarray(y, dtype=np.float64)
        B = f["x"].shape[0]
        dz3 = ((f["score"] - y) / B).reshape(-1, 1)
        g = {"W3": f["h2"].T @ dz3, "b3": dz3.sum(axis=0)}
        dz2 = dz3 @ params["W3"].T          # missing (1 - h2^2)
        g["W2"] = f["h1"].T @ dz2
        g["b2"] = dz2.sum(axis=0)
        dz1 = (dz2 @ params["W2"].T) * (1.0 - f["h1"] ** 2)
        g["W1"] = f["x"].T @ dz1
        g["b1"] = dz1.sum(axis=0)
        return g
    monkeypatch.setattr(mlp, "backward", bad)
    _fails(tm.test_gradient_matches_central_differences, 0)


# ------------------------------------------------------------ two-qubit rounding
import test_oracle_pairs as tp  # noqa: E402


def test_pair_density_without_conjugate_is_caught(monkeypatch):
    def bad(amps, nq, t1, t2):
        v = amps.reshape([2] * nq)
        ax1, ax2 = nq - 1 - t1, nq - 1 - t2
        v = np.moveaxis(v, [ax2, ax1], [nq - 2, nq - 1]).reshape(-1, 4)
        rho = v.T @ v  # conjugate dropped
        return rho / np.trace(rho)
    monkeypatch.setattr(factor, "pair_density", bad)
    _fails(tp.test_pair_density_by_definition, 3, 1)


def test_pair_bits_in_the_wrong_order_are_caught(monkeypatch):
    good = factor.pair_density
    monkeypatch.setattr(factor, "pair_density", lambda a, n, t1, t2: good(a, n, t2, t1))
    _fails(tp.test_pair_density_by_definition, 0, 4)


def test_smallest_eigenvalue_as_eps_is_caught(monkeypatch):
    def bad(rho):
        w, vecs = np.linalg.eigh(rho)
        return float(w[0]), vecs[:, -1].astype(complex)
    monkeypatch.setattr(factor, "pair_dominant", bad)
    _fails(tp.test_pair_spectrum_is_schmidt_weights, 1)


def test_projection_on_the_weakest_term_is_caught(monkeypatch):
    good = factor.pair_dominant

    def bad(rho):
        eps, _ = good(rho)
        return eps, np.linalg.eigh(rho)[1][:, 0].astype(complex)
    monkeypatch.setattr(factor, "pair_dominant", bad)
    _fails(tp.test_projection_overlap_is_dominant_weight, 0)


def test_projection_without_conjugate_phi_is_caught(monkeypatch):
    def bad(amps, nq, t1, t2, phi):
        v = amps.reshape([2] * nq)
        ax1, ax2 = nq - 1 - t1, nq - 1 - t2
        v = np.moveaxis(v, [ax2, ax1], [nq - 2, nq - 1]).reshape(-1, 4)
        b = v @ phi
        return b / math.sqrt(float(np.vdot(b, b).real))
    monkeypatch.setattr(factor, "project_out_pair", bad)
    _fails(tp.test_projection_overlap_is_dominant_weight, 1)


# ------------------------------------------------------------ schedule and optimizer
def test_rest_not_marked_dirty_after_rounding_is_caught(monkeypatch):
    good = factor.FactorizedState.test_qubit

    def bad(self, q, p):
        before = set(self.dirty)
        rounded = good(self, q, p)
        if rounded:
            self.dirty = before - {q}  # the co-members keep their old marks
        return rounded
    monkeypatch.setattr(factor.FactorizedState, "test_qubit", bad)
    assert tf.fixed_point_violations("matching") + tf.fixed_point_violations("grid")


def test_highest_dirty_first_is_caught(monkeypatch):
    def bad(self, p):
        count = 0
        while self.dirty:
            count += int(self.test_qubit(max(self.dirty), p))
        return count
    monkeypatch.setattr(factor.FactorizedState, "try_separate", bad)
    for case in tf.load_schedule_cases("sdrp_schedule.txt"):
        _fails(tf.test_golden_schedule_order, case)


def test_adam_without_momentum_accumulation_is_caught(monkeypatch):
    def bad(params, grads, m, v, step, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
        for k, _ in mlp.SHAPES:
            m[k] = (1.0 - b1) * grads[k]  # the b1 * m term dropped
            v[k] = b2 * v[k] + (1.0 - b2) * grads[k] ** 2
            mh = m[k] / (1.0 - b1 ** step)
            vh = v[k] / (1.0 - b2 ** step)
            params[k] = params[k] - lr * mh / (np.sqrt(vh) + eps)
    monkeypatch.setattr(mlp, "adam_step", bad)
    _fails(tm.test_adam_constant_gradient_moves_lr_each_step)
    _fails(tm.test_adam_two_steps_by_hand)
