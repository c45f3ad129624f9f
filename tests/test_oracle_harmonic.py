"""The harmonic FBC loop on the CPU with the oracle's Green operator and relaxation:
pins the loop harness and two facts the paper states (CPU only, no GPU).

* Remark 1: when the atomistic model is the harmonic model, the FBC method converges in
  two steps -- the second (AH) solve, with the pad from one Green update, is already
  the solution, so the second incompatibility force vanishes to rounding;
* the fixed point is the global harmonic solution u* = G f_ext (Section 2.3.1), up to the
  rigid translation fixed by the mean-zero pad condition (eq. mean(u^p)=0).
"""
import numpy as np
import pytest

from oracle import apply as oap, green as ogr, relax as orx

from harmonic_fbc import HarmonicDisc, external_force, run_loop

NZ, M, R_A = 8, 64, 3.0


@pytest.fixture(scope="module")
def disc():
    return HarmonicDisc(NZ, R_A)


def _exact(disc, f_ext):
    out = np.concatenate([disc.cols_a, disc.cols_ipp])
    g = ogr.green_modes_dense(NZ, M, M, out, disc.cols_a)
    u = oap.apply_green(g, f_ext[None])[0]
    return u - u[:, disc.n_a:].mean(axis=(0, 1))          # pad mean zero


def _oracle_update(disc, relax):
    g = ogr.green_modes_dense(NZ, M, M, disc.cols_ipp, disc.cols_ip)
    st = orx.RelaxState(n_rhs=1, relax=relax, tol_f=1e-12)
    state = {"u": np.zeros((1, NZ, disc.n_ipp, 3))}

    def update(f_in, k):
        state["u"], _ = orx.relax_step(st, f_in[None], state["u"], lambda f: oap.apply_green(g, f))
        return state["u"][0]
    return update


def test_sets_are_consistent(disc):
    assert disc.n_a > 50 and disc.n_ip > 20 and disc.n_ipp > disc.n_ip
    a = {tuple(c) for c in disc.cols_a}
    assert not a & {tuple(c) for c in disc.cols_ipp}


def test_remark1_two_step_convergence_and_fixed_point(disc):
    f_ext = external_force(disc, seed=3)
    u_a, u_p, hist = run_loop(disc, f_ext, _oracle_update(disc, relax=False), 4)
    assert hist[0] > 1e-3                           # the first step does correct the pad
    assert hist[1] < 1e-12 * hist[0], hist          # converged in the second step
    ref = _exact(disc, f_ext)
    got = np.concatenate([u_a, u_p], axis=1)
    assert np.linalg.norm(got - ref) / np.linalg.norm(ref) < 1e-10


def test_relaxed_loop_reaches_the_same_fixed_point(disc):
    f_ext = external_force(disc, seed=4)
    u_a, u_p, hist = run_loop(disc, f_ext, _oracle_update(disc, relax=True), 5)
    ref = _exact(disc, f_ext)
    got = np.concatenate([u_a, u_p], axis=1)
    assert np.linalg.norm(got - ref) / np.linalg.norm(ref) < 1e-10
