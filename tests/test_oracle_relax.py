"""Pins for the residual-based relaxation (Section 2.3.3, Algorithm 2) and the
BF16 split representation (not GPU)."""
import numpy as np

from oracle import relax, split


def test_alpha_closed_form_for_scaled_residual():
    # f_{k+1} = lambda f_k  =>  alpha_{k+1} = alpha_k / (1 - lambda)
    rng = np.random.default_rng(0)
    f = rng.normal(size=(4, 6, 10, 3))
    lam = np.array([0.5, -0.3, 0.9, 0.1])
    a0 = np.array([1.0, 2.0, 0.7, 1.3])
    a1 = relax.relax_alpha(lam[:, None, None, None] * f, f, a0)
    assert np.allclose(a1, a0 / (1 - lam), rtol=1e-13)
    # lambda > 1 gives a negative value, reset to 1
    a2 = relax.relax_alpha(1.5 * f, f, a0)
    assert np.all(a2 == 1.0)
    # zero denominator keeps the previous value
    a3 = relax.relax_alpha(f, f, a0)
    assert np.array_equal(a3, a0)


def test_alpha_matches_aitken_formula_generic():
    rng = np.random.default_rng(1)
    fo = rng.normal(size=(2, 50))
    fn = rng.normal(size=(2, 50))
    a = np.array([0.8, 1.1])
    out = relax.relax_alpha(fn, fo, a)
    for r in range(2):
        ref = -a[r] * np.dot(fo[r], fn[r] - fo[r]) / np.dot(fn[r] - fo[r], fn[r] - fo[r])
        assert np.isclose(out[r], ref if ref >= 0 else 1.0, rtol=1e-14)


def test_alpha_lower_bound_variant():
    """Remark in Section 2.3.3: alpha_{k+1} bounded below by alpha_min.  With
    f_{k+1} = lambda f_k the unbounded value is alpha_k / (1 - lambda)."""
    rng = np.random.default_rng(3)
    f = rng.normal(size=(4, 6, 10, 3))
    lam = np.array([-3.0, -0.25, 0.5, 1.5])          # 0.25, 0.8, 2, negative (-> 1)
    a0 = np.ones(4)
    plain = relax.relax_alpha(lam[:, None, None, None] * f, f, a0)
    assert np.allclose(plain, [0.25, 0.8, 2.0, 1.0], rtol=1e-13)
    bounded = relax.relax_alpha(lam[:, None, None, None] * f, f, a0, alpha_min=0.5)
    assert np.allclose(bounded, [0.5, 0.8, 2.0, 1.0], rtol=1e-13)
    # a bound above 1 also lifts the reset value of negative alphas
    assert np.allclose(relax.relax_alpha(1.5 * f, f, a0, alpha_min=1.2), 1.2)
    # the step bound still caps the bounded value
    st = relax.RelaxState(n_rhs=1, relax=True, du_max=1e-3, alpha_min=0.9, tol_f=0.0)
    u = np.zeros((1, 6, 4, 3))
    apply_fn = lambda g: g[:, :, :4, :]
    for g in (f[:1], 0.5 * f[:1], -2.0 * f[:1]):
        u, out = relax.relax_step(st, g, u, apply_fn)
    assert out["step_inf"][0] <= 1e-3 * (1 + 1e-14)


def test_step_clamp():
    a = np.array([2.0, 0.5])
    w_inf = np.array([1.0, 1.0])
    out = relax.clamp_step(a, w_inf, 1.5)
    assert np.allclose(out, [1.5, 0.5])


def test_relax_step_sequence():
    # alpha = 1 for k < 2; at k = 2 Relax(f3, f2, alpha_2 = 1); raw f passed to Relax
    rng = np.random.default_rng(2)
    shape = (2, 4, 5, 3)
    fs = [rng.normal(size=shape) for _ in range(4)]
    apply_fn = lambda f: f[:, :, :3, :] * 0.5          # any linear map with the pad layout
    st = relax.RelaxState(n_rhs=2, relax=True, tol_f=1e-3)
    u = np.zeros((2, 4, 3, 3))
    alphas = []
    for f in fs:
        u, out = relax.relax_step(st, f, u, apply_fn)
        alphas.append(out["alpha"])
        assert np.abs(u.mean(axis=(1, 2))).max() < 1e-14
    assert np.all(alphas[0] == 1) and np.all(alphas[1] == 1)
    assert np.allclose(alphas[2], relax.relax_alpha(fs[2], fs[1], np.ones(2)))
    assert np.allclose(alphas[3], relax.relax_alpha(fs[3], fs[2], alphas[2]))
    assert st.k == 4


def test_bf16_split_bound():
    rng = np.random.default_rng(3)
    x = np.concatenate([rng.normal(size=20000) * 10.0 ** rng.integers(-20, 20, size=20000),
                        np.array([1.0, -1.0, 1 + 2 ** -8, 1 + 2 ** -9 + 2 ** -17, 3.0, 1e-30, 65504.0])])
    hi, lo = split.split_bf16(x)
    # hi and lo are exact bf16 values
    for v in (hi, lo):
        assert np.all((v.view(np.uint32) & 0xFFFF) == 0)
    err = np.abs(x - hi.astype(np.float64) - lo.astype(np.float64))
    # 2^-16 relative, plus the float32 rounding of x itself (2^-24)
    assert np.all(err <= (2.0 ** -16 + 2.0 ** -23) * np.abs(x))


def test_bf16_round_ties_to_even():
    v = np.array([1 + 2 ** -8, 1 + 3 * 2 ** -8, 1 + 2 ** -8 + 2 ** -20], dtype=np.float32)
    r = split.round_bf16(v)
    assert r[0] == 1.0 and r[1] == 1 + 4 * 2 ** -8 and r[2] == 1 + 2 ** -7
