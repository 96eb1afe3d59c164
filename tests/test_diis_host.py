"""Host logic of the DIIS solver (paper_2206_07660_amd/diis.py) on numpy vectors:
the Pulay coefficients against a direct constrained least-squares solve, the
Gram-matrix bookkeeping of a bounded history, and convergence on a linear
fixed-point map, where DIIS with a full history is equivalent to GMRES and
reaches the solution in about n + 1 iterations (history pairs whose residuals
become linearly dependent near the solution are dropped, which costs a few)."""
import numpy as np

from paper_2206_07660_amd.diis import DIISCore


def np_core(depth=6, mixing=1.0):
    def axpby(a, x, b, y):
        if x is None:
            y *= b
        else:
            y *= b
            y += a * x
    return DIISCore(lambda u, v: complex(np.vdot(u, v)), axpby,
                    lambda: np.empty(N_DIM, complex), depth=depth, mixing=mixing)


N_DIM = 12


def brute_coefficients(fs):
    # c = e_last + D t, D = [e_i - e_last]: unconstrained least squares in t
    F = np.stack(fs, axis=1)
    n = F.shape[1]
    if n == 1:
        return np.ones(1)
    Fr = np.concatenate([F.real, F.imag])
    D = Fr[:, :-1] - Fr[:, -1:]
    t = np.linalg.lstsq(D, -Fr[:, -1], rcond=None)[0]
    return np.concatenate([t, [1.0 - t.sum()]])


def test_coefficients_match_constrained_least_squares():
    rng = np.random.default_rng(5)
    core = np_core(depth=5)
    fs = []
    for i in range(5):
        # residuals of very different sizes, as late iterations have
        f = (rng.normal(size=N_DIM) + 1j * rng.normal(size=N_DIM)) * 10.0 ** (-2 * i)
        x = rng.normal(size=N_DIM) + 0j
        core.push(x, f)
        fs.append(f)
        c = core.coefficients()
        ref = brute_coefficients(fs)
        assert abs(c.sum() - 1.0) < 1e-12
        res, res_ref = np.linalg.norm(np.stack(fs, 1) @ c), np.linalg.norm(np.stack(fs, 1) @ ref)
        assert res <= res_ref * (1 + 1e-9) + 1e-300
        assert np.allclose(c, ref, rtol=1e-8, atol=1e-10)


def test_bounded_history_keeps_the_gram_matrix():
    rng = np.random.default_rng(6)
    core = np_core(depth=3)
    for _ in range(7):
        core.push(rng.normal(size=N_DIM) + 0j, rng.normal(size=N_DIM) + 1j * rng.normal(size=N_DIM))
    assert len(core) == 3
    G = np.array([[np.vdot(a, b).real for b in core.fs] for a in core.fs])
    assert np.allclose(core.B, G, rtol=1e-13)


def test_extrapolation_is_the_combination_of_updated_points():
    rng = np.random.default_rng(7)
    core = np_core(depth=4, mixing=0.3)
    for _ in range(4):
        core.push(rng.normal(size=N_DIM) + 0j, rng.normal(size=N_DIM) + 0j)
    out = np.empty(N_DIM, complex)
    c = core.extrapolate(out)
    ref = sum(ci * (x + 0.3 * f) for ci, x, f in zip(c, core.xs, core.fs))
    assert np.allclose(out, ref, rtol=1e-13, atol=1e-15)


def test_linear_fixed_point_converges_in_about_n_iterations():
    rng = np.random.default_rng(8)
    n = N_DIM
    A = rng.normal(size=(n, n))
    A *= 0.9 / np.abs(np.linalg.eigvals(A)).max()       # a contraction only in spectral radius
    b = rng.normal(size=n)
    x_star = np.linalg.solve(np.eye(n) - A, b)
    core = np_core(depth=n + 2)
    x = np.zeros(n, complex)
    hist = []
    for it in range(n + 5):
        f = A @ x.real + b - x.real + 0j
        hist.append(np.abs(f).max())
        if hist[-1] < 1e-10:
            break
        core.push(x, f)
        core.extrapolate(x)
    print("max |F| per iteration", ["%.1e" % h for h in hist])
    assert hist[-1] < 1e-10
    assert np.abs(x.real - x_star).max() < 1e-9
    # plain iteration x <- A x + b is far from converged after as many steps
    y = np.zeros(n)
    for _ in range(n + 2):
        y = A @ y + b
    assert np.abs(y - x_star).max() > 1e-3


def test_reset_forgets_the_history():
    rng = np.random.default_rng(9)
    core = np_core(depth=4)
    for _ in range(3):
        core.push(rng.normal(size=N_DIM) + 0j, rng.normal(size=N_DIM) + 0j)
    core.reset()
    assert len(core) == 0 and core.B.shape == (0, 0)
    x, f = rng.normal(size=N_DIM) + 0j, rng.normal(size=N_DIM) + 0j
    core.push(x, f)
    out = np.empty(N_DIM, complex)
    c = core.extrapolate(out)
    assert np.allclose(c, [1.0]) and np.allclose(out, x + f)
