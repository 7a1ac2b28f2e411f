"""Pins of the oracle's single-cell arithmetic against facts fixed by the
mathematics: textbook D3Q27 weights, closed-form equilibrium moments, the
definition of central moments, the set-partition definition of joint
cumulants, conservation laws, lattice symmetry and fixed points."""
import itertools
import math

import numpy as np
import pytest

from oracle import mlp_ref

C27 = np.array([[i % 3 - 1, (i // 3) % 3 - 1, i // 9 - 1] for i in range(27)])


def rand_pops(rng, rho=1.0, amp=0.2):
    """random positive populations around the rest weights"""
    w1 = np.array([1 / 6, 2 / 3, 1 / 6])
    w = np.array([w1[c[0] + 1] * w1[c[1] + 1] * w1[c[2] + 1] for c in C27])
    return rho * w * (1.0 + amp * rng.uniform(-1, 1, 27))


def test_weights_textbook(orc):
    c, w = orc.lattice()
    assert np.array_equal(c, C27)
    expect = {0: 8 / 27, 1: 2 / 27, 2: 1 / 54, 3: 1 / 216}
    for i in range(27):
        assert w[i] == pytest.approx(expect[int(np.abs(c[i]).sum())], rel=1e-15)
    assert w.sum() == pytest.approx(1.0, abs=1e-15)
    # isotropy up to fourth order: sum w c_a c_b = delta/3
    assert np.allclose(np.einsum("i,ia,ib->ab", w, c, c), np.eye(3) / 3, atol=1e-15)
    assert np.allclose(np.einsum("i,ia->a", w, c), 0, atol=1e-16)


def test_equilibrium_raw_moments_closed_form(orc):
    """sum c_x^a c_y^b c_z^c f_eq = rho m_a(ux) m_b(uy) m_c(uz),
    m0 = 1, m1 = u, m2 = u^2 + 1/3"""
    rng = np.random.default_rng(1)
    for _ in range(5):
        rho = rng.uniform(0.8, 1.2)
        u = rng.uniform(-0.15, 0.15, 3)
        f = orc.feq(rho, u)
        m = lambda k, v: [1.0, v, v * v + 1 / 3][k]
        for a, b, cc in itertools.product(range(3), repeat=3):
            raw = np.sum(C27[:, 0] ** a * C27[:, 1] ** b * C27[:, 2] ** cc * f)
            assert raw == pytest.approx(rho * m(a, u[0]) * m(b, u[1]) * m(cc, u[2]),
                                        abs=1e-15)
    c, w = orc.lattice()
    assert np.allclose(orc.feq(1.0, [0, 0, 0]), w, atol=1e-17)


def test_central_moments_definition(orc):
    rng = np.random.default_rng(2)
    for _ in range(5):
        f = rand_pops(rng)
        u = rng.uniform(-0.1, 0.1, 3)
        d = C27 - u
        ref = np.array([np.sum(d[:, 0] ** (m % 3) * d[:, 1] ** ((m // 3) % 3) *
                               d[:, 2] ** (m // 9) * f) for m in range(27)])
        assert np.allclose(orc.central_moments(f, u, direct=True), ref, atol=1e-15)
        assert np.allclose(orc.central_moments(f, u), ref, atol=2e-15)
        assert np.allclose(orc.central_to_pops(ref, u), f, atol=2e-15)


def _partitions(items):
    if len(items) == 1:
        yield [items]
        return
    first, rest = items[0], items[1:]
    for smaller in _partitions(rest):
        for k in range(len(smaller)):
            yield smaller[:k] + [[first] + smaller[k]] + smaller[k + 1:]
        yield [[first]] + smaller


def _joint_cumulant(p, X, labels):
    """kappa(X_l1..X_ln) = sum over set partitions pi of
    (-1)^(|pi|-1) (|pi|-1)! prod_B E[prod_{i in B} X_li]"""
    total = 0.0
    for part in _partitions(list(range(len(labels)))):
        prod = 1.0
        for B in part:
            prod *= np.sum(p * np.prod([X[:, labels[i]] for i in B], axis=0))
        k = len(part)
        total += (-1) ** (k - 1) * math.factorial(k - 1) * prod
    return total


def test_cumulants_equal_joint_cumulants(orc):
    """Orders 2..6 against the set-partition definition for a random
    27-point distribution about its own mean."""
    rng = np.random.default_rng(3)
    f = rand_pops(rng, rho=1.07, amp=0.5)
    rho = f.sum()
    u = (C27 * f[:, None]).sum(0) / rho
    kap = orc.central_moments(f, u)
    Cm = orc.cumulants(kap)
    p = f / rho
    X = C27 - u
    for m in range(27):
        a, b, c = m % 3, (m // 3) % 3, m // 9
        if a + b + c < 2:
            continue
        labels = [0] * a + [1] * b + [2] * c
        assert Cm[m] == pytest.approx(_joint_cumulant(p, X, labels), abs=2e-15), m
    # inverse map
    back = orc.cumulants_inverse(Cm)
    assert np.allclose(back, kap, atol=2e-15)


def test_product_distribution_has_no_mixed_cumulants(orc):
    rng = np.random.default_rng(4)
    q = [rng.uniform(0.1, 1.0, 3) for _ in range(3)]
    q = [v / v.sum() for v in q]
    f = np.array([1.1 * q[0][c[0] + 1] * q[1][c[1] + 1] * q[2][c[2] + 1] for c in C27])
    u = (C27 * f[:, None]).sum(0) / f.sum()
    Cm = orc.cumulants(orc.central_moments(f, u))
    for m in range(27):
        a, b, c = m % 3, (m // 3) % 3, m // 9
        if a + b + c >= 2 and sum(x > 0 for x in (a, b, c)) >= 2:
            assert abs(Cm[m]) < 1e-15, m
    # pure second order = 1-D variance
    var = [np.sum(q[d] * (np.array([-1, 0, 1]) - u[d]) ** 2) for d in range(3)]
    assert Cm[2] == pytest.approx(var[0], abs=1e-15)
    assert Cm[6] == pytest.approx(var[1], abs=1e-15)
    assert Cm[18] == pytest.approx(var[2], abs=1e-15)


@pytest.mark.parametrize("seed", range(4))
def test_collision_conserves_mass_and_momentum_with_force(orc, seed):
    rng = np.random.default_rng(10 + seed)
    f = rand_pops(rng, rho=rng.uniform(0.9, 1.1))
    F = rng.uniform(-1e-3, 1e-3, 3)
    om = rng.uniform(0.3, 1.95, 10)
    fo = orc.collide(f, F, om)
    assert fo.sum() == pytest.approx(f.sum(), rel=1e-14)
    j0 = (C27 * f[:, None]).sum(0)
    j1 = (C27 * fo[:, None]).sum(0)
    assert np.allclose(j1, j0 + F, atol=1e-15)


def test_unit_rates_give_equilibrium(orc):
    rng = np.random.default_rng(5)
    f = rand_pops(rng, amp=0.4)
    rho = f.sum()
    u = (C27 * f[:, None]).sum(0) / rho
    fo = orc.collide(f, [0, 0, 0], np.ones(10))
    assert np.allclose(fo, orc.feq(rho, u), atol=1e-15)


def test_equilibrium_is_fixed_point(orc):
    rng = np.random.default_rng(6)
    u = rng.uniform(-0.1, 0.1, 3)
    fe = orc.feq(1.03, u)
    om = rng.uniform(0.5, 1.9, 10)
    assert np.allclose(orc.collide(fe, [0, 0, 0], om), fe, atol=1e-16)


def test_shear_rate_relaxes_second_order_only(orc):
    """with omega_2..10 = 1 the off-diagonal second cumulant keeps the
    fraction (1 - omega_1), the others are at equilibrium"""
    rng = np.random.default_rng(7)
    f = rand_pops(rng, amp=0.3)
    rho = f.sum()
    u = (C27 * f[:, None]).sum(0) / rho
    kap = orc.central_moments(f, u)
    om1 = 1.7
    fo = orc.collide(f, [0, 0, 0], [om1] + [1.0] * 9)
    kap_o = orc.central_moments(fo, u)
    assert kap_o[1 + 3] / rho == pytest.approx((1 - om1) * kap[1 + 3] / rho, abs=1e-15)
    dxy = (kap[2] - kap[6]) / rho
    assert (kap_o[2] - kap_o[6]) / rho == pytest.approx((1 - om1) * dxy, abs=1e-15)
    assert (kap_o[2] + kap_o[6] + kap_o[18]) / rho == pytest.approx(1.0, abs=1e-15)


def _symmetries():
    for perm in itertools.permutations(range(3)):
        for signs in itertools.product([1, -1], repeat=3):
            S = np.zeros((3, 3), dtype=int)
            for r in range(3):
                S[r, perm[r]] = signs[r]
            yield S


def test_collision_commutes_with_cubic_group(orc):
    rng = np.random.default_rng(8)
    f = rand_pops(rng, amp=0.3)
    F = rng.uniform(-1e-3, 1e-3, 3)
    om = rng.uniform(0.5, 1.9, 10)
    fo = orc.collide(f, F, om)
    idx = {tuple(c): i for i, c in enumerate(C27)}
    n = 0
    for S in _symmetries():
        sigma = np.array([idx[tuple(S @ c)] for c in C27])  # c_sigma(i) = S c_i
        g = np.empty(27)
        g[sigma] = f
        go = orc.collide(g, S @ F, om)
        assert np.allclose(go[sigma], fo, atol=1e-15)
        n += 1
    assert n == 48


def _q_norm(kap):
    rho = kap[0]
    A = np.array([[kap[2], kap[4], kap[10]], [kap[4], kap[6], kap[12]],
                  [kap[10], kap[12], kap[18]]]) / rho - np.eye(3) / 3
    P = A - np.trace(A) / 3 * np.eye(3)
    return A, np.sqrt(np.sum(P * P))


def test_smagorinsky_implicit_relation(orc):
    """nu_t = Cs^2 |S| with |S| = sqrt(2) Q / (2 c_s^2 tau) and
    nu_t = c_s^2 (tau - tau0) (Hou et al. 1996)"""
    rng = np.random.default_rng(9)
    for cs in (0.1, 0.17):
        f = rand_pops(rng, amp=0.3)
        rho = f.sum()
        u = (C27 * f[:, None]).sum(0) / rho
        kap = orc.central_moments(f, u)
        om0 = 1.95
        om = orc.smagorinsky_omega(kap, om0, cs)
        tau, tau0 = 1 / om, 1 / om0
        _, Q = _q_norm(kap)
        lhs = (tau - tau0) / 3.0
        rhs = cs * cs * np.sqrt(2.0) * Q / (2.0 / 3.0 * tau)
        assert abs(lhs - rhs) <= 1e-12 * max(abs(lhs), 1e-12)
        assert om < om0
    assert orc.smagorinsky_omega(kap, 1.95, 0.0) == pytest.approx(1.95, rel=1e-15)


def test_closure_features_are_invariants(orc):
    rng = np.random.default_rng(11)
    f = rand_pops(rng, amp=0.3)
    rho = f.sum()
    u = (C27 * f[:, None]).sum(0) / rho
    kap = orc.central_moments(f, u)
    feat = orc.closure_features(kap, 1.9)
    A, Q = _q_norm(kap)
    lam = np.linalg.eigvalsh(A)
    assert feat[0] == pytest.approx(lam.sum(), abs=1e-15)
    assert feat[1] == pytest.approx(lam[0] * lam[1] + lam[0] * lam[2] + lam[1] * lam[2],
                                    abs=1e-15)
    assert feat[2] == pytest.approx(np.prod(lam), abs=1e-16)
    assert feat[3] == pytest.approx(Q, rel=1e-13)
    assert feat[4] == pytest.approx(rho - 1, abs=1e-15)
    om = orc.smagorinsky_omega(kap, 1.9, 0.1)
    assert feat[5] == pytest.approx((1 / om - 1 / 1.9) / 3, rel=1e-12)


# ------------------------------------------------------------ closure network
def test_mlp_c_forward_matches_numpy(orc):
    rng = np.random.default_rng(12)
    blob = mlp_ref.init_blob(seed=3, mu=rng.normal(0, 1e-3, 6),
                             sigma=rng.uniform(0.5, 2.0, 6) * 1e-3, nu_scale=2e-3)
    feats = rng.normal(0, 2e-3, (64, 6))
    for emu in (False, True):
        ref, _ = mlp_ref.forward(blob, feats, emulate_bf16=emu)
        got = np.array([orc.mlp_nu_t(blob, x, emu) for x in feats])
        assert np.allclose(got, ref, rtol=1e-12, atol=1e-18)


def test_bf16_rounding_is_round_to_nearest_even(orc):
    # 1 + 2^-8 is a tie between 1 and 1 + 2^-7: even mantissa wins (1.0)
    assert orc.bf16_round(1.0 + 2.0 ** -8) == 1.0
    assert orc.bf16_round(1.0 + 3 * 2.0 ** -8) == 1.0 + 2.0 ** -6
    assert orc.bf16_round(1.0 + 2.0 ** -8 + 2.0 ** -20) == 1.0 + 2.0 ** -7
    assert mlp_ref.bf16(np.array([1.0 + 2.0 ** -8]))[0] == 1.0


def test_mlp_gradient_matches_finite_differences():
    rng = np.random.default_rng(13)
    blob = mlp_ref.init_blob(seed=5, mu=np.zeros(6), sigma=np.ones(6), nu_scale=1.0)
    X = rng.normal(0, 1, (16, 6))
    y = rng.uniform(0.1, 1.0, 16)
    L, g = mlp_ref.loss_and_grad(blob, X, y)
    h = 1e-6
    for k in rng.choice(mlp_ref.NPARAM, 60, replace=False).tolist() + [1312]:
        bp, bm = blob.copy(), blob.copy()
        bp[k] += h
        bm[k] -= h
        fd = (mlp_ref.loss_and_grad(bp, X, y)[0] - mlp_ref.loss_and_grad(bm, X, y)[0]) / (2 * h)
        assert g[k] == pytest.approx(fd, rel=1e-6, abs=1e-10), k


def test_adam_first_step_is_signed_lr():
    g = np.array([3.0, -0.5, 1e-3])
    p, m, v = mlp_ref.adam_step(np.zeros(3), g, np.zeros(3), np.zeros(3), 1, lr=0.01, eps=0.0)
    assert np.allclose(p, -0.01 * np.sign(g), rtol=1e-15)


# ------------------------------------------------------------ relaxation groups
# Reading of the cumulant collision (Sec. 2.1; the rates are not printed):
# which combination of cumulants each of omega_1..omega_10 relaxes. With one
# rate at 1/2 and every other rate at 1, every cumulant of order >= 2 goes to
# its equilibrium except the combination that rate names, which keeps half
# its pre-collision value. The cumulants on both sides come from the
# set-partition definition above, applied to the populations before and
# after the collision, not from the oracle's cumulant map.
def _all_cumulants(f, u):
    rho = f.sum()
    p, X = f / rho, C27 - u
    out = {}
    for m in range(27):
        a, b, c = m % 3, (m // 3) % 3, m // 9
        if a + b + c >= 2:
            out[(a, b, c)] = _joint_cumulant(p, X, [0] * a + [1] * b + [2] * c)
    return out


def _groups(C):
    """The combinations the rates act on, as named by the reading; each is
    a tuple of linear combinations of cumulants (equilibrium value 0 except
    the second-order trace, whose equilibrium is 1)."""
    g = {}
    g[1] = (C[(1, 1, 0)], C[(1, 0, 1)], C[(0, 1, 1)],
            C[(2, 0, 0)] - C[(0, 2, 0)], C[(2, 0, 0)] - C[(0, 0, 2)])
    g[2] = (C[(2, 0, 0)] + C[(0, 2, 0)] + C[(0, 0, 2)] - 1.0,)
    g[3] = (C[(1, 2, 0)] + C[(1, 0, 2)], C[(2, 1, 0)] + C[(0, 1, 2)], C[(2, 0, 1)] + C[(0, 2, 1)])
    g[4] = (C[(1, 2, 0)] - C[(1, 0, 2)], C[(2, 1, 0)] - C[(0, 1, 2)], C[(2, 0, 1)] - C[(0, 2, 1)])
    g[5] = (C[(1, 1, 1)],)
    g[6] = (C[(2, 2, 0)] - 2 * C[(2, 0, 2)] + C[(0, 2, 2)], C[(2, 2, 0)] + C[(2, 0, 2)] - 2 * C[(0, 2, 2)])
    g[7] = (C[(2, 2, 0)] + C[(2, 0, 2)] + C[(0, 2, 2)],)
    g[8] = (C[(2, 1, 1)], C[(1, 2, 1)], C[(1, 1, 2)])
    g[9] = (C[(2, 2, 1)], C[(2, 1, 2)], C[(1, 2, 2)])
    g[10] = (C[(2, 2, 2)],)
    return g


@pytest.mark.parametrize("k", range(1, 11))
def test_each_rate_relaxes_its_named_group(orc, k):
    """omega_k = 1/2, all other rates 1: the group of omega_k keeps half of
    its pre-collision value, every other group is at equilibrium. The ten
    groups hold 23 independent combinations of the 23 cumulants of orders
    2..6 (5+1+3+3+1+2+1+3+3+1), so together the ten cases fix the whole
    assignment: exchanging two rates (e.g. the sums and differences of third
    order, or the fourth-order trace and its differences) fails two of them."""
    rng = np.random.default_rng(100 + k)
    f = rand_pops(rng, rho=rng.uniform(0.9, 1.1), amp=0.45)
    rho = f.sum()
    u = (C27 * f[:, None]).sum(0) / rho
    om = np.ones(10)
    om[k - 1] = 0.5
    fo = orc.collide(f, [0.0, 0.0, 0.0], om)
    pre, post = _groups(_all_cumulants(f, u)), _groups(_all_cumulants(fo, u))
    assert max(abs(v) for v in pre[k]) > 1e-5  # the group is really excited (tolerance 3e-15)
    for g in range(1, 11):
        for a, b in zip(pre[g], post[g]):
            want = 0.5 * a if g == k else 0.0
            assert b == pytest.approx(want, abs=3e-15), (k, g)


def test_groups_cover_every_cumulant():
    """The 23 group combinations are linearly independent over the 23
    cumulants of orders 2..6, so the per-rate test above leaves no cumulant
    unconstrained."""
    keys = [(m % 3, (m // 3) % 3, m // 9) for m in range(27)]
    keys = [key for key in keys if sum(key) >= 2]
    rows = []
    for key in keys:
        C = {q: (1.0 if q == key else 0.0) for q in keys}
        rows.append(np.concatenate([np.array(v, dtype=float) for _, v in sorted(_groups(C).items())]))
    A = np.array(rows)
    A[:, 5] += 1.0  # the trace group's offset of -1 is not linear; remove it
    assert A.shape == (23, 23)
    assert np.linalg.matrix_rank(A) == 23


# ------------------------------------------------------------ inlet plane
def test_inflow_plane_linear_ramp_closed_form():
    """Frozen-box inlet (reading of the turbine-row inflow: a periodic box
    convected through the inlet, Taylor's hypothesis). For a box that is an
    affine ramp a + b s in the convected index s, the inlet at position
    p = advect t is mean + a + b p inside [0, lt - 1]; between the last slice
    and the wrap it interpolates towards slice 0; positions repeat with
    period lt; without a box it is the mean."""
    import oracle
    rng = np.random.default_rng(21)
    nz, ny, lt = 3, 4, 8
    mean = rng.normal(0, 1, (3, nz, ny))
    a = rng.normal(0, 1, (3, nz, ny))
    b = rng.normal(0, 1, (3, nz, ny))
    box = a[:, None] + b[:, None] * np.arange(lt)[None, :, None, None]
    adv = 0.25
    for p, want in ((0.0, mean + a), (2.25, mean + a + 2.25 * b), (5.0, mean + a + 5 * b),
                    (6.75, mean + a + 6.75 * b),
                    (7.5, mean + a + 0.5 * (7 * b)),          # half way from slice 7 back to slice 0
                    (lt + 2.25, mean + a + 2.25 * b),        # one period later
                    (3 * lt + 6.75, mean + a + 6.75 * b)):
        got = oracle.inflow_plane(mean, box, adv, p / adv)
        assert np.allclose(got, want, rtol=0, atol=1e-12), p
    assert np.array_equal(oracle.inflow_plane(mean, None, adv, 17.0), mean)


# ------------------------------------------------------------ network forward, hand-set weights
def _handset_blob(j, p, q, mu, sigma, b1, b2, b3, w1, w2, w3, nu_scale):
    """A network whose output depends on input feature j through hidden unit
    p of layer 1 and unit q of layer 2 only: W1[p][j] = w1, W2[q][p] = w2,
    w3[q] = w3; everything else zero."""
    blob = np.zeros(mlp_ref.NBLOB)
    s = mlp_ref.SL
    W1 = np.zeros((32, 6))
    W1[p, j] = w1
    W2 = np.zeros((32, 32))
    W2[q, p] = w2
    bb1, bb2, ww3 = np.zeros(32), np.zeros(32), np.zeros(32)
    bb1[p], bb2[q], ww3[q] = b1, b2, w3
    blob[s["W1"][0]] = W1.reshape(-1)
    blob[s["b1"][0]] = bb1
    blob[s["W2"][0]] = W2.reshape(-1)
    blob[s["b2"][0]] = bb2
    blob[s["w3"][0]] = ww3
    blob[s["b3"][0]] = b3
    blob[s["mu"][0]] = mu
    blob[s["sigma"][0]] = sigma
    blob[s["nu_scale"][0]] = nu_scale
    return blob


@pytest.mark.parametrize("j,p,q", [(0, 0, 0), (1, 7, 3), (2, 31, 30), (3, 5, 17), (4, 12, 12), (5, 20, 1)])
def test_mlp_forward_handset_closed_form(orc, j, p, q):
    """nu_t = nu_s softplus(w3 max(0, w2 max(0, w1 (x_j - mu_j)/sigma_j + b1) + b2) + b3)
    for the hand-set network, in both oracle modes (every value here is a
    short dyadic fraction, exact in bfloat16, so the emulating mode gives the
    same closed form). A transposed W1 or W2, a wrong hidden index, a dropped
    bias or a missing ReLU changes the result."""
    mu, sigma = np.full(6, 0.25), np.full(6, 0.5)   # 1/sigma = 2 exactly
    w1, w2, w3, b1, b2, b3, nus = 2.0, 0.5, 1.5, 0.5, 0.25, -1.0, 0.75
    blob = _handset_blob(j, p, q, mu, sigma, b1, b2, b3, w1, w2, w3, nus)
    for xj in (1.75, 0.5, -1.0, 0.25, 3.0):
        x = np.full(6, 4.0)       # the other features must not matter
        x[j] = xj
        xh = (xj - 0.25) / 0.5
        h1 = max(0.0, w1 * xh + b1)
        h2 = max(0.0, w2 * h1 + b2)
        z = w3 * h2 + b3
        want = nus * math.log1p(math.exp(z))
        for emu in (False, True):
            assert orc.mlp_nu_t(blob, x, emu) == pytest.approx(want, rel=1e-15), (xj, emu)
            nu, _ = mlp_ref.forward(blob, x[None, :], emulate_bf16=emu)
            assert nu[0] == pytest.approx(want, rel=1e-15), (xj, emu)
