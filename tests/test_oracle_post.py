"""Pins of the oracle's post-processing (eqs. 1, 2, 5-8 and the ABCD step)
against independent derivations and closed forms."""
import numpy as np
import pytest

from oracle import post


def _rand_net(rng, N, nf=5):
    S = (rng.normal(size=(nf, N, N)) + 1j * rng.normal(size=(nf, N, N))) * 0.3
    Zr = rng.uniform(5, 300, size=(nf, N)) + 1j * rng.uniform(-80, 80, size=(nf, N))
    return S, Zr


@pytest.mark.parametrize("N", [1, 2, 3])
def test_renormalization_equals_power_wave_route(N):
    """Eq. 5 (as read) equals going through the impedance matrix: Z from the
    power waves at Z_r, then power waves at 50 ohm (Kurokawa)."""
    rng = np.random.default_rng(11 + N)
    S, Zr = _rand_net(rng, N)
    a = post.renormalize(S, Zr, 50.0)
    Z = post.z_from_power_waves(S, Zr)
    b = post.power_waves_from_z(Z, np.full(Zr.shape, 50.0 + 0j))
    assert np.max(np.abs(a - b)) < 1e-12


def test_renormalization_printed_b_is_identity():
    """The printed B = (Z' - Z_r)(Z' - Z_r)^-1 is the identity, which makes
    eq. 5 singular (I - B S* with B = I); the conjugate-sum reading is the
    one that agrees with the power-wave route above."""
    zr = np.array([30.0 + 5j, 70.0 - 2j])
    zp = np.array([50.0, 50.0])
    B_printed = np.diag(zp - zr) @ np.linalg.inv(np.diag(zp - zr))
    assert np.allclose(B_printed, np.eye(2))


def test_renormalization_to_own_reference_is_identity():
    rng = np.random.default_rng(5)
    S, _ = _rand_net(rng, 2)
    Zr = np.full((S.shape[0], 2), 50.0 + 0j)
    assert np.max(np.abs(post.renormalize(S, Zr, 50.0) - S)) < 1e-14


def test_uniform_25_ohm_line_gives_eq7():
    """A reflectionless 25 ohm line (S* = [[0, k], [k, 0]]) referred to 50
    ohm reproduces eq. 7 with Gamma = -1/3 and kappa = exp(-j beta l)."""
    bl = np.linspace(0.1, 9.0, 40)
    kappa = np.exp(-1j * bl)
    S_star = np.zeros((bl.size, 2, 2), complex)
    S_star[:, 0, 1] = S_star[:, 1, 0] = kappa
    Zr = np.full((bl.size, 2), 25.0 + 0j)
    S = post.renormalize(S_star, Zr, 50.0)
    s11, s21 = post.lossless_line_s(-1.0 / 3.0, kappa)
    assert np.max(np.abs(S[:, 0, 0] - s11)) < 1e-14
    assert np.max(np.abs(S[:, 1, 0] - s21)) < 1e-14
    assert np.max(np.abs(S[:, 1, 1] - s11)) < 1e-14
    # the printed numerator (1 - kappa^2) kappa is not what the algebra gives
    printed = (1 - kappa ** 2) * kappa / (1 - kappa ** 2 / 9.0)
    assert np.max(np.abs(S[:, 1, 0] - printed)) > 0.1


def test_abcd_of_uniform_line():
    """ABCD of a matched uniform line (Pozar): A = D = cos bl,
    B = j Zc sin bl, C = j sin bl / Zc, so Z0 = sqrt(B/C) = Zc."""
    bl = np.linspace(0.2, 3.0, 15)
    zc = 37.5
    S_star = np.zeros((bl.size, 2, 2), complex)
    S_star[:, 0, 1] = S_star[:, 1, 0] = np.exp(-1j * bl)
    Zr = np.full((bl.size, 2), zc + 0j)
    T = post.abcd_from_z(post.z_from_power_waves(S_star, Zr))
    assert np.max(np.abs(T[:, 0, 0] - np.cos(bl))) < 1e-12
    assert np.max(np.abs(T[:, 0, 1] - 1j * zc * np.sin(bl))) < 1e-11
    assert np.max(np.abs(T[:, 1, 0] - 1j * np.sin(bl) / zc)) < 1e-12
    assert np.max(np.abs(post.characteristic_impedance(S_star, Zr) - zc)) < 1e-11


def test_phase_delay_of_pure_delay():
    f = np.linspace(10e12, 300e12, 64)
    tau = 12.4e-15
    s21 = 0.8 * np.exp(-2j * np.pi * f * tau)
    f2 = np.linspace(60e12, 300e12, 64)
    # on f2 the lowest frequency already carries more than half a turn
    assert 2 * np.pi * f2[0] * tau > np.pi
    for ff in (f, f2):
        got = post.phase_delay(0.8 * np.exp(-2j * np.pi * ff * tau), ff)
        assert np.max(np.abs(got / tau - 1)) < 1e-12


def test_s_star_protocol_on_synthetic_spectra():
    """Eq. 1 and eq. 2 on spectra built from a known 2-port: port j driven
    with incident a_j, reflection r_j, transmission t."""
    nf = 7
    rng = np.random.default_rng(3)
    a = rng.normal(size=(2, nf)) + 1j * rng.normal(size=(2, nf))
    z = np.array([20.0 + 3j, 45.0 - 1j])
    r = np.array([0.2 - 0.1j, -0.3j])
    t = 0.7 * np.exp(-0.5j)
    Vinc = a.copy()
    Iinc = a / z[:, None]
    Vtot = np.zeros((2, 2, nf), complex)
    for j in range(2):
        i = 1 - j
        Vtot[j, j] = a[j] * (1 + r[j])
        # transmitted voltage such that the power-normalized transmission is t
        Vtot[j, i] = t * a[j] * np.sqrt(z[i] / z[j])
    S, Zr = post.s_star(Vinc, Iinc, Vtot)
    assert np.allclose(Zr, np.broadcast_to(z, (nf, 2)))
    assert np.allclose(S[:, 0, 0], r[0]) and np.allclose(S[:, 1, 1], r[1])
    assert np.allclose(S[:, 1, 0], t) and np.allclose(S[:, 0, 1], t)
