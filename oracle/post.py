"""FP64 post-processing of port spectra into network parameters.

TEST INFRASTRUCTURE ONLY (part of the oracle).  Plain numpy, one frequency
at a time where that keeps the algebra readable.

Conventions (the paper leaves them open; these are the readings used
throughout):
  * spectra are DFTs with kernel exp(-j 2 pi f t) at the true sample times;
  * ports are numbered 0..N-1; ``Vinc[j]``/``Iinc[j]`` are the voltage and
    current spectra at port j in the run where port j drives a locally
    uniform line (the incident run); ``Vtot[j, i]`` is the voltage spectrum at
    port i in the run where port j drives the full circuit (the total run);
  * the principal square root is used in eq. 1; ``*`` in eq. 5 is read as the
    complex conjugate when applied to B and A and as "the 50 ohm quantity"
    for G* and Z_r*, and B's second factor is read as (Z' + conj(Z_r))^-1
    (the printed (Z' - Z_r)(Z' - Z_r)^-1 is the identity).
"""
from __future__ import annotations

import numpy as np


def reference_impedance(Vinc_port: np.ndarray, Iinc_port: np.ndarray) -> np.ndarray:
    """Eq. 2: Z_r(y_j, f) = F[V_inc] / F[I_inc] at the driving port."""
    return Vinc_port / Iinc_port


def s_star(Vinc: np.ndarray, Iinc: np.ndarray, Vtot: np.ndarray):
    """Eq. 1, power-mode scattering matrix under matched loads.

    Vinc, Iinc: [N, nf]; Vtot: [N (driving j), N (port i), nf].
    Returns S*[nf, N, N] and Z_r[nf, N].
    """
    N, nf = Vinc.shape
    Zr = reference_impedance(Vinc, Iinc).T          # [nf, N]
    S = np.zeros((nf, N, N), dtype=complex)
    for j in range(N):
        for i in range(N):
            if i == j:
                # reflected voltage = total - incident at the driving port
                S[:, i, j] = (Vtot[j, j] - Vinc[j]) / Vinc[j]
            else:
                S[:, i, j] = Vtot[j, i] / Vinc[j] * np.sqrt(Zr[:, j] / Zr[:, i])
    return S, Zr


def renormalize(S_star: np.ndarray, Zr: np.ndarray, z_new: float = 50.0) -> np.ndarray:
    """Eqs. 5-6: S referred to real reference impedances z_new.

    B = (Z' - Z_r)(Z' + conj Z_r)^-1, A = G'^-1 G (I - conj B),
    S = A^-1 (S* - conj B) (I - B S*)^-1 conj A, with G = diag(|Re Z_r|^-1/2),
    G' = diag(z_new^-1/2), Z' = diag(z_new).
    """
    nf, N, _ = S_star.shape
    out = np.zeros_like(S_star)
    I = np.eye(N)
    for f in range(nf):
        zr = Zr[f]
        B = np.diag((z_new - zr) / (z_new + np.conj(zr)))
        G = np.diag(1.0 / np.sqrt(np.abs(zr.real)))
        Gp_inv = np.diag(np.full(N, np.sqrt(z_new)))
        A = Gp_inv @ G @ (I - np.conj(B))
        Sf = S_star[f]
        out[f] = np.linalg.inv(A) @ (Sf - np.conj(B)) @ np.linalg.inv(I - B @ Sf) @ np.conj(A)
    return out


def z_from_power_waves(S_star: np.ndarray, Zr: np.ndarray) -> np.ndarray:
    """Impedance matrix from power-wave S with reference impedances Z_r
    (Kurokawa 1965): with F = diag(1/(2 sqrt|Re Z_r|)) and S_p = F^-1 S F,
    Z = (I - S_p)^-1 (S_p Z_r + conj Z_r)."""
    nf, N, _ = S_star.shape
    out = np.zeros_like(S_star)
    I = np.eye(N)
    for f in range(nf):
        zr = Zr[f]
        F = np.diag(1.0 / (2.0 * np.sqrt(np.abs(zr.real))))
        Sp = np.linalg.inv(F) @ S_star[f] @ F
        out[f] = np.linalg.inv(I - Sp) @ (Sp @ np.diag(zr) + np.diag(np.conj(zr)))
    return out


def power_waves_from_z(Z: np.ndarray, zref: np.ndarray) -> np.ndarray:
    """Power-wave S of an impedance matrix for reference impedances zref
    (Kurokawa 1965): S = F (Z - conj Zref)(Z + Zref)^-1 F^-1."""
    nf, N, _ = Z.shape
    out = np.zeros_like(Z)
    for f in range(nf):
        zr = zref[f]
        F = np.diag(1.0 / (2.0 * np.sqrt(np.abs(zr.real))))
        out[f] = F @ (Z[f] - np.diag(np.conj(zr))) @ np.linalg.inv(Z[f] + np.diag(zr)) @ np.linalg.inv(F)
    return out


def abcd_from_z(Z: np.ndarray) -> np.ndarray:
    """Two-port ABCD from Z (Pozar): A = Z11/Z21, B = det Z / Z21,
    C = 1/Z21, D = Z22/Z21."""
    z11, z12, z21, z22 = Z[:, 0, 0], Z[:, 0, 1], Z[:, 1, 0], Z[:, 1, 1]
    det = z11 * z22 - z12 * z21
    out = np.zeros_like(Z)
    out[:, 0, 0] = z11 / z21
    out[:, 0, 1] = det / z21
    out[:, 1, 0] = 1.0 / z21
    out[:, 1, 1] = z22 / z21
    return out


def characteristic_impedance(S_star: np.ndarray, Zr: np.ndarray) -> np.ndarray:
    """Overall Z0 of a 2-port through its ABCD matrix (Sec. II-A, last
    paragraph): Z0 = sqrt(B/C), principal branch (Re Z0 >= 0)."""
    T = abcd_from_z(z_from_power_waves(S_star, Zr))
    z0 = np.sqrt(T[:, 0, 1] / T[:, 1, 0])
    return np.where(z0.real < 0, -z0, z0)


def phase_delay(S_ij: np.ndarray, freqs: np.ndarray) -> np.ndarray:
    """Eq. 8: delay from the unwrapped phase of a transmission entry.

    The phase is unwrapped with period 2 pi along the frequency grid; the
    remaining free multiple of 2 pi is fixed by asking the straight line
    through the two lowest frequencies to pass closest to zero phase at
    f = 0 (a pure delay has zero phase at DC).  With the exp(-j 2 pi f t)
    kernel a delay gives a negative phase slope, so tau = -theta / (2 pi f)
    (the magnitude of the printed theta / (360 f) with theta in degrees)."""
    theta = np.unwrap(np.angle(S_ij))
    if len(freqs) > 1:
        f0, f1 = freqs[0], freqs[1]
        intercept = theta[0] - f0 * (theta[1] - theta[0]) / (f1 - f0)
        theta = theta - 2.0 * np.pi * np.round(intercept / (2.0 * np.pi))
    return -theta / (2.0 * np.pi * freqs)


def lossless_line_s(gamma: np.ndarray, kappa: np.ndarray):
    """Eq. 7 for a uniform lossless line between mismatched references:
    S11 = (1 - kappa^2) Gamma / (1 - kappa^2 Gamma^2),
    S21 = (1 - Gamma^2) kappa / (1 - kappa^2 Gamma^2)
    (the printed S21 numerator (1 - kappa^2) kappa is read as
    (1 - Gamma^2) kappa), kappa = exp(-j beta l) for the exp(-j 2 pi f t)
    kernel."""
    den = 1.0 - kappa ** 2 * gamma ** 2
    return (1.0 - kappa ** 2) * gamma / den, (1.0 - gamma ** 2) * kappa / den


def sparams(freqs, Vinc, Iinc, Vtot, z_ref=50.0):
    """The whole post-processing chain: S*, S at z_ref, Z_r, Z0 (2-ports)
    and the phase delay of every off-diagonal S* entry."""
    Ss, Zr = s_star(Vinc, Iinc, Vtot)
    S = renormalize(Ss, Zr, z_ref)
    N = Ss.shape[1]
    Z0 = characteristic_impedance(Ss, Zr) if N == 2 else None
    tau = np.zeros(Ss.shape, dtype=float)
    for i in range(N):
        for j in range(N):
            if i != j:
                tau[:, i, j] = phase_delay(Ss[:, i, j], freqs)
    return {"S_star": Ss, "S": S, "Zr": Zr, "Z0": Z0, "tau": tau}


def single_excitation_protocol(V: np.ndarray, I: np.ndarray):
    """Protocol arrays for a uniform, mirror-symmetric 2-port simulated once,
    driven at port 0 (V, I: [2, nf] spectra of that run).

    On a uniform line the incident and total runs coincide.  The run driven
    at port 1 is the mirror image of the run driven at port 0, so port 1 sees
    in it what port 0 sees in the simulated run and vice versa."""
    Vinc = np.stack([V[0], V[0]])
    Iinc = np.stack([I[0], I[0]])
    Vtot = np.stack([np.stack([V[0], V[1]]), np.stack([V[1], V[0]])])
    return Vinc, Iinc, Vtot


def protocol_from_runs(spectra):
    """Spectra of the four runs of the per-port protocol (Sec. II-A) in the
    arrangement ``sparams`` takes.  ``spectra`` maps "inc1", "inc2", "tot1",
    "tot2" to (V[probe, f], I[probe, f]) with probe 0 = port 1, 1 = port 2.
    Vinc[j], Iinc[j]: port j in the run driving port j on its uniform line;
    Vtot[j, i]: port i in the full-circuit run driven at port j."""
    V1, I1 = spectra["inc1"]
    V2, I2 = spectra["inc2"]
    T1, _ = spectra["tot1"]
    T2, _ = spectra["tot2"]
    Vinc = np.stack([V1[0], V2[1]])
    Iinc = np.stack([I1[0], I2[1]])
    Vtot = np.stack([np.stack([T1[0], T1[1]]), np.stack([T2[0], T2[1]])])
    return Vinc, Iinc, Vtot
