// FP64 host post-processing: port spectra -> S*, S at a real reference
// impedance, Z_r, the overall Z0 of a 2-port and the phase delay
// (eqs. 1, 2, 5-8 and the ABCD step of Sec. II-A).
#include <cmath>
#include <complex>
#include <vector>

#include "../../include/fdtd.h"

namespace {

using cd = std::complex<double>;

struct Mat {
    int n;
    std::vector<cd> a;
    explicit Mat(int n_) : n(n_), a((size_t)n_ * n_, cd(0, 0)) {}
    cd &operator()(int r, int c) { return a[(size_t)r * n + c]; }
    cd operator()(int r, int c) const { return a[(size_t)r * n + c]; }
};

Mat mul(const Mat &x, const Mat &y)
{
    Mat z(x.n);
    for (int r = 0; r < x.n; ++r)
        for (int c = 0; c < x.n; ++c) {
            cd s = 0;
            for (int t = 0; t < x.n; ++t) s += x(r, t) * y(t, c);
            z(r, c) = s;
        }
    return z;
}

// Gauss-Jordan inverse with partial pivoting; false if singular.
bool inverse(const Mat &m, Mat &out)
{
    const int n = m.n;
    Mat a = m;
    out = Mat(n);
    for (int r = 0; r < n; ++r) out(r, r) = 1.0;
    for (int col = 0; col < n; ++col) {
        int piv = col;
        for (int r = col + 1; r < n; ++r)
            if (std::abs(a(r, col)) > std::abs(a(piv, col))) piv = r;
        if (!(std::abs(a(piv, col)) > 0)) return false;
        if (piv != col)
            for (int c = 0; c < n; ++c) {
                std::swap(a(piv, c), a(col, c));
                std::swap(out(piv, c), out(col, c));
            }
        const cd inv = 1.0 / a(col, col);
        for (int c = 0; c < n; ++c) {
            a(col, c) *= inv;
            out(col, c) *= inv;
        }
        for (int r = 0; r < n; ++r) {
            if (r == col) continue;
            const cd f = a(r, col);
            if (f == cd(0, 0)) continue;
            for (int c = 0; c < n; ++c) {
                a(r, c) -= f * a(col, c);
                out(r, c) -= f * out(col, c);
            }
        }
    }
    return true;
}

cd load(const double *p, size_t idx) { return cd(p[2 * idx], p[2 * idx + 1]); }
void store(double *p, size_t idx, cd v)
{
    p[2 * idx] = v.real();
    p[2 * idx + 1] = v.imag();
}

// wrap an angle difference into (-pi, pi]
double wrap(double d)
{
    const double two_pi = 2.0 * M_PI;
    double w = std::fmod(d + M_PI, two_pi);
    if (w < 0) w += two_pi;
    w -= M_PI;
    if (w == -M_PI && d > 0) w = M_PI;
    return w;
}

}  // namespace

extern "C" fdtd_status fdtd_sparams(int32_t np, int32_t nf, const double *f, const double *Vinc,
                                    const double *Iinc, const double *Vtot, double z_ref,
                                    double *S_star, double *S, double *Zr, double *Z0,
                                    double *tau)
{
    if (np < 1 || np > 16 || nf < 1 || !f || !Vinc || !Iinc || !Vtot || !(z_ref > 0))
        return FDTD_E_INVALID_ARG;
    const size_t N = (size_t)np;
    std::vector<cd> ss((size_t)nf * N * N), zr((size_t)nf * N);
    try {
        for (int k = 0; k < nf; ++k) {
            // eq. 2: reference impedance of each port from its incident run
            for (size_t j = 0; j < N; ++j) {
                const cd v = load(Vinc, j * nf + k), c = load(Iinc, j * nf + k);
                zr[k * N + j] = v / c;
            }
            // eq. 1
            for (size_t j = 0; j < N; ++j) {
                const cd vinc = load(Vinc, j * nf + k);
                for (size_t i = 0; i < N; ++i) {
                    const cd vt = load(Vtot, (j * N + i) * nf + k);
                    cd s;
                    if (i == j) s = (vt - vinc) / vinc;
                    else s = vt / vinc * std::sqrt(zr[k * N + j] / zr[k * N + i]);
                    ss[((size_t)k * N + i) * N + j] = s;
                }
            }
        }
        for (const cd &v : ss)
            if (!std::isfinite(v.real()) || !std::isfinite(v.imag())) return FDTD_E_DIVERGED;
        if (S_star)
            for (size_t q = 0; q < ss.size(); ++q) store(S_star, q, ss[q]);
        if (Zr)
            for (size_t q = 0; q < zr.size(); ++q) store(Zr, q, zr[q]);

        for (int k = 0; k < nf; ++k) {
            Mat Ss(np);
            for (size_t r = 0; r < N; ++r)
                for (size_t c = 0; c < N; ++c) Ss(r, c) = ss[((size_t)k * N + r) * N + c];
            const cd *z = &zr[k * N];
            if (S) {
                // eqs. 5-6 with B = (Z' - Zr)(Z' + conj Zr)^-1 (diagonal)
                std::vector<cd> B(N), A(N);
                for (size_t i = 0; i < N; ++i) {
                    B[i] = (z_ref - z[i]) / (z_ref + std::conj(z[i]));
                    const double g = 1.0 / std::sqrt(std::fabs(z[i].real()));
                    A[i] = std::sqrt(z_ref) * g * (1.0 - std::conj(B[i]));
                }
                Mat M(np), L(np);
                for (size_t r = 0; r < N; ++r)
                    for (size_t c = 0; c < N; ++c) {
                        M(r, c) = (r == c ? 1.0 : 0.0) - B[r] * Ss(r, c);
                        L(r, c) = Ss(r, c) - (r == c ? std::conj(B[r]) : cd(0, 0));
                    }
                Mat Mi(np);
                if (!inverse(M, Mi)) return FDTD_E_DIVERGED;
                Mat P = mul(L, Mi);
                for (size_t r = 0; r < N; ++r)
                    for (size_t c = 0; c < N; ++c)
                        store(S, ((size_t)k * N + r) * N + c, P(r, c) * std::conj(A[c]) / A[r]);
            }
            if (Z0 && np == 2) {
                // Kurokawa power waves at Zr -> Z, then ABCD -> sqrt(B/C)
                Mat Sp(np), IminusSp(np), Rhs(np);
                std::vector<double> F(N);
                for (size_t i = 0; i < N; ++i) F[i] = 1.0 / (2.0 * std::sqrt(std::fabs(z[i].real())));
                for (size_t r = 0; r < N; ++r)
                    for (size_t c = 0; c < N; ++c) {
                        Sp(r, c) = Ss(r, c) * F[c] / F[r];
                        IminusSp(r, c) = (r == c ? 1.0 : 0.0) - Sp(r, c);
                    }
                for (size_t r = 0; r < N; ++r)
                    for (size_t c = 0; c < N; ++c)
                        Rhs(r, c) = Sp(r, c) * z[c] + (r == c ? std::conj(z[r]) : cd(0, 0));
                Mat Inv(np);
                if (!inverse(IminusSp, Inv)) return FDTD_E_DIVERGED;
                Mat Z = mul(Inv, Rhs);
                const cd det = Z(0, 0) * Z(1, 1) - Z(0, 1) * Z(1, 0);
                const cd Bab = det / Z(1, 0), Cab = 1.0 / Z(1, 0);
                cd z0 = std::sqrt(Bab / Cab);
                if (z0.real() < 0) z0 = -z0;
                store(Z0, k, z0);
            }
        }
        if (tau) {
            for (size_t i = 0; i < N; ++i)
                for (size_t j = 0; j < N; ++j) {
                    std::vector<double> th(nf);
                    for (int k = 0; k < nf; ++k) {
                        const double a = std::arg(ss[((size_t)k * N + i) * N + j]);
                        th[k] = k == 0 ? a : th[k - 1] + wrap(a - std::arg(ss[((size_t)(k - 1) * N + i) * N + j]));
                    }
                    if (nf > 1) {
                        const double icpt = th[0] - f[0] * (th[1] - th[0]) / (f[1] - f[0]);
                        const double shift = 2.0 * M_PI * std::round(icpt / (2.0 * M_PI));
                        for (double &v : th) v -= shift;
                    }
                    for (int k = 0; k < nf; ++k)
                        tau[((size_t)k * N + i) * N + j] = i == j ? 0.0 : -th[k] / (2.0 * M_PI * f[k]);
                }
        }
    } catch (...) {
        return FDTD_E_NOMEM;
    }
    return FDTD_OK;
}
