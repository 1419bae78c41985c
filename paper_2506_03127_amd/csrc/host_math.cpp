// Host-side tables of the path propagation: the short-time propagator
// U = exp(-i H dt) (eq. SysP) and the influence coefficients eta (eq. inf_fun).
//
// U comes from a cyclic Jacobi eigendecomposition of the real symmetric
// 2M x 2M embedding [[Re H, -Im H], [Im H, Re H]] of the Hermitian H: real
// functions of H embed as the same functions of the embedding, so
// cos(H dt) and sin(H dt) are read off its first block column and
// U = cos(H dt) - i sin(H dt).
//
// eta: the window integrals of the bath response alpha(t) (the explicit forms
// are only cited in Sec. 2), written through g(t) = int_0^t int_0^t' alpha:
//   interior x interior, lag d >= 1 : g((d+1)dt) - 2 g(d dt) + g((d-1)dt)
//   interior self                   : g(dt)
//   end point x interior, lag d     : g(d dt + h) - g(d dt) - g(d dt - h) + g((d-1)dt)
//   end point self                  : g(h)
//   initial x final, lag d          : g(d dt) - 2 g(d dt - h) + g((d-1)dt),     h = dt/2.
// g is evaluated as
//   Re g(t) = (1/pi) int_0^inf J/w^2 coth(beta w/2) 2 sin^2(w t/2) dw
//   Im g(t) = (1/pi) int_0^inf J/w^2 sin(w t) dw  -  lambda t,
// with lambda = (1/pi) int J/w dw in closed form (alpha wc/2 for the Ohmic
// part, lam for each peak).  The integrals use 16-point Gauss-Legendre panels
// on [0, W]: panels no wider than a quarter period of w t, refined around each
// peak; beyond W only the t-independent part of Re g is kept (its oscillating
// part and that of Im g are below 1e-16 there), integrated in u = 1/w.

#include <cmath>
#include <cstring>
#include <vector>
#include <algorithm>

#include "host_math.h"

namespace quapi_host {

// ------------------------------------------------------------------ Jacobi
// Eigen-decomposition of a real symmetric n x n matrix A (row-major, destroyed),
// n <= kJacobiMax.  On return d[k] are the eigenvalues and column k of V the
// eigenvectors.  Works in the caller's arrays: no heap memory.
constexpr int kJacobiMax = 16;

static void jacobi_symmetric(double* A, int n, double* d, double* V) {
    for (int i = 0; i < n * n; ++i) V[i] = 0.0;
    for (int i = 0; i < n; ++i) V[i * n + i] = 1.0;
    double scale = 0.0;
    for (int i = 0; i < n * n; ++i) scale = std::max(scale, std::fabs(A[i]));
    if (scale == 0.0) scale = 1.0;
    for (int sweep = 0; sweep < 100; ++sweep) {
        double off = 0.0;
        for (int i = 0; i < n; ++i)
            for (int j = i + 1; j < n; ++j) off += A[i * n + j] * A[i * n + j];
        if (std::sqrt(off) <= 1e-300 + 1e-17 * scale) break;
        for (int p = 0; p < n; ++p) {
            for (int q = p + 1; q < n; ++q) {
                const double apq = A[p * n + q];
                if (apq == 0.0) continue;
                const double app = A[p * n + p], aqq = A[q * n + q];
                const double theta = (aqq - app) / (2.0 * apq);
                const double t = (theta >= 0 ? 1.0 : -1.0) /
                                 (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
                const double c = 1.0 / std::sqrt(t * t + 1.0), s = t * c;
                for (int k = 0; k < n; ++k) {      // A <- A J  (columns p, q)
                    const double akp = A[k * n + p], akq = A[k * n + q];
                    A[k * n + p] = c * akp - s * akq;
                    A[k * n + q] = s * akp + c * akq;
                }
                for (int k = 0; k < n; ++k) {      // A <- J^T A  (rows p, q)
                    const double apk = A[p * n + k], aqk = A[q * n + k];
                    A[p * n + k] = c * apk - s * aqk;
                    A[q * n + k] = s * apk + c * aqk;
                }
                for (int k = 0; k < n; ++k) {      // V <- V J
                    const double vkp = V[k * n + p], vkq = V[k * n + q];
                    V[k * n + p] = c * vkp - s * vkq;
                    V[k * n + q] = s * vkp + c * vkq;
                }
            }
        }
    }
    for (int i = 0; i < n; ++i) d[i] = A[i * n + i];
}

bool hermitian_ok(int M, const double* H /* 2*M*M */) {
    double mx = 1.0;
    for (int i = 0; i < M * M; ++i) mx = std::max(mx, std::hypot(H[2 * i], H[2 * i + 1]));
    for (int i = 0; i < M; ++i)
        for (int j = 0; j < M; ++j) {
            const double dre = H[2 * (i * M + j)] - H[2 * (j * M + i)];
            const double dim = H[2 * (i * M + j) + 1] + H[2 * (j * M + i) + 1];
            if (!(std::hypot(dre, dim) <= 1e-12 * mx)) return false;
        }
    return true;
}

// U = exp(-i H dt) for M <= 8, from the real symmetric 2M x 2M form of H
// (no heap memory)
void propagator(int M, const double* H, double dt, double* U /* 2*M*M */) {
    const int n = 2 * M;
    double S[kJacobiMax * kJacobiMax] = {}, d[kJacobiMax], V[kJacobiMax * kJacobiMax];
    for (int i = 0; i < M; ++i)
        for (int j = 0; j < M; ++j) {
            const double re = H[2 * (i * M + j)], im = H[2 * (i * M + j) + 1];
            S[i * n + j] = re;
            S[(i + M) * n + (j + M)] = re;
            S[i * n + (j + M)] = -im;
            S[(i + M) * n + j] = im;
        }
    jacobi_symmetric(S, n, d, V);
    for (int i = 0; i < M; ++i)
        for (int j = 0; j < M; ++j) {
            double c_re = 0, c_im = 0, s_re = 0, s_im = 0;
            for (int k = 0; k < n; ++k) {
                const double ck = std::cos(d[k] * dt), sk = std::sin(d[k] * dt);
                const double top = V[i * n + k] * V[j * n + k];        // block (i, j)
                const double bot = V[(i + M) * n + k] * V[j * n + k];  // block (i+M, j)
                c_re += ck * top;
                c_im += ck * bot;
                s_re += sk * top;
                s_im += sk * bot;
            }
            // U = cos(H dt) - i sin(H dt)
            U[2 * (i * M + j)] = c_re + s_im;
            U[2 * (i * M + j) + 1] = c_im - s_re;
        }
}

// ------------------------------------------------------------------ eta
namespace {

struct GaussLegendre {
    double x[16], w[16];
    GaussLegendre() {
        const int n = 16;
        for (int i = 0; i < n; ++i) {
            double z = std::cos(M_PI * (i + 0.75) / (n + 0.5));
            for (int it = 0; it < 100; ++it) {
                double p0 = 1.0, p1 = 0.0;
                for (int k = 1; k <= n; ++k) {
                    const double p2 = p1;
                    p1 = p0;
                    p0 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p2) / k;
                }
                const double dp = n * (z * p0 - p1) / (z * z - 1.0);
                const double dz = p0 / dp;
                z -= dz;
                if (std::fabs(dz) < 1e-16) {
                    x[i] = z;
                    w[i] = 2.0 / ((1.0 - z * z) * dp * dp);
                    break;
                }
                x[i] = z;
                w[i] = 2.0 / ((1.0 - z * z) * dp * dp);
            }
        }
    }
};

struct Spectral {
    double alpha, wc;
    std::vector<double> w0, gam, lam;
    double J(double w) const {
        double j = 0.0;
        if (alpha != 0.0) j += 0.5 * M_PI * alpha * w * std::exp(-w / wc);
        for (size_t k = 0; k < w0.size(); ++k) {
            const double a = w0[k] * w0[k] - w * w;
            j += 2.0 * lam[k] * gam[k] * w0[k] * w0[k] * w / (a * a + gam[k] * gam[k] * w * w);
        }
        return j;
    }
    double lambda_total() const {
        double l = 0.5 * alpha * wc;
        for (double x : lam) l += x;
        return l;
    }
};

template <class F>
double panels(const std::vector<double>& edges, const GaussLegendre& gl, F f) {
    double tot = 0.0;
    for (size_t e = 0; e + 1 < edges.size(); ++e) {
        const double a = edges[e], b = edges[e + 1], h = 0.5 * (b - a), m = 0.5 * (a + b);
        double s = 0.0;
        for (int i = 0; i < 16; ++i) s += gl.w[i] * f(m + h * gl.x[i]);
        tot += h * s;
    }
    return tot;
}

}  // namespace

int eta_columns(double ohmic_alpha, double ohmic_wc, int n_peaks, const double* peaks,
                double beta, double dt, int K, double* eta /* 2*3*(K+1) */) {
    Spectral sp;
    sp.alpha = ohmic_alpha;
    sp.wc = ohmic_wc;
    for (int k = 0; k < n_peaks; ++k) {
        sp.w0.push_back(peaks[3 * k]);
        sp.gam.push_back(peaks[3 * k + 1]);
        sp.lam.push_back(peaks[3 * k + 2]);
    }
    const GaussLegendre gl;
    const double tmax = (K + 1) * dt;

    // panel edges on [0, W]
    double W = 50.0;
    if (sp.alpha != 0.0) W = std::max(W, 80.0 * sp.wc);
    for (size_t k = 0; k < sp.w0.size(); ++k) W = std::max(W, std::max(400.0, 20.0 * sp.w0[k]));
    const double width = std::min(0.25, 0.5 * M_PI / std::max(tmax, 1e-6));   // <= quarter period
    std::vector<double> edges;
    for (double x = 0.0; x < W; x += width) edges.push_back(x);
    for (size_t k = 0; k < sp.w0.size(); ++k) {
        const double g = sp.gam[k], c = sp.w0[k];
        for (double s = -60.0; s <= 60.0; s += 0.25) {
            const double x = c + s * g;
            if (x > 0.0 && x < W) edges.push_back(x);
        }
    }
    edges.push_back(W);
    std::sort(edges.begin(), edges.end());
    edges.erase(std::unique(edges.begin(), edges.end(),
                            [](double a, double b) { return std::fabs(a - b) < 1e-12; }),
                edges.end());

    // t-independent part of Re g beyond W, in u = 1/w on (0, 1/W]
    std::vector<double> uedges;
    for (int i = 0; i <= 64; ++i) uedges.push_back((1.0 / W) * i / 64.0);
    const double re_tail = panels(uedges, gl, [&](double u) {
        if (u <= 0.0) return 0.0;
        const double w = 1.0 / u;
        // int_W^inf J/w^2 coth(beta w/2) dw = int_0^{1/W} J(1/u) coth(beta/(2u)) du
        return sp.J(w) / std::tanh(0.5 * beta * w);
    });
    const double lam_tot = sp.lambda_total();

    auto g = [&](double t, double* gre, double* gim) {
        if (t == 0.0) { *gre = 0.0; *gim = 0.0; return; }
        const double re = panels(edges, gl, [&](double w) {
            if (w <= 0.0) return 0.0;
            const double s = std::sin(0.5 * w * t);
            return sp.J(w) / (w * w) * 2.0 * s * s / std::tanh(0.5 * beta * w);
        });
        const double im = panels(edges, gl, [&](double w) {
            if (w <= 0.0) return 0.0;
            return sp.J(w) / (w * w) * std::sin(w * t);
        });
        // the oscillating part of the Re tail averages out; the constant part
        // (1 - cos -> 1) is the integral computed above
        *gre = (re + re_tail) / M_PI;
        *gim = im / M_PI - lam_tot * t;
    };

    const int nh = 2 * K + 3;   // g on the half-step grid, j*dt/2
    std::vector<double> Gr(nh), Gi(nh);
    for (int j = 0; j < nh; ++j) g(0.5 * dt * j, &Gr[j], &Gi[j]);
    const int n = K + 1;
    auto put = [&](int col, int d, double re, double im) {
        eta[2 * (col * n + d)] = re;
        eta[2 * (col * n + d) + 1] = im;
    };
    put(0, 0, Gr[2], Gi[2]);
    put(1, 0, Gr[1], Gi[1]);
    put(2, 0, Gr[1], Gi[1]);
    for (int d = 1; d <= K; ++d) {
        const int a = 2 * d;
        put(0, d, Gr[a + 2] - 2.0 * Gr[a] + Gr[a - 2], Gi[a + 2] - 2.0 * Gi[a] + Gi[a - 2]);
        put(1, d, Gr[a + 1] - Gr[a] - Gr[a - 1] + Gr[a - 2], Gi[a + 1] - Gi[a] - Gi[a - 1] + Gi[a - 2]);
        put(2, d, Gr[a] - 2.0 * Gr[a - 1] + Gr[a - 2], Gi[a] - 2.0 * Gi[a - 1] + Gi[a - 2]);
    }
    return 0;
}

}  // namespace quapi_host
