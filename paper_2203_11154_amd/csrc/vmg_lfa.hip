// Local Fourier analysis of the smoothers on the host (Sec. 2.1): the complex
// relaxation weight omega that minimises the smoothing factor mu_loc of
// eq. (4), for the complex relaxation parameter the paper leaves as future
// work after Example 3.
//
// With every symbol scaled by h^2, the smoothing symbol of eq. (7) is
//   S(theta) = 1 - omega s(theta),   s = M(theta) L(theta),
//   L = 4 + eta - 2 cos t1 - 2 cos t2,
//   M = a + b (cos t1 + cos t2) + c cos t1 cos t2        (Vanka, eq. (6))
//   M = 1 / (4 + eta)                                    (point Jacobi),
// with eta = lambda h^2.  Both depend on theta only through c_i = cos t_i,
// and the high frequencies [-pi/2, 3pi/2)^2 minus [-pi/2, pi/2)^2 are exactly
// the points with c1 <= 0 or c2 <= 0; since s is symmetric in (c1, c2), the
// rectangle c1 in [-1, 0], c2 in [-1, 1] covers them.  It is sampled on a
// uniform grid.
//
// mu(omega) = max_k |1 - omega s_k| is a maximum of moduli of affine
// functions of omega, hence convex in (Re omega, Im omega).  |1 - omega s| is
// convex in s as well, so the maximum over the samples is attained at a
// vertex of their convex hull: the hull (monotone chain) replaces the samples.
// The minimum is found by the central-cut ellipsoid method (Shor; Nemirovski
// and Yudin; Khachiyan), which needs only a subgradient and converges for
// any convex function; it starts from a disk that contains every omega with
// mu < 1: |1 - omega s_K| < 1 puts omega within 1/|s_K| of 1/s_K, and the
// sample of largest modulus gives the smallest such disk.
#include "../../include/vanka_mg.h"

#include <algorithm>
#include <cmath>
#include <complex>
#include <thread>
#include <vector>

namespace {

using cd = std::complex<double>;

constexpr int NC1 = 193;  // samples of c1 in [-1, 0]
constexpr int NC2 = 385;  // samples of c2 in [-1, 1] (the same spacing)
constexpr int ELLIPSOID_STEPS = 400;

// Convex hull (counter-clockwise, no collinear points) of points in the plane.
std::vector<cd> convex_hull(std::vector<cd> p) {
    std::sort(p.begin(), p.end(), [](const cd& u, const cd& v) {
        return u.real() < v.real() || (u.real() == v.real() && u.imag() < v.imag());
    });
    p.erase(std::unique(p.begin(), p.end()), p.end());
    if (p.size() < 3) return p;
    auto cross = [](const cd& o, const cd& a, const cd& b) {
        return (a.real() - o.real()) * (b.imag() - o.imag()) - (a.imag() - o.imag()) * (b.real() - o.real());
    };
    std::vector<cd> h(2 * p.size());
    size_t k = 0;
    for (size_t i = 0; i < p.size(); ++i) {
        while (k >= 2 && cross(h[k - 2], h[k - 1], p[i]) <= 0) --k;
        h[k++] = p[i];
    }
    for (size_t i = p.size() - 1, t = k + 1; i-- > 0;) {
        while (k >= t && cross(h[k - 2], h[k - 1], p[i]) <= 0) --k;
        h[k++] = p[i];
    }
    h.resize(k - 1);
    return h;
}

// Hull of the high-frequency samples s = M L for one eta.
std::vector<cd> symbol_hull(cd eta, int smoother) {
    cd a, b, c;
    if (smoother == 1) {
        a = 1.0 / (4.0 + eta);
        b = c = 0.0;
    } else {
        const cd den = (2.0 + eta) * (4.0 + eta) * (6.0 + eta);
        a = (14.0 + 8.0 * eta + eta * eta) / den;
        b = 1.0 / ((2.0 + eta) * (6.0 + eta));
        c = 2.0 / den;
    }
    std::vector<cd> s;
    s.reserve((size_t)NC1 * NC2);
    for (int i = 0; i < NC1; ++i) {
        const double c1 = -1.0 + (double)i / (NC1 - 1);
        for (int j = 0; j < NC2; ++j) {
            const double c2 = -1.0 + 2.0 * j / (NC2 - 1);
            const cd l = 4.0 + eta - 2.0 * c1 - 2.0 * c2;
            const cd m = a + b * (c1 + c2) + c * (c1 * c2);
            s.push_back(m * l);
        }
    }
    return convex_hull(std::move(s));
}

// mu(omega) over the hull vertices; g receives a subgradient with respect to
// (Re omega, Im omega) (the gradient of the largest term).
double mu_at(const std::vector<cd>& v, cd w, double g[2]) {
    double best = -1.0;
    size_t kb = 0;
    for (size_t k = 0; k < v.size(); ++k) {
        const double f = std::abs(1.0 - w * v[k]);
        if (f > best) {
            best = f;
            kb = k;
        }
    }
    const cd u = 1.0 - w * v[kb];
    if (best > 0.0) {
        // d|u|/dx = Re(conj(u) du/dx) / |u|, du/dx = -s, du/dy = -i s
        g[0] = std::real(std::conj(u) * (-v[kb])) / best;
        g[1] = std::real(std::conj(u) * (cd(0.0, -1.0) * v[kb])) / best;
    } else {
        g[0] = g[1] = 0.0;
    }
    return best;
}

void optimise(cd eta, int smoother, cd* omega, double* mu) {
    const std::vector<cd> v = symbol_hull(eta, smoother);
    size_t kmax = 0;
    for (size_t k = 1; k < v.size(); ++k)
        if (std::abs(v[k]) > std::abs(v[kmax])) kmax = k;
    double g[2];
    cd best_w = 1.0;
    double best_f = mu_at(v, best_w, g);
    if (std::abs(v[kmax]) == 0.0) {
        *omega = best_w;
        *mu = best_f;
        return;
    }
    // ellipsoid {x : (x - c)^T P^{-1} (x - c) <= 1} in (Re, Im)
    const cd c0 = 1.0 / v[kmax];
    double cx = c0.real(), cy = c0.imag();
    const double r = 1.01 / std::abs(v[kmax]);
    double p00 = r * r, p01 = 0.0, p11 = r * r;
    for (int it = 0; it < ELLIPSOID_STEPS; ++it) {
        const double f = mu_at(v, cd(cx, cy), g);
        if (f < best_f) {
            best_f = f;
            best_w = cd(cx, cy);
        }
        const double q0 = p00 * g[0] + p01 * g[1], q1 = p01 * g[0] + p11 * g[1];  // P g
        const double gpg = g[0] * q0 + g[1] * q1;
        if (!(gpg > 0.0)) break;
        const double sc = 1.0 / std::sqrt(gpg);
        const double b0 = q0 * sc, b1 = q1 * sc;  // P g / sqrt(g^T P g)
        // n = 2: c -= b / 3,  P = 4/3 (P - 2/3 b b^T)
        cx -= b0 / 3.0;
        cy -= b1 / 3.0;
        p00 = 4.0 / 3.0 * (p00 - 2.0 / 3.0 * b0 * b0);
        p01 = 4.0 / 3.0 * (p01 - 2.0 / 3.0 * b0 * b1);
        p11 = 4.0 / 3.0 * (p11 - 2.0 / 3.0 * b1 * b1);
    }
    *omega = best_w;
    *mu = best_f;
}

}  // namespace

extern "C" int vanka_mg_lfa_omega(const double* eta, int32_t count, int32_t smoother, double* omega, double* mu) {
    if (!eta || !omega || count < 0 || smoother < 0 || smoother > 1) return VMG_INVALID_ARG;
    // independent problems: split over host threads (each writes its own
    // entries)
    auto work = [&](int32_t k0, int32_t k1) {
        for (int32_t k = k0; k < k1; ++k) {
            cd w;
            double m;
            optimise(cd(eta[2 * k], eta[2 * k + 1]), smoother, &w, &m);
            omega[2 * k] = w.real();
            omega[2 * k + 1] = w.imag();
            if (mu) mu[k] = m;
        }
    };
    const int32_t nt =
        std::max<int32_t>(1, std::min<int32_t>({count / 4, 16, (int32_t)std::thread::hardware_concurrency()}));
    auto lo = [&](int32_t t) { return (int32_t)((int64_t)count * t / nt); };
    // ranges 1.. on their own threads, range 0 here; a range whose thread
    // cannot start runs here as well (nothing may throw across the C ABI)
    std::vector<std::thread> pool;
    int32_t started = 1;
    try {
        for (; started < nt; ++started) pool.emplace_back(work, lo(started), lo(started + 1));
    } catch (...) {
    }
    work(lo(0), lo(1));
    for (int32_t t = started; t < nt; ++t) work(lo(t), lo(t + 1));
    for (auto& th : pool) th.join();
    return VMG_OK;
}
