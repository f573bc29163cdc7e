"""Local and rigorous Fourier analysis of the Vanka and Jacobi smoothers
(Sec. 2.1; test infrastructure only).

All symbols are scaled by h^2 so that they depend on eta = lambda h^2 only:
  h^2 L~(theta)  = 4 + eta - 2 cos t1 - 2 cos t2,
  M~_e(theta)/h^2 = a + b cos t1 + b cos t2 + c cos t1 cos t2     (Sec. 2.1),
  S~(theta)      = 1 - omega (M~_e/h^2)(h^2 L~)                   (eq. (7)).
Low frequencies T^L = [-pi/2, pi/2)^2, high T^H = [-pi/2, 3pi/2)^2 minus T^L.
"""
import numpy as np

from .operators import vanka_abc


def symbol_L(t1, t2, eta):
    """h^2 times the symbol of L_j (Sec. 2.1)."""
    return 4.0 + eta - 2.0 * np.cos(t1) - 2.0 * np.cos(t2)


def symbol_M_vanka(t1, t2, eta):
    """Symbol of M_{e,j} divided by h^2 (Sec. 2.1)."""
    a, b, c = vanka_abc(eta)
    c1, c2 = np.cos(t1), np.cos(t2)
    return a + b * c1 + b * c2 + c * c1 * c2


def symbol_M_jacobi(t1, t2, eta):
    """Symbol of the point-Jacobi inverse diagonal, divided by h^2."""
    return 1.0 / (4.0 + eta) + 0.0 * t1 + 0.0 * t2


def symbol_S(t1, t2, eta, omega, smoother="vanka"):
    """Smoothing symbol of eq. (7), 1 - omega M~ L~."""
    m = symbol_M_vanka if smoother == "vanka" else symbol_M_jacobi
    return 1.0 - omega * m(t1, t2, eta) * symbol_L(t1, t2, eta)


def high_frequency_grid(n=128):
    """Uniform samples of T^H: the node-centred n x n grid on [-pi/2, 3pi/2)^2
    (n a multiple of 4, so theta = 0, pi/2 and pi are nodes) with the points of
    T^L = [-pi/2, pi/2)^2 removed."""
    n = 4 * ((n + 3) // 4)
    t = -np.pi / 2 + 2 * np.pi * np.arange(n) / n
    t1, t2 = np.meshgrid(t, t, indexing="ij")
    low = (t1 >= -np.pi / 2 - 1e-12) & (t1 < np.pi / 2 - 1e-12) & (t2 >= -np.pi / 2 - 1e-12) & (t2 < np.pi / 2 - 1e-12)
    return t1[~low], t2[~low]


def smoothing_factor(eta, omega, smoother="vanka", n=128):
    """mu_loc of eq. (4): max over sampled T^H of |S~(theta)| (the symbol is
    a scalar for a point smoother or the stencil form of eq. (6))."""
    t1, t2 = high_frequency_grid(n)
    return float(np.max(np.abs(symbol_S(t1, t2, eta, omega, smoother))))


def _two_grid_blocks(t1, t2, eta, omega, nu, smoother):
    """4x4 two-grid symbols S~^nu (I - P~ L~_H^{-1} R~ L~_h) for low
    frequencies theta = (t1, t2), one block per sample.

    Harmonics theta^alpha = theta + (0,0), (pi,0), (0,pi), (pi,pi).  Full
    weighting has symbol R~ = (1 + cos t1^a)(1 + cos t2^a)/4 and linear
    interpolation the same values as a column (standard LFA of the transfers
    named in Sec. 3); the coarse operator is the re-discretisation
    (4 + 4 eta - 2 cos 2t1 - 2 cos 2t2)/4 in units of 1/h^2.
    """
    shifts = [(0.0, 0.0), (np.pi, 0.0), (0.0, np.pi), (np.pi, np.pi)]
    m = len(t1)
    Lh = np.empty((m, 4), dtype=np.complex128)
    Sh = np.empty((m, 4), dtype=np.complex128)
    R = np.empty((m, 4), dtype=np.float64)
    for a, (s1, s2) in enumerate(shifts):
        u1, u2 = t1 + s1, t2 + s2
        Lh[:, a] = symbol_L(u1, u2, eta)
        Sh[:, a] = symbol_S(u1, u2, eta, omega, smoother)
        R[:, a] = 0.25 * (1.0 + np.cos(u1)) * (1.0 + np.cos(u2))
    LH = (4.0 + 4.0 * eta - 2.0 * np.cos(2 * t1) - 2.0 * np.cos(2 * t2)) / 4.0
    # K = I - P LH^{-1} R Lh, P = R^T
    K = np.eye(4)[None, :, :] - (R[:, :, None] * R[:, None, :]) * (Lh[:, None, :] / LH[:, None, None])
    Snu = Sh ** nu
    return Snu[:, :, None] * K


def low_frequency_grid(n=64):
    """Cell-centred n x n samples of T^L (theta = 0 is never hit)."""
    t = -np.pi / 2 + np.pi * (np.arange(n) + 0.5) / n
    t1, t2 = np.meshgrid(t, t, indexing="ij")
    return t1.ravel(), t2.ravel()


def two_grid_factor(eta, omega, nu, smoother="vanka", n=64):
    """LFA two-grid convergence factor rho(nu): max over sampled T^L of the
    spectral radius of the 4x4 two-grid symbol, nu pre-smoothing steps and no
    post-smoothing (rho depends only on the total number of steps)."""
    t1, t2 = low_frequency_grid(n)
    blocks = _two_grid_blocks(t1, t2, eta, omega, nu, smoother)
    return float(np.max(np.abs(np.linalg.eigvals(blocks))))


def optimal_omega(eta, smoother="vanka", objective="two_grid", omegas=None):
    """Real omega minimising the LFA factor (Sec. 2.1, eq. (5)); Table 1 takes
    the minimiser of rho(1).  Returns (omega, factor) from a scan."""
    if omegas is None:
        omegas = np.round(np.arange(0.50, 1.2001, 0.01), 2)
    best = None
    for w in omegas:
        f = two_grid_factor(eta, w, 1, smoother) if objective == "two_grid" else smoothing_factor(eta, w, smoother)
        if best is None or f < best[1] - 1e-12:
            best = (float(w), f)
    return best


def optimal_complex_omega(eta, smoother="vanka", n=64):
    """Complex omega minimising the smoothing factor mu_loc of eq. (4) (the
    complex relaxation parameter of the future work after Example 3): a scan
    of the complex plane refined by Nelder-Mead.  Returns (omega, mu)."""
    import scipy.optimize
    t1, t2 = high_frequency_grid(n)

    def mu(p):
        return float(np.max(np.abs(symbol_S(t1, t2, eta, p[0] + 1j * p[1], smoother))))

    best = None
    for wr in np.linspace(0.3, 1.5, 25):
        for wi in np.linspace(-0.8, 0.8, 33):
            v = mu((wr, wi))
            if best is None or v < best[1]:
                best = ((wr, wi), v)
    res = scipy.optimize.minimize(mu, best[0], method="Nelder-Mead", options={"xatol": 1e-6, "fatol": 1e-9})
    w = res.x[0] + 1j * res.x[1]
    return w, mu(res.x)


def rfa_two_grid_spectrum(n, eta, omega, nu1, nu2, smoother="vanka"):
    """Eigenvalues of the two-grid operator on an n x n Dirichlet grid
    (h = 1/(n+1), exact coarse solve) from its sine-mode blocks.

    Sine modes phi_kl are eigenvectors of L_j and of the stencil smoother.
    Full weighting maps phi_{k,l} to the coarse mode (k, l) with the factor
    (1 + cos k pi h)/2 per direction, and the aliased partner N+1-k with
    -(1 - cos k pi h)/2; linear interpolation maps back with the same
    factors.  Modes with k or l = (n+1)/2 restrict to zero.  Returns all n^2
    eigenvalues of S^{nu2} K S^{nu1}.
    """
    h = 1.0 / (n + 1)
    nc = (n - 1) // 2
    H = 2 * h
    out = []

    def ch(k):
        return np.cos(k * np.pi * h)

    def sym_S(k, l):
        return symbol_S(k * np.pi * h, l * np.pi * h, eta, omega, smoother)

    def sym_L(k, l):
        return symbol_L(k * np.pi * h, l * np.pi * h, eta) / (h * h)

    def rf(k):
        # restriction factor of fine mode k onto coarse mode min(k, n+1-k)
        return (1 + ch(k)) / 2 if k <= nc else -(1 - ch(n + 1 - k)) / 2

    for k in range(1, nc + 1):
        for l in range(1, nc + 1):
            modes = [(k, l), (n + 1 - k, l), (k, n + 1 - l), (n + 1 - k, n + 1 - l)]
            R = np.array([rf(p) * rf(q) for p, q in modes])
            LHkl = (4.0 + eta * 4.0 - 2 * np.cos(k * np.pi * H) - 2 * np.cos(l * np.pi * H)) / (H * H)
            Lh = np.array([sym_L(p, q) for p, q in modes])
            K = np.eye(4) - np.outer(R, R * Lh) / LHkl
            S = np.diag([sym_S(p, q) for p, q in modes])
            T = np.linalg.matrix_power(S, nu2) @ K @ np.linalg.matrix_power(S, nu1)
            out.extend(np.linalg.eigvals(T))
    mid = (n + 1) // 2
    # lines through the middle frequency: no coarse-grid correction
    for k in range(1, n + 1):
        for l in range(1, n + 1):
            if k == mid or l == mid:
                out.append(sym_S(k, l) ** (nu1 + nu2))
    return np.array(out)
