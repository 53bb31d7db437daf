"""Discrete Spectral Ewald k-space algorithm in plain numpy, FP64.

TEST INFRASTRUCTURE ONLY: imported by tests/, by the smoke check and by the
benchmark's CPU-baseline leg, never by the product library.  It shares no code
with the GPU path: the parameter rules, windows, Green's functions, transforms
and gathering are all restated here from the paper.

It follows the paper's Algorithm 4 step by step:
  0. parameters  (Section 3.3, Section 6, Table lambda)
  1. gridding    H(x) = sum_n q_n W(x - x_n)_*          (Eq. gridding)
  2. transform   FFT (3P), AFT (2P, 1P; Algorithm 1), (2 Mt)^3 FFT (0P)
  3. scaling     e^{-k^2/4xi^2} W^(k)^{-2} G^{DP}(k)    (Eq. scale), with the
                 modified Green's functions of Section 3.1 and, for 0P, the
                 effective Green's function of Algorithm 3
  4. inverse     IFFT / AIFT (Algorithm 2)
  5. gathering   trapezoidal rule for Eq. (complete_integral); gradients by
                 differentiating the gathering window (Eq. force-method-1)

Normalisation: with numpy's FFT conventions (forward unscaled, inverse 1/n on
each padded length) the discrete transforms carry no further factors, and the
gathered potential is 4 pi h^3 sum_j W(x_m - x_j) Ht_j (trapezoidal rule of
Eq. complete_integral on the grid of spacing h).

Readings of the paper taken here (each listed in the design notes):
  * the AIFT truncates the padded free directions back to Mt points (the
    extended grid), not to M;
  * the stencil of a particle at grid coordinate t covers the P points
    floor(t)-P/2+1 ... floor(t)+P/2, so that all P points share the offset
    xbar = 1 - 2 frac(t) inside their subintervals;
  * Mt, s0*Mt and s*Mt are rounded up to even integers and then up to the next
    integer whose only prime factors are 2, 3, 5, 7;
  * the 0P effective Green's function keeps the signed offsets -Mt..Mt-1 of
    the upsampled real-space kernel.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np
from scipy import special

# ---------------------------------------------------------------------------
# Step 0: parameters
# ---------------------------------------------------------------------------

LAMBDA = {  # Table lambda (Section 6)
    "gaussian": {0: 1.0, 1: 1.5, 2: 1.5},
    "pkb": {0: 1.3, 1: 2.4, 2: 2.4},
    "kb": {0: 1.3, 1: 2.4, 2: 2.4},
    "es": {0: 1.3, 1: 2.4, 2: 2.4},   # the ES window approximates KB (Section 4): KB's values
}
S0 = {0: 2.8, 1: 2.5, 2: 2.0}  # Section 3.4 / Section 6


def smooth_even_up(n: int) -> int:
    """Smallest even integer >= n whose prime factors are all in {2,3,5,7}."""
    m = max(2, int(n))
    if m % 2:
        m += 1
    while True:
        r = m
        for p in (2, 3, 5, 7):
            while r % p == 0:
                r //= p
        if r == 1:
            return m
        m += 2


def fc(x: float) -> float:
    """f_c(x) of Eq. (fc-expression)."""
    c1, c2, c3, c4 = 12.62, 0.8909, 0.01411, 4.315e-5
    return math.exp(-c1 / x ** 2) * (c2 + c3 * x + c4 * x * x)


def B_scale(Q: float, xi: float, L: float) -> float:
    """B = sqrt(Q) f_c(xi L) / L (Section 5.2), Q = sum q^2."""
    return math.sqrt(Q) * fc(xi * L) / L


def kp_kspace_error(Q: float, xi: float, L: float, M: int) -> float:
    """Kolafa-Perram k-space truncation estimate, Eq. (KP_fourier_space),
    with k_inf = M/2."""
    kinf = M / 2.0
    return math.sqrt(Q) * xi * math.pi ** -2 * kinf ** -1.5 * math.exp(-(math.pi * kinf / (xi * L)) ** 2)


def kp_realspace_error(Q: float, xi: float, L: float, rc: float) -> float:
    """Kolafa-Perram real-space estimate, Eq. (KP_real_space)."""
    return math.sqrt(Q) * xi ** -2 * (L * rc) ** -1.5 * math.exp(-(xi * rc) ** 2)


def pollution_bound(window: str, x: float) -> float:
    """f_W(x) of Eq. (error_pollution); pollution when P > f_W(M/(xi L))."""
    if window == "gaussian":
        return x * x + 0.2 * x + 2.25
    return 0.7 * x * x + 0.2 * x + 1.8


def aft_s(M: int, Mt: int, B: float, eps: float) -> float:
    """Eq. (estimate-s)."""
    return (M / Mt) * (1.0 + math.log(B / (2.0 * eps)) / (2.0 * math.pi))


def aft_nl(M: int, Mt: int, B: float, eps: float) -> int:
    """Eq. (estimate-nl)."""
    return int(math.ceil((M / (Mt - M)) * math.log(B / (2.0 * eps)) / (2.0 * math.pi) - 1.0))


@dataclasses.dataclass
class Params:
    D: int
    L: float
    xi: float
    M: int
    P: int
    window: str = "pkb"   # "gaussian", "pkb" (piecewise polynomial KB), "kb" (exact KB) or "es"
    deriv_fit: bool = False     # PKB: fit W'_KB separately for the gradient (Section 7.2)
    shape: float | None = None  # alpha (Gaussian) or beta (KB); default from Section 6
    nu: int | None = None       # PKB degree; default min(P/2+2, 9)
    lam: float | None = None    # Table lambda
    s0: float | None = None
    s: float | None = None
    n_l: int | None = None
    # triply periodic rectangular boxes: grid points along y and z (the box
    # is M h x My h x Mz h, one grid spacing h = L/M); None: a cube
    My: int | None = None
    Mz: int | None = None

    def __post_init__(self):
        if self.M % 2 or self.P % 2 or self.P > self.M:
            raise ValueError("M and P must be even with P <= M (Section 3.3)")
        if self.My is None:
            self.My = self.M
        if self.Mz is None:
            self.Mz = self.M
        if (self.My, self.Mz) != (self.M, self.M):
            # rectangular periodic cells: triply periodic boxes, or a doubly
            # periodic cell M h x My h with the free direction of extent L
            if self.D not in (2, 3) or (self.D == 2 and self.Mz != self.M):
                raise ValueError("rectangular cells are triply periodic, or doubly periodic in x and y")
            if self.My % 2 or self.Mz % 2 or self.P > min(self.My, self.Mz):
                raise ValueError("My and Mz must be even and at least P")
        if self.shape is None:
            self.shape = (math.pi / 2) * self.P * 0.91 if self.window == "gaussian" else 2.5 * self.P
        if self.nu is None:
            self.nu = min(self.P // 2 + 2, 9)
        if self.D < 3:
            if self.lam is None:
                self.lam = LAMBDA[self.window][self.D]
            if self.s0 is None:
                self.s0 = S0[self.D]
        if self.D in (1, 2) and (self.s is None or self.n_l is None):
            raise ValueError("2P/1P need s and n_l (use with_aft_estimates)")

    # Algorithm 4, step 0
    @property
    def h(self):
        return self.L / self.M

    @property
    def Mt(self):
        if self.D == 3:
            return self.M
        return smooth_even_up(2 * math.ceil((self.M + self.lam * self.P) / 2))

    @property
    def Lt(self):
        return self.h * self.Mt

    @property
    def R(self):
        return math.sqrt(3 - self.D) * self.Lt

    @property
    def n0(self):
        """Length of the zero-mode (2P/1P) or precompute (0P) free transform."""
        return smooth_even_up(math.ceil(self.s0 * self.Mt - 1e-9))

    @property
    def nI(self):
        return smooth_even_up(math.ceil(self.s * self.Mt - 1e-9))

    @property
    def Md(self):
        """Grid points per periodic direction (M, My, Mz)."""
        return (self.M, self.My, self.Mz)

    @property
    def Ld(self):
        """Box side per periodic direction, Md[d] h (L itself where Md[d] = M)."""
        return tuple(self.L if m == self.M else m * self.h for m in self.Md)

    @property
    def grid_shape(self):
        """Gridding grid: M (My, Mz) points in periodic and Mt in free directions."""
        return tuple(self.Md[d] if d < self.D else self.Mt for d in range(3))


def kinf_for_tolerance(Q: float, xi: float, L: float, eps: float) -> float:
    """Largest wavenumber index k_inf of Eq. (KP_kinf) for an absolute rms
    tolerance eps: the inverse of Eq. (KP_fourier_space), through the
    principal branch of the Lambert W function."""
    arg = (4.0 / 3.0) * (Q / (math.pi * xi * L ** 3 * eps ** 2)) ** (2.0 / 3.0)
    return math.sqrt(3.0) * xi * L / (2.0 * math.pi) * math.sqrt(float(special.lambertw(arg).real))


def support_for_tolerance(window: str, B: float, eps: float) -> int:
    """Window support P from the approximation estimates of Section 5.2,
    eps = 2 B e^{-(pi/2) P c} (Gaussian, c^2 = 0.91) or 10 B e^{-2.5 P} (KB /
    PKB), rounded up to an even integer (at least 2)."""
    if window == "gaussian":
        P = math.log(2.0 * B / eps) / ((math.pi / 2.0) * math.sqrt(0.91))
    else:
        P = math.log(10.0 * B / eps) / 2.5
    return max(2, 2 * math.ceil(P / 2.0 - 1e-12))


def recipe(D, L, xi, Q, eps, window="pkb") -> Params:
    """The parameter selection of Section 6 for an absolute rms tolerance
    eps at a given xi: M = 2 k_inf (Eq. KP_kinf), rounded up to an even
    7-smooth integer; P from the approximation estimate; when P > f_W(M/(xi
    L)) (error pollution, Eq. error_pollution) M grows by 5 % and P by 4; the
    shape, nu, lambda, s0 rules; s and n_l from Eqs. (estimate-s),
    (estimate-nl)."""
    B = B_scale(Q, xi, L)
    M = smooth_even_up(math.ceil(2.0 * kinf_for_tolerance(Q, xi, L, eps) - 1e-9))
    P = support_for_tolerance(window, B, eps)
    if P > pollution_bound(window, M / (xi * L)):
        M = smooth_even_up(math.ceil(1.05 * M - 1e-9))
        P += 4
    M = max(M, smooth_even_up(P))
    return with_aft_estimates(D, L, xi, M, P, Q, eps, window=window)


def with_aft_estimates(D, L, xi, M, P, Q, eps, window="pkb", **kw) -> Params:
    """Params with s and n_l from Eqs. (estimate-s), (estimate-nl).
    s is kept >= 1 and n_l in [0, M/2]."""
    p = Params(D=D, L=L, xi=xi, M=M, P=P, window=window, s=1.0, n_l=0, **kw)
    if D in (1, 2):
        B = B_scale(Q, xi, L)
        p.s = max(1.0, aft_s(M, p.Mt, B, eps))
        p.n_l = min(max(aft_nl(M, p.Mt, B, eps), 0), M // 2)
    return p


# ---------------------------------------------------------------------------
# Windows (Section 4)
# ---------------------------------------------------------------------------

def kb(u, P, beta):
    """KB window, Eq. (kaiser_window), in grid units u = x/h (w = P/2)."""
    z = 2.0 * np.asarray(u, dtype=np.float64) / P
    inside = np.abs(z) <= 1.0
    arg = beta * np.sqrt(np.where(inside, 1.0 - z * z, 0.0))
    return np.where(inside, special.i0(arg) / special.i0(beta), 0.0)


def kb_du(u, P, beta):
    """d/du of the KB window."""
    z = 2.0 * np.asarray(u, dtype=np.float64) / P
    inside = np.abs(z) < 1.0
    sq = np.sqrt(np.where(inside, 1.0 - z * z, 1.0))
    val = -special.i1(beta * sq) * beta * z * (2.0 / P) / (sq * special.i0(beta))
    return np.where(inside, val, 0.0)


def pkb_coefficients(P, beta, nu, fn=None):
    """Coefficients c[i, j] of the PKB window (Section 4.1): on subinterval i
    of [-w, w] (i = 0..P-1, each of length h) the KB window is interpolated by
    sum_j c[i,j] xbar^j at the nu+1 Chebyshev points
    xbar_k = cos(pi (k - 1/2)/(nu+1)), Eqs. (polynomial-ansatz), (polynomial-linsys).
    fn replaces the KB window by another function of u (grid units), such as
    its derivative for the separately fitted W'_KB of Section 7.2."""
    fn = kb if fn is None else fn
    k = np.arange(1, nu + 2)
    xb = np.cos(np.pi * (k - 0.5) / (nu + 1))
    V = xb[:, None] ** np.arange(nu + 1)[None, :]
    c = np.empty((P, nu + 1))
    for i in range(P):
        u = -P / 2 + i + (xb + 1.0) / 2.0   # subinterval i in grid units
        c[i] = np.linalg.solve(V, fn(u, P, beta))
    return c


def es(u, P, beta):
    """ES window, Eq. (expsemicirc_window), in grid units u = x/h (w = P/2)."""
    z = 2.0 * np.asarray(u, dtype=np.float64) / P
    inside = np.abs(z) <= 1.0
    return np.where(inside, np.exp(beta * (np.sqrt(np.where(inside, 1.0 - z * z, 0.0)) - 1.0)), 0.0)


def es_du(u, P, beta):
    """d/du of the ES window (0 at the end points, where it is not
    differentiable)."""
    z = 2.0 * np.asarray(u, dtype=np.float64) / P
    inside = np.abs(z) < 1.0
    sq = np.sqrt(np.where(inside, 1.0 - z * z, 1.0))
    return np.where(inside, -es(u, P, beta) * beta * z * (2.0 / P) / sq, 0.0)


def es_ft(k, h, P, beta):
    """Fourier transform of the ES window, which has no closed form
    (Section 4): int_{-w}^{w} W(x) cos(k x) dx by adaptive quadrature, after
    x = w sin(theta), which removes the square-root end behaviour:
    2 w int_0^{pi/2} e^{beta (cos theta - 1)} cos(k w sin theta) cos theta dtheta."""
    from scipy import integrate
    w = P * h / 2.0
    out = []
    for kk in np.atleast_1d(np.asarray(k, dtype=np.float64)).ravel():
        f = lambda th: math.exp(beta * (math.cos(th) - 1.0)) * math.cos(kk * w * math.sin(th)) * math.cos(th)
        out.append(2.0 * w * integrate.quad(f, 0.0, math.pi / 2, limit=500, epsabs=0.0, epsrel=2e-14)[0])
    return np.reshape(np.array(out), np.shape(k))


def window_ft(k, h, P, window, shape):
    """1D Fourier transform of the window used in the scaling step:
    untruncated Gaussian (Section 4) or the exact KB transform,
    Eq. (kaiser_ft).  k in physical units, w = P h / 2."""
    w = P * h / 2.0
    k = np.asarray(k, dtype=np.float64)
    if window == "es":
        return es_ft(k, h, P, shape)
    if window == "gaussian":
        a = shape
        return np.sqrt(np.pi / a) * w * np.exp(-k * k * w * w / (4.0 * a))
    b = shape
    d = b * b - k * k * w * w
    sd = np.sqrt(np.abs(d))
    with np.errstate(invalid="ignore", divide="ignore"):
        pos = np.where(sd > 0, np.sinh(sd) / np.where(sd > 0, sd, 1.0), 1.0)
        neg = np.where(sd > 0, np.sin(sd) / np.where(sd > 0, sd, 1.0), 1.0)
    return 2.0 * w * np.where(d >= 0, pos, neg) / special.i0(b)


def weights_1d(t, p: Params):
    """Window weights of the P stencil points of particles at grid coordinate
    t (array), and their derivatives with respect to the particle coordinate.

    Returns (j0, W, dW) with j0 = floor(t) - P/2 + 1 (int array), W and dW of
    shape (len(t), P); stencil point i sits at grid index j0 + i."""
    P = p.P
    fl = np.floor(t)
    j0 = fl.astype(np.int64) - P // 2 + 1
    f = t - fl
    i = np.arange(P)
    u = (j0[:, None] + i[None, :]) - t[:, None]   # grid point minus particle, grid units
    if p.window == "gaussian":
        a = p.shape
        W = np.exp(-a * (2.0 * u / P) ** 2)
        dWdt = W * 2.0 * a * (2.0 / P) ** 2 * u     # u = j - t
    elif p.window == "kb":
        W = kb(u, P, p.shape)
        dWdt = -kb_du(u, P, p.shape)
    elif p.window == "es":
        W = es(u, P, p.shape)
        dWdt = -es_du(u, P, p.shape)
    else:
        c = pkb_coefficients(P, p.shape, p.nu)    # (P, nu+1)
        xb = 1.0 - 2.0 * f                          # same for all P subintervals
        powers = xb[:, None] ** np.arange(p.nu + 1)[None, :]
        W = powers @ c.T
        if p.deriv_fit:
            # Section 7.2: W'_KB fitted by the same procedure (same P, beta, nu);
            # d/dt W(j - t) = -W'(u)
            dWdt = -(powers @ pkb_coefficients(P, p.shape, p.nu, fn=kb_du).T)
        else:
            dpow = np.zeros_like(powers)
            dpow[:, 1:] = np.arange(1, p.nu + 1)[None, :] * powers[:, :-1]
            dWdt = -2.0 * (dpow @ c.T)              # d xbar / dt = -2
    return j0, W, dWdt / p.h


def grid_coords(x, p: Params):
    """Grid coordinate t of each particle in each direction: periodic
    directions start at 0; free directions start at -delta_L/2 (Algorithm 4,
    step 1), an integer number (Mt - M)/2 of cells below 0."""
    x = np.asarray(x, dtype=np.float64)
    t = np.empty_like(x)
    for d in range(3):
        if d < p.D:
            t[:, d] = np.mod(x[:, d], p.Ld[d]) / p.h
        else:
            t[:, d] = x[:, d] / p.h + (p.Mt - p.M) // 2
    return t


# ---------------------------------------------------------------------------
# Step 1: gridding
# ---------------------------------------------------------------------------

def gridding(x, q, p: Params):
    """H on the M^D x Mt^(3-D) grid, Eq. (gridding), periodic wrap in the
    periodic directions.  Array index order [ix, iy, iz]."""
    t = grid_coords(x, p)
    shape = p.grid_shape
    parts = [weights_1d(t[:, d], p) for d in range(3)]
    H = np.zeros(int(np.prod(shape)))
    idx = []
    for d in range(3):
        j0, W, _ = parts[d]
        j = j0[:, None] + np.arange(p.P)[None, :]
        if d < p.D:
            j = np.mod(j, p.Md[d])
        elif j.min() < 0 or j.max() >= p.Mt:
            raise ValueError("particle outside the box in a free direction")
        idx.append(j)
    q = np.asarray(q, dtype=np.float64)
    for a in range(p.P):
        wa = q * parts[0][1][:, a]
        ia = idx[0][:, a] * shape[1]
        for b in range(p.P):
            wab = wa * parts[1][1][:, b]
            iab = (ia + idx[1][:, b]) * shape[2]
            for c in range(p.P):
                H += np.bincount(iab + idx[2][:, c], weights=wab * parts[2][1][:, c],
                                 minlength=H.size)
    return H.reshape(shape), (t, parts, idx)


# ---------------------------------------------------------------------------
# Step 3 ingredients: modified Green's functions (Section 3.1)
# ---------------------------------------------------------------------------

def G_hat_0P(k, R):
    """Eq. (G_hat_0d)."""
    k = np.asarray(k, dtype=np.float64)
    with np.errstate(invalid="ignore", divide="ignore"):
        v = 2.0 * (np.sin(R * k / 2.0) / k) ** 2
    return np.where(k == 0, R * R / 2.0, v)


def G_hat_1P_zero(kap, R):
    """Eq. (G_hat_1d), periodic wavenumber zero, kap = |(k2,k3)|."""
    kap = np.asarray(kap, dtype=np.float64)
    with np.errstate(invalid="ignore", divide="ignore"):
        v = (1.0 - special.j0(R * kap)) / kap ** 2 - R * math.log(R) * special.j1(R * kap) / kap
    return np.where(kap == 0, R * R / 4.0 * (1.0 - 2.0 * math.log(R)), v)


def G_hat_2P_zero(kap, R):
    """Eq. (G_hat_2d), periodic wavenumber zero, kap = |k3|."""
    kap = np.abs(np.asarray(kap, dtype=np.float64))
    with np.errstate(invalid="ignore", divide="ignore"):
        v = (1.0 - np.cos(R * kap) - R * kap * np.sin(R * kap)) / kap ** 2
    return np.where(kap == 0, -R * R / 2.0, v)


def precompute_0P(p: Params):
    """Algorithm 3: effective free-space Green's function on the (2 Mt)^3 grid
    of wavenumbers k_i = pi n / Lt.  Returns a real (2Mt)^3 array in FFT order."""
    Mt, n0 = p.Mt, p.n0
    h = p.h
    kk = 2.0 * np.pi * np.fft.fftfreq(n0, d=h)     # 2 pi n / (s0 Lt)
    K = np.sqrt(kk[:, None, None] ** 2 + kk[None, :, None] ** 2 + kk[None, None, :] ** 2)
    Ghat = G_hat_0P(K, p.R)
    G = np.fft.ifftn(Ghat)                            # step 2
    off = np.arange(-Mt, Mt)                          # signed offsets kept, step 3
    sel = np.mod(off, n0)
    Gt = G[np.ix_(sel, sel, sel)]
    pos = np.mod(off, 2 * Mt)                         # placed in FFT order
    GR = np.empty((2 * Mt,) * 3, dtype=complex)
    GR[np.ix_(pos, pos, pos)] = Gt
    return np.fft.fftn(GR).real                       # step 4


def _free_k(n_len, h):
    """Free-direction wavenumbers of a transform of length n_len over a grid
    of spacing h: kappa = 2 pi n / (n_len h), n in FFT order."""
    return 2.0 * np.pi * np.fft.fftfreq(n_len, d=h)


def _periodic_k(M, L):
    return 2.0 * np.pi * np.fft.fftfreq(M, d=L / M)


def _sep(k, p: Params):
    """e^{-k^2/4 xi^2} / W^(k)^2 for one direction."""
    return np.exp(-k * k / (4.0 * p.xi ** 2)) / window_ft(k, p.h, p.P, p.window, p.shape) ** 2


# ---------------------------------------------------------------------------
# Steps 2-4: transform, scale, inverse transform
# ---------------------------------------------------------------------------

def _pad_fft(a, axes, n):
    """Zero-pad along the given axes to length n and FFT over them."""
    return np.fft.fftn(a, s=[n] * len(axes), axes=axes)


def _ifft_trunc(a, axes, m):
    """IFFT along the given axes and keep the first m points of each."""
    b = np.fft.ifftn(a, axes=axes)
    sl = [slice(None)] * b.ndim
    for ax in axes:
        sl[ax] = slice(0, m)
    return b[tuple(sl)]


def _mode_classes(p: Params):
    """Boolean masks over the periodic FFT modes: zero mode, set I (Eq. I)
    and set J (Eq. J)."""
    n = np.fft.fftfreq(p.M, d=1.0 / p.M)   # signed integers
    if p.D == 2:
        n1, n2 = np.meshgrid(n, np.fft.fftfreq(p.My, d=1.0 / p.My), indexing="ij")
        zero = (n1 == 0) & (n2 == 0)
        # the set I bounds the wavenumber, |k_d| <= 2 pi n_l / L, in each
        # periodic direction: index n_l along x, n_l My / M along y (the
        # same n_l for a square cell)
        box = (np.abs(n1) <= p.n_l) & (np.abs(n2) <= (p.n_l * p.My) // p.M)
    else:
        zero = n == 0
        box = np.abs(n) <= p.n_l
    I = box & ~zero
    J = ~box
    return zero, I, J


def _ik(k, deriv, d):
    """Factor i k_d of force method 2 (Section 7.2) for direction d, or 1.
    The Nyquist wavenumber of an even-length transform gets the factor 0 so
    that the derivative of a real grid stays real."""
    if deriv != d:
        return 1.0
    k = np.asarray(k, dtype=np.float64)
    n = k.shape[0]
    f = 1j * k
    if n % 2 == 0:
        f = f.copy()
        f[n // 2] = 0.0
    return f


def scaled_convolution(H, p: Params, GR=None, deriv=None):
    """Steps 2-4 of Algorithm 4 on the gridded H: returns Ht (real, same shape).

    deriv = d in {0, 1, 2}: force method 2 of Section 7.2 -- the scaling step
    is multiplied by i k_d (k_d the wavenumber of direction d on the grid that
    direction is transformed on), so the result is the derivative of Ht along
    d."""
    D, M, Mt, L, h = p.D, p.M, p.Mt, p.L, p.h
    if D == 3:
        Hh = np.fft.fftn(H)
        # one wavenumber vector per direction, k = 2 pi n / L_d (a cube: all equal)
        kx, ky, kz = (_periodic_k(m, l) for m, l in zip(p.Md, p.Ld))
        K2 = kx[:, None, None] ** 2 + ky[None, :, None] ** 2 + kz[None, None, :] ** 2
        S = _sep(kx, p)[:, None, None] * _sep(ky, p)[None, :, None] * _sep(kz, p)[None, None, :]
        with np.errstate(divide="ignore"):
            G = np.where(K2 == 0, 0.0, 1.0 / np.where(K2 == 0, 1.0, K2))  # Eq. (G_hat_3d)
        ik = (np.reshape(_ik(kx, deriv, 0), (-1, 1, 1)) * np.reshape(_ik(ky, deriv, 1), (1, -1, 1))
              * np.reshape(_ik(kz, deriv, 2), (1, 1, -1)))
        return np.fft.ifftn(ik * S * G * Hh).real

    if D == 0:
        if GR is None:
            GR = precompute_0P(p)
        n = 2 * Mt
        Hh = _pad_fft(H, (0, 1, 2), n)
        k = _free_k(n, h)
        sep = _sep(k, p)
        S = sep[:, None, None] * sep[None, :, None] * sep[None, None, :]
        ik = (np.reshape(_ik(k, deriv, 0), (-1, 1, 1)) * np.reshape(_ik(k, deriv, 1), (1, -1, 1))
              * np.reshape(_ik(k, deriv, 2), (1, 1, -1)))
        return _ifft_trunc(ik * S * GR * Hh, (0, 1, 2), Mt).real

    zero, I, J = _mode_classes(p)
    kp = _periodic_k(M, L)
    sep_p = _sep(kp, p)
    if D == 2:
        # Algorithm 1, step 1: FFT in the periodic directions x, y (y of
        # length My, side My h, in a rectangular cell)
        My = p.My
        kq = _periodic_k(My, p.Ld[1])
        sep_q = _sep(kq, p)
        Hk = np.fft.fft2(H, axes=(0, 1))
        out = np.zeros((M, My, Mt), dtype=complex)
        for mask, length in ((zero, p.n0), (I, p.nI), (J, Mt)):
            if not mask.any():
                continue
            sub = Hk[mask]                                  # (modes, Mt)
            Hs = _pad_fft(sub, (1,), length)                # Algorithm 1, steps 2-4
            kap = _free_k(length, h)
            k1 = np.broadcast_to(kp[:, None], (M, My))[mask]
            k2 = np.broadcast_to(kq[None, :], (M, My))[mask]
            s12 = (np.broadcast_to(sep_p[:, None], (M, My)) * np.broadcast_to(sep_q[None, :], (M, My)))[mask]
            kk2 = k1 ** 2 + k2 ** 2
            if mask is zero:
                G = G_hat_2P_zero(kap, p.R)[None, :] * np.ones((sub.shape[0], 1))
            else:
                G = 1.0 / (kk2[:, None] + kap[None, :] ** 2)    # Eq. (G_hat_2d), k != 0
            S = s12[:, None] * _sep(kap, p)[None, :] * G
            ik12 = (np.broadcast_to(np.reshape(_ik(kp, deriv, 0), (-1, 1)), (M, My))
                    * np.broadcast_to(np.reshape(_ik(kq, deriv, 1), (1, -1)), (M, My)))[mask]
            S = S * ik12[:, None] * np.reshape(_ik(kap, deriv, 2), (1, -1))
            out[mask] = _ifft_trunc(S * Hs, (1,), Mt)       # Algorithm 2, steps 1-4
        return np.fft.ifft2(out, axes=(0, 1)).real          # Algorithm 2, step 5

    # D == 1: periodic x, free y and z
    Hk = np.fft.fft(H, axis=0)
    out = np.zeros((M, Mt, Mt), dtype=complex)
    for mask, length in ((zero, p.n0), (I, p.nI), (J, Mt)):
        if not mask.any():
            continue
        sub = Hk[mask]                                      # (modes, Mt, Mt)
        Hs = _pad_fft(sub, (1, 2), length)
        kap = _free_k(length, h)
        KAP2 = kap[:, None] ** 2 + kap[None, :] ** 2
        sk = _sep(kap, p)
        S2 = sk[:, None] * sk[None, :]
        k1 = kp[mask]
        if mask is zero:
            G = G_hat_1P_zero(np.sqrt(KAP2), p.R)[None, :, :]
        else:
            G = 1.0 / (k1[:, None, None] ** 2 + KAP2[None, :, :])   # Eq. (G_hat_1d), k != 0
        S = sep_p[mask][:, None, None] * S2[None, :, :] * G
        S = (S * np.reshape(np.broadcast_to(_ik(kp, deriv, 0), (M,))[mask], (-1, 1, 1))
             * np.reshape(_ik(kap, deriv, 1), (1, -1, 1)) * np.reshape(_ik(kap, deriv, 2), (1, 1, -1)))
        out[mask] = _ifft_trunc(S * Hs, (1, 2), Mt)
    return np.fft.ifft(out, axis=0).real


# ---------------------------------------------------------------------------
# Step 5: gathering
# ---------------------------------------------------------------------------

def gathering(Ht, geom, p: Params, targets=None, grad=False):
    """phi_m = 4 pi h^3 sum_j W(x_m - x_j) Ht_j (trapezoidal rule of Eq.
    complete_integral) and optionally grad phi_m by differentiating W
    (Eq. force-method-1)."""
    t, parts, idx = geom
    n = t.shape[0]
    sel = np.arange(n) if targets is None else np.asarray(targets)
    Hf = Ht.reshape(-1)
    shape = Ht.shape
    phi = np.zeros(sel.size)
    g = np.zeros((sel.size, 3))
    W = [parts[d][1][sel] for d in range(3)]
    dW = [parts[d][2][sel] for d in range(3)]
    I = [idx[d][sel] for d in range(3)]
    for a in range(p.P):
        ia = I[0][:, a] * shape[1]
        for b in range(p.P):
            iab = (ia + I[1][:, b]) * shape[2]
            for c in range(p.P):
                v = Hf[iab + I[2][:, c]]
                wx, wy, wz = W[0][:, a], W[1][:, b], W[2][:, c]
                phi += v * wx * wy * wz
                if grad:
                    g[:, 0] += v * dW[0][:, a] * wy * wz
                    g[:, 1] += v * wx * dW[1][:, b] * wz
                    g[:, 2] += v * wx * wy * dW[2][:, c]
    c0 = 4.0 * np.pi * p.h ** 3
    return c0 * phi, c0 * g


def spectral_ewald(x, q, p: Params, targets=None, grad=True, GR=None, force_method=1):
    """Algorithm 4: the SE approximation of phi^{D,F} (without the self
    term) and its gradient at the targets (default: all particles).

    force_method 1 differentiates the gathering window (Eq. force-method-1);
    force_method 2 differentiates in Fourier space (Section 7.2): the scaling
    step carries i k_d, steps 4 and 5 run once per direction, and each
    gathering uses the window itself."""
    H, geom = gridding(x, q, p)
    if p.D == 0 and GR is None:
        GR = precompute_0P(p)
    Ht = scaled_convolution(H, p, GR=GR)
    if not grad or force_method == 1:
        return gathering(Ht, geom, p, targets=targets, grad=grad)
    phi, _ = gathering(Ht, geom, p, targets=targets, grad=False)
    g = np.stack([gathering(scaled_convolution(H, p, GR=GR, deriv=d), geom, p, targets=targets)[0]
                  for d in range(3)], axis=1)
    return phi, g


def energy(q, phi):
    """E = 1/2 sum_m q_m phi_m: the energy whose q-derivative is phi and whose
    x-derivative is q grad phi."""
    return 0.5 * float(np.dot(q, phi))
