// Direct FP64 Ewald sums: the plain definition of the potential that the
// Spectral Ewald k-space path approximates.
//
// TEST INFRASTRUCTURE ONLY.  Nothing in the product path links, loads or calls
// this file.  It shares no code with the GPU library.
//
// Every sum is written out term by term, one target at a time, in double
// precision.  Speed is not a goal; the loops are parallelised over targets with
// OpenMP only so that the tests finish.
//
// Paper: Shamshirgar, Bagge, Tornberg, "Fast Ewald summation for electrostatic
// potentials with arbitrary periodicity" (arXiv:1712.04732).
//   real space      : Section 2, Eq. (real_space_ewald)
//   3P k-space      : Section 3, Eq. (fourier_space_explicit_3P)
//   2P k-space      : Section 2, Eqs. (2pno0) [read with "+" between the two
//                     exponential-erfc terms] and (2p0)
//   1P k-space      : Section 2, Eqs. (1pno0) and (1p0), with the incomplete
//                     Bessel function K0(a,b) = int_1^inf e^{-a t - b/t}/t dt
//   0P k-space      : Section 2, remark after Eq. (fourier_space_nonzero_ewald):
//                     the free-space k-space sum is the complement of the
//                     real-space sum minus the self term.
//   self term       : Section 2, phi_self = -2 xi/sqrt(pi) q_m
//
// Positions are (N,3) row-major doubles.  Targets are indices into the source
// list; the self pair (n == m, image 0) is excluded where the definition
// excludes it.
#include <cmath>
#include <cstddef>
#include <vector>

namespace {

constexpr double kPi = 3.14159265358979323846264338327950288;
constexpr double kEulerGamma = 0.57721566490153286060651209008240243;

// ---------------------------------------------------------------------------
// Incomplete modified Bessel function of the second kind (Section 2, after
// Eq. 1pno0):  K0(a,b) = int_1^inf exp(-a t - b/t) / t dt,  a > 0, b >= 0.
// With t = e^u:  K0(a,b) = int_0^inf exp(-a e^u - b e^-u) du.
// Its b-derivative is  dK0/db = -int_1^inf exp(-a t - b/t)/t^2 dt
//                            = -int_0^inf exp(-a e^u - b e^-u) e^-u du.
// Composite 8-point Gauss-Legendre on panels of width 1/32 in u, up to the
// point where a e^u exceeds 45 (the integrand is below e^-45 beyond it).
// ---------------------------------------------------------------------------
const double kGLx[8] = {-0.9602898564975363, -0.7966664774136267, -0.5255324099163290,
                        -0.1834346424956498, 0.1834346424956498,  0.5255324099163290,
                        0.7966664774136267,  0.9602898564975363};
const double kGLw[8] = {0.1012285362903763, 0.2223810344533745, 0.3137066458778873,
                        0.3626837833783620, 0.3626837833783620, 0.3137066458778873,
                        0.2223810344533745, 0.1012285362903763};

void incomplete_k0(double a, double b, double* k0, double* dk0_db) {
  double umax = std::log(45.0 / a);
  if (umax < 1.0) umax = 1.0;
  const double width = 1.0 / 32.0;
  const int panels = (int)std::ceil(umax / width);
  double s0 = 0.0, s1 = 0.0;
  for (int p = 0; p < panels; ++p) {
    const double lo = p * width;
    const double mid = lo + 0.5 * width;
    for (int i = 0; i < 8; ++i) {
      const double u = mid + 0.5 * width * kGLx[i];
      const double eu = std::exp(u);
      const double f = std::exp(-a * eu - b / eu);
      s0 += kGLw[i] * f;
      s1 += kGLw[i] * f / eu;
    }
  }
  *k0 = 0.5 * width * s0;
  *dk0_db = -0.5 * width * s1;
}

// gamma + log(x) + E1(x) for x > 0 (Eq. 1p0).  For x < 1 this is the entire
// function Ein(x) = sum_{k>=1} (-1)^{k+1} x^k / (k k!); for x >= 1 it is
// evaluated from its parts with E1(x) = -Ei(-x).
double ein(double x) {
  if (x < 1.0) {
    double term = x, s = 0.0;
    for (int k = 1; k < 60; ++k) {
      s += term / k;
      term *= -x / (k + 1);
    }
    return s;
  }
  return kEulerGamma + std::log(x) - std::expint(-x);
}

// d/dx [gamma + log x + E1(x)] = (1 - e^-x)/x
double dein(double x) {
  if (x < 1e-8) return 1.0 - 0.5 * x;
  return -std::expm1(-x) / x;
}

}  // namespace

extern "C" {

// Real-space sum, Eq. (real_space_ewald):
//   phi^R_m = sum'_{p in P_D} sum_n q_n erfc(xi |x_m - x_n + p|) / |x_m - x_n + p|
// over all images with |x_mn + p| < rc; the term n == m, p == 0 is excluded.
// grad (may be NULL) receives d phi^R / d x_m, shape (T,3).
int oracle_real_space(int D, double L, double xi, double rc, long N, const double* x,
                      const double* q, long T, const long* tgt, double* phi, double* grad) {
  if (D < 0 || D > 3 || L <= 0 || xi <= 0 || rc <= 0) return 1;
  const int nimg = (int)std::ceil(rc / L) + 1;
  const int ix = D >= 1 ? nimg : 0, iy = D >= 2 ? nimg : 0, iz = D >= 3 ? nimg : 0;
#pragma omp parallel for schedule(dynamic, 4)
  for (long t = 0; t < T; ++t) {
    const long m = tgt[t];
    double s = 0.0, gx = 0.0, gy = 0.0, gz = 0.0;
    for (long n = 0; n < N; ++n) {
      for (int a = -ix; a <= ix; ++a)
        for (int b = -iy; b <= iy; ++b)
          for (int c = -iz; c <= iz; ++c) {
            if (n == m && a == 0 && b == 0 && c == 0) continue;
            const double dx = x[3 * m] - x[3 * n] + a * L;
            const double dy = x[3 * m + 1] - x[3 * n + 1] + b * L;
            const double dz = x[3 * m + 2] - x[3 * n + 2] + c * L;
            const double r = std::sqrt(dx * dx + dy * dy + dz * dz);
            if (r >= rc) continue;
            const double e = std::erfc(xi * r) / r;
            s += q[n] * e;
            // d/dr [erfc(xi r)/r] = -erfc(xi r)/r^2 - 2 xi/sqrt(pi) e^{-xi^2 r^2}/r
            const double dr = -e / r - 2.0 * xi / std::sqrt(kPi) * std::exp(-xi * xi * r * r) / r;
            gx += q[n] * dr * dx / r;
            gy += q[n] * dr * dy / r;
            gz += q[n] * dr * dz / r;
          }
    }
    phi[t] = s;
    if (grad) {
      grad[3 * t] = gx;
      grad[3 * t + 1] = gy;
      grad[3 * t + 2] = gz;
    }
  }
  return 0;
}

// k-space (Fourier-space) part phi^{DP,F} of Eq. (fourier_space_nonzero_ewald),
// evaluated through its closed forms.  nmax bounds the periodic wavenumbers,
// k_i = 2 pi n_i / L with |n_i| <= nmax.  grad may be NULL.
int oracle_kspace(int D, double L, double xi, int nmax, long N, const double* x,
                  const double* q, long T, const long* tgt, double* phi, double* grad) {
  if (D < 0 || D > 3 || L <= 0 || xi <= 0 || nmax < 0) return 1;
  const double dk = 2.0 * kPi / L;
  const double sqpi = std::sqrt(kPi);

  if (D == 3) {
    // Eq. (fourier_space_explicit_3P): (4 pi / L^3) sum_{k != 0}
    //   e^{-k^2/4xi^2}/k^2 sum_n q_n cos(k . (x_m - x_n)); the k = 0 term is
    // dropped (spherical order, neutrality, tin foil).  For each k the sum
    // over n is the structure factor S(k) = sum_n q_n e^{-i k.x_n}, and
    // sum_n q_n cos(k.(x_m - x_n)) = Re(S(k) e^{i k.x_m}).
    const int side = 2 * nmax + 1;
    const long nmodes = (long)side * side * side;
    std::vector<double> acc(4 * (size_t)T, 0.0);
#pragma omp parallel
    {
      std::vector<double> loc(4 * (size_t)T, 0.0);
#pragma omp for schedule(dynamic, 16)
      for (long mode = 0; mode < nmodes; ++mode) {
        const int a = (int)(mode / ((long)side * side)) - nmax;
        const int b = (int)((mode / side) % side) - nmax;
        const int c = (int)(mode % side) - nmax;
        if (a == 0 && b == 0 && c == 0) continue;
        const double kx = dk * a, ky = dk * b, kz = dk * c;
        const double k2 = kx * kx + ky * ky + kz * kz;
        const double f = std::exp(-k2 / (4.0 * xi * xi)) / k2;
        if (f == 0.0) continue;
        double sre = 0.0, sim = 0.0;
        for (long n = 0; n < N; ++n) {
          const double ph = kx * x[3 * n] + ky * x[3 * n + 1] + kz * x[3 * n + 2];
          sre += q[n] * std::cos(ph);
          sim -= q[n] * std::sin(ph);
        }
        for (long t = 0; t < T; ++t) {
          const long m = tgt[t];
          const double ph = kx * x[3 * m] + ky * x[3 * m + 1] + kz * x[3 * m + 2];
          const double cr = std::cos(ph), ci = std::sin(ph);
          // S e^{i k.x_m} = (sre + i sim)(cr + i ci)
          const double re = sre * cr - sim * ci, im = sre * ci + sim * cr;
          loc[4 * t] += f * re;
          // d/dx_m Re(S e^{i k.x_m}) = -k Im(S e^{i k.x_m})
          loc[4 * t + 1] -= f * kx * im;
          loc[4 * t + 2] -= f * ky * im;
          loc[4 * t + 3] -= f * kz * im;
        }
      }
#pragma omp critical
      for (size_t i = 0; i < loc.size(); ++i) acc[i] += loc[i];
    }
    const double c0 = 4.0 * kPi / (L * L * L);
    for (long t = 0; t < T; ++t) {
      phi[t] = c0 * acc[4 * t];
      if (grad) {
        grad[3 * t] = c0 * acc[4 * t + 1];
        grad[3 * t + 1] = c0 * acc[4 * t + 2];
        grad[3 * t + 2] = c0 * acc[4 * t + 3];
      }
    }
    return 0;
  }

  if (D == 2) {
#pragma omp parallel for schedule(dynamic, 1)
    for (long t = 0; t < T; ++t) {
      const long m = tgt[t];
      double s = 0.0, gx = 0.0, gy = 0.0, gz = 0.0;
      for (long n = 0; n < N; ++n) {
        const double vx = x[3 * m] - x[3 * n], vy = x[3 * m + 1] - x[3 * n + 1];
        const double z = x[3 * m + 2] - x[3 * n + 2];
        // k != 0, Eq. (2pno0):
        //  (pi/L^2) sum_{k != 0} e^{i k.v}/k [e^{kz} erfc(k/2xi + xi z)
        //                                   + e^{-kz} erfc(k/2xi - xi z)]
        double sn = 0.0, snx = 0.0, sny = 0.0, snz = 0.0;
        for (int a = -nmax; a <= nmax; ++a)
          for (int b = -nmax; b <= nmax; ++b) {
            if (a == 0 && b == 0) continue;
            const double kx = dk * a, ky = dk * b;
            const double k = std::sqrt(kx * kx + ky * ky);
            const double ap = k / (2.0 * xi) + xi * z, am = k / (2.0 * xi) - xi * z;
            // a term whose erfc argument exceeds 27 is below 1e-300 in size
            const double tp = ap > 27.0 ? 0.0 : std::exp(k * z) * std::erfc(ap);
            const double tm = am > 27.0 ? 0.0 : std::exp(-k * z) * std::erfc(am);
            const double c = std::cos(kx * vx + ky * vy), si = std::sin(kx * vx + ky * vy);
            sn += c * (tp + tm) / k;
            snx -= kx * si * (tp + tm) / k;
            sny -= ky * si * (tp + tm) / k;
            // d/dz of the bracket is k (tp - tm); the Gaussian parts cancel
            snz += c * (tp - tm);
          }
        const double cn = kPi / (L * L);
        // k = 0, Eq. (2p0): -(2 sqrt(pi)/L^2) [e^{-xi^2 z^2}/xi + sqrt(pi) z erf(xi z)]
        const double c0 = -2.0 * sqpi / (L * L);
        const double s0 = c0 * (std::exp(-xi * xi * z * z) / xi + sqpi * z * std::erf(xi * z));
        const double s0z = c0 * sqpi * std::erf(xi * z);
        s += q[n] * (cn * sn + s0);
        gx += q[n] * cn * snx;
        gy += q[n] * cn * sny;
        gz += q[n] * (cn * snz + s0z);
      }
      phi[t] = s;
      if (grad) {
        grad[3 * t] = gx;
        grad[3 * t + 1] = gy;
        grad[3 * t + 2] = gz;
      }
    }
    return 0;
  }

  if (D == 1) {
#pragma omp parallel for schedule(dynamic, 1)
    for (long t = 0; t < T; ++t) {
      const long m = tgt[t];
      double s = 0.0, gx = 0.0, gy = 0.0, gz = 0.0;
      for (long n = 0; n < N; ++n) {
        const double vx = x[3 * m] - x[3 * n];
        const double wy = x[3 * m + 1] - x[3 * n + 1], wz = x[3 * m + 2] - x[3 * n + 2];
        const double rho2 = wy * wy + wz * wz;
        const double b = xi * xi * rho2;
        // k != 0, Eq. (1pno0): (1/L) sum_{k != 0} e^{i k x} K0(k^2/4xi^2, rho^2 xi^2)
        double sn = 0.0, snx = 0.0, snb = 0.0;
        for (int a = 1; a <= nmax; ++a) {
          const double k = dk * a;
          double k0, dk0;
          incomplete_k0(k * k / (4.0 * xi * xi), b, &k0, &dk0);
          // k and -k together: 2 cos(k x)
          sn += 2.0 * std::cos(k * vx) * k0;
          snx -= 2.0 * k * std::sin(k * vx) * k0;
          snb += 2.0 * std::cos(k * vx) * dk0;
        }
        double phin = sn / L, gxn = snx / L;
        double gbn = snb / L;  // d phi / d b
        // k = 0, Eq. (1p0), n != m: -(1/L) [gamma + log(xi^2 rho^2) + E1(xi^2 rho^2)]
        if (n != m) {
          phin += -ein(b) / L;
          gbn += -dein(b) / L;
        }
        s += q[n] * phin;
        gx += q[n] * gxn;
        // db/dw_m = 2 xi^2 w
        gy += q[n] * gbn * 2.0 * xi * xi * wy;
        gz += q[n] * gbn * 2.0 * xi * xi * wz;
      }
      phi[t] = s;
      if (grad) {
        grad[3 * t] = gx;
        grad[3 * t + 1] = gy;
        grad[3 * t + 2] = gz;
      }
    }
    return 0;
  }

  // D == 0: phi^F_m = sum_{n != m} q_n erf(xi r)/r + 2 xi/sqrt(pi) q_m
#pragma omp parallel for schedule(dynamic, 4)
  for (long t = 0; t < T; ++t) {
    const long m = tgt[t];
    double s = 2.0 * xi / sqpi * q[m], gx = 0.0, gy = 0.0, gz = 0.0;
    for (long n = 0; n < N; ++n) {
      if (n == m) continue;
      const double dx = x[3 * m] - x[3 * n], dy = x[3 * m + 1] - x[3 * n + 1],
                   dz = x[3 * m + 2] - x[3 * n + 2];
      const double r = std::sqrt(dx * dx + dy * dy + dz * dz);
      const double e = std::erf(xi * r) / r;
      s += q[n] * e;
      const double dr = 2.0 * xi / sqpi * std::exp(-xi * xi * r * r) / r - e / r;
      gx += q[n] * dr * dx / r;
      gy += q[n] * dr * dy / r;
      gz += q[n] * dr * dz / r;
    }
    phi[t] = s;
    if (grad) {
      grad[3 * t] = gx;
      grad[3 * t + 1] = gy;
      grad[3 * t + 2] = gz;
    }
  }
  return 0;
}

// The plain free-space Coulomb sum sum_{n != m} q_n / |x_m - x_n| (Eq. potential
// with P_0 = {0}), and its gradient.  Used for the 0P split identity.
int oracle_coulomb_free(long N, const double* x, const double* q, long T, const long* tgt,
                        double* phi, double* grad) {
#pragma omp parallel for schedule(dynamic, 4)
  for (long t = 0; t < T; ++t) {
    const long m = tgt[t];
    double s = 0.0, gx = 0.0, gy = 0.0, gz = 0.0;
    for (long n = 0; n < N; ++n) {
      if (n == m) continue;
      const double dx = x[3 * m] - x[3 * n], dy = x[3 * m + 1] - x[3 * n + 1],
                   dz = x[3 * m + 2] - x[3 * n + 2];
      const double r = std::sqrt(dx * dx + dy * dy + dz * dz);
      s += q[n] / r;
      gx -= q[n] * dx / (r * r * r);
      gy -= q[n] * dy / (r * r * r);
      gz -= q[n] * dz / (r * r * r);
    }
    phi[t] = s;
    if (grad) {
      grad[3 * t] = gx;
      grad[3 * t + 1] = gy;
      grad[3 * t + 2] = gz;
    }
  }
  return 0;
}

// Triply periodic rectangular box with sides Ls[0..2]: the periodic lattice
// of Section 2 with a side per direction (the paper's remark that the domain
// need not be a cube).  Real space, Eq. (real_space_ewald): images
// (a Ls[0], b Ls[1], c Ls[2]) within rc, the n == m term at p = 0 excluded.
int oracle_real_space_box3(const double* Ls, double xi, double rc, long N, const double* x, const double* q,
                           long T, const long* tgt, double* phi, double* grad) {
  if (!Ls || Ls[0] <= 0 || Ls[1] <= 0 || Ls[2] <= 0 || xi <= 0 || rc <= 0) return 1;
  int ni[3];
  for (int d = 0; d < 3; ++d) ni[d] = (int)std::ceil(rc / Ls[d]) + 1;
#pragma omp parallel for schedule(dynamic, 4)
  for (long t = 0; t < T; ++t) {
    const long m = tgt[t];
    double s = 0.0, gx = 0.0, gy = 0.0, gz = 0.0;
    for (long n = 0; n < N; ++n)
      for (int a = -ni[0]; a <= ni[0]; ++a)
        for (int b = -ni[1]; b <= ni[1]; ++b)
          for (int c = -ni[2]; c <= ni[2]; ++c) {
            if (n == m && a == 0 && b == 0 && c == 0) continue;
            const double dx = x[3 * m] - x[3 * n] + a * Ls[0];
            const double dy = x[3 * m + 1] - x[3 * n + 1] + b * Ls[1];
            const double dz = x[3 * m + 2] - x[3 * n + 2] + c * Ls[2];
            const double r = std::sqrt(dx * dx + dy * dy + dz * dz);
            if (r >= rc) continue;
            const double e = std::erfc(xi * r) / r;
            s += q[n] * e;
            const double dr = -e / r - 2.0 * xi / std::sqrt(kPi) * std::exp(-xi * xi * r * r) / r;
            gx += q[n] * dr * dx / r;
            gy += q[n] * dr * dy / r;
            gz += q[n] * dr * dz / r;
          }
    phi[t] = s;
    if (grad) {
      grad[3 * t] = gx;
      grad[3 * t + 1] = gy;
      grad[3 * t + 2] = gz;
    }
  }
  return 0;
}

// Fourier-space part of the rectangular triply periodic box, Eq.
// (fourier_space_explicit_3P) with the box volume V = Ls[0] Ls[1] Ls[2] in
// place of L^3 and k = 2 pi (n1/Ls[0], n2/Ls[1], n3/Ls[2]), |n_d| <= nmax[d]:
//   (4 pi / V) sum_{k != 0} e^{-k^2/4xi^2}/k^2 Re(S(k) e^{i k.x_m}),
// S(k) = sum_n q_n e^{-i k.x_n}; the k = 0 term is dropped as in the cube.
int oracle_kspace_box3(const double* Ls, double xi, const int* nmax, long N, const double* x, const double* q,
                       long T, const long* tgt, double* phi, double* grad) {
  if (!Ls || !nmax || Ls[0] <= 0 || Ls[1] <= 0 || Ls[2] <= 0 || xi <= 0) return 1;
  if (nmax[0] < 0 || nmax[1] < 0 || nmax[2] < 0) return 1;
  const int sx = 2 * nmax[0] + 1, sy = 2 * nmax[1] + 1, sz = 2 * nmax[2] + 1;
  const long nmodes = (long)sx * sy * sz;
  std::vector<double> acc(4 * (size_t)T, 0.0);
#pragma omp parallel
  {
    std::vector<double> loc(4 * (size_t)T, 0.0);
#pragma omp for schedule(dynamic, 16)
    for (long mode = 0; mode < nmodes; ++mode) {
      const int a = (int)(mode / ((long)sy * sz)) - nmax[0];
      const int b = (int)((mode / sz) % sy) - nmax[1];
      const int c = (int)(mode % sz) - nmax[2];
      if (a == 0 && b == 0 && c == 0) continue;
      const double kx = 2.0 * kPi * a / Ls[0], ky = 2.0 * kPi * b / Ls[1], kz = 2.0 * kPi * c / Ls[2];
      const double k2 = kx * kx + ky * ky + kz * kz;
      const double f = std::exp(-k2 / (4.0 * xi * xi)) / k2;
      if (f == 0.0) continue;
      double sre = 0.0, sim = 0.0;
      for (long n = 0; n < N; ++n) {
        const double ph = kx * x[3 * n] + ky * x[3 * n + 1] + kz * x[3 * n + 2];
        sre += q[n] * std::cos(ph);
        sim -= q[n] * std::sin(ph);
      }
      for (long t = 0; t < T; ++t) {
        const long m = tgt[t];
        const double ph = kx * x[3 * m] + ky * x[3 * m + 1] + kz * x[3 * m + 2];
        const double cr = std::cos(ph), ci = std::sin(ph);
        const double re = sre * cr - sim * ci, im = sre * ci + sim * cr;
        loc[4 * t] += f * re;
        loc[4 * t + 1] -= f * kx * im;
        loc[4 * t + 2] -= f * ky * im;
        loc[4 * t + 3] -= f * kz * im;
      }
    }
#pragma omp critical
    for (size_t i = 0; i < loc.size(); ++i) acc[i] += loc[i];
  }
  const double c0 = 4.0 * kPi / (Ls[0] * Ls[1] * Ls[2]);
  for (long t = 0; t < T; ++t) {
    phi[t] = c0 * acc[4 * t];
    if (grad) {
      grad[3 * t] = c0 * acc[4 * t + 1];
      grad[3 * t + 1] = c0 * acc[4 * t + 2];
      grad[3 * t + 2] = c0 * acc[4 * t + 3];
    }
  }
  return 0;
}

// Doubly periodic lattice with a rectangular cell Ls[0] x Ls[1] in x, y and
// z free (the paper's remark that the domain need not be a cube, with the
// 2P sums of Section 2).  Real space, Eq. (real_space_ewald): images
// (a Ls[0], b Ls[1], 0) within rc, the n == m term at p = 0 excluded.
int oracle_real_space_box2(const double* Ls, double xi, double rc, long N, const double* x, const double* q,
                           long T, const long* tgt, double* phi, double* grad) {
  if (!Ls || Ls[0] <= 0 || Ls[1] <= 0 || xi <= 0 || rc <= 0) return 1;
  const int na = (int)std::ceil(rc / Ls[0]) + 1, nb = (int)std::ceil(rc / Ls[1]) + 1;
#pragma omp parallel for schedule(dynamic, 4)
  for (long t = 0; t < T; ++t) {
    const long m = tgt[t];
    double s = 0.0, gx = 0.0, gy = 0.0, gz = 0.0;
    for (long n = 0; n < N; ++n)
      for (int a = -na; a <= na; ++a)
        for (int b = -nb; b <= nb; ++b) {
          if (n == m && a == 0 && b == 0) continue;
          const double dx = x[3 * m] - x[3 * n] + a * Ls[0];
          const double dy = x[3 * m + 1] - x[3 * n + 1] + b * Ls[1];
          const double dz = x[3 * m + 2] - x[3 * n + 2];
          const double r = std::sqrt(dx * dx + dy * dy + dz * dz);
          if (r >= rc) continue;
          const double e = std::erfc(xi * r) / r;
          s += q[n] * e;
          const double dr = -e / r - 2.0 * xi / std::sqrt(kPi) * std::exp(-xi * xi * r * r) / r;
          gx += q[n] * dr * dx / r;
          gy += q[n] * dr * dy / r;
          gz += q[n] * dr * dz / r;
        }
    phi[t] = s;
    if (grad) {
      grad[3 * t] = gx;
      grad[3 * t + 1] = gy;
      grad[3 * t + 2] = gz;
    }
  }
  return 0;
}

// Fourier-space part for the rectangular 2P cell: Eqs. (2pno0) and (2p0)
// with the cell area A = Ls[0] Ls[1] in place of L^2 and
// k = 2 pi (n1/Ls[0], n2/Ls[1]), |n_d| <= nmax[d].
int oracle_kspace_box2(const double* Ls, double xi, const int* nmax, long N, const double* x, const double* q,
                       long T, const long* tgt, double* phi, double* grad) {
  if (!Ls || !nmax || Ls[0] <= 0 || Ls[1] <= 0 || xi <= 0 || nmax[0] < 0 || nmax[1] < 0) return 1;
  const double sqpi = std::sqrt(kPi), A = Ls[0] * Ls[1];
#pragma omp parallel for schedule(dynamic, 1)
  for (long t = 0; t < T; ++t) {
    const long m = tgt[t];
    double s = 0.0, gx = 0.0, gy = 0.0, gz = 0.0;
    for (long n = 0; n < N; ++n) {
      const double vx = x[3 * m] - x[3 * n], vy = x[3 * m + 1] - x[3 * n + 1];
      const double z = x[3 * m + 2] - x[3 * n + 2];
      double sn = 0.0, snx = 0.0, sny = 0.0, snz = 0.0;
      for (int a = -nmax[0]; a <= nmax[0]; ++a)
        for (int b = -nmax[1]; b <= nmax[1]; ++b) {
          if (a == 0 && b == 0) continue;
          const double kx = 2.0 * kPi * a / Ls[0], ky = 2.0 * kPi * b / Ls[1];
          const double k = std::sqrt(kx * kx + ky * ky);
          const double ap = k / (2.0 * xi) + xi * z, am = k / (2.0 * xi) - xi * z;
          const double tp = ap > 27.0 ? 0.0 : std::exp(k * z) * std::erfc(ap);
          const double tm = am > 27.0 ? 0.0 : std::exp(-k * z) * std::erfc(am);
          const double c = std::cos(kx * vx + ky * vy), si = std::sin(kx * vx + ky * vy);
          sn += c * (tp + tm) / k;
          snx -= kx * si * (tp + tm) / k;
          sny -= ky * si * (tp + tm) / k;
          snz += c * (tp - tm);
        }
      const double cn = kPi / A;
      const double c0 = -2.0 * sqpi / A;
      const double s0 = c0 * (std::exp(-xi * xi * z * z) / xi + sqpi * z * std::erf(xi * z));
      const double s0z = c0 * sqpi * std::erf(xi * z);
      s += q[n] * (cn * sn + s0);
      gx += q[n] * cn * snx;
      gy += q[n] * cn * sny;
      gz += q[n] * (cn * snz + s0z);
    }
    phi[t] = s;
    if (grad) {
      grad[3 * t] = gx;
      grad[3 * t + 1] = gy;
      grad[3 * t + 2] = gz;
    }
  }
  return 0;
}

// Exposed for the tests that pin the quadrature: K0(a,b) and dK0/db.
void oracle_incomplete_k0(double a, double b, double* k0, double* dk0_db) {
  incomplete_k0(a, b, k0, dk0_db);
}

double oracle_ein(double x) { return ein(x); }

}  // extern "C"
