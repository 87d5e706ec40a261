// Host-side lattice Green's function table and its padded spectrum.
//
// G is the lattice Green's function of the unscaled 5-point Laplacian
// (Sec. 2.1: L^-1 by the lattice Green's function), gauge G(0,0) = 0:
//   G(m,n) = 1/(2 pi) int_0^pi [1 - cos(m th) e^{-n t}] / sinh t dth,
//   cosh t = 2 - cos th, n >= m >= 0,
// evaluated with composite 16-point Gauss-Legendre quadrature for
// r <= 128 and with the three-term far-field expansion beyond.
// The spectrum is the 2-D DFT of the even (2n)^2 periodic extension
// K(i,j) = G(min(i,2n-i), min(j,2n-j)) - c, which is real; only
// 0 <= k1,k2 <= n is kept.
#include <cmath>
#include <complex>
#include <thread>
#include <vector>

#include "gpf_internal.h"

namespace gpf {
namespace {

constexpr int kQuadRadius = 128;
constexpr double kPi = 3.14159265358979323846;
constexpr double kEulerGamma = 0.57721566490153286061;

struct GaussLegendre16 {
  double x[16], w[16];
  GaussLegendre16() {
    const int n = 16;
    for (int i = 0; i < n; ++i) {
      double z = std::cos(kPi * (i + 0.75) / (n + 0.5));
      double dp = 1.0;
      for (int it = 0; it < 100; ++it) {
        double p0 = 1.0, p1 = 0.0;
        for (int k = 1; k <= n; ++k) {  // Legendre recurrence
          double p2 = p1;
          p1 = p0;
          p0 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p2) / k;
        }
        dp = n * (z * p0 - p1) / (z * z - 1.0);
        const double dz = p0 / dp;
        z -= dz;
        if (std::fabs(dz) < 1e-16) break;
      }
      {  // derivative at the converged node for the weight
        double p0 = 1.0, p1 = 0.0;
        for (int k = 1; k <= n; ++k) {
          double p2 = p1;
          p1 = p0;
          p0 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p2) / k;
        }
        dp = n * (z * p0 - p1) / (z * z - 1.0);
      }
      x[i] = z;
      w[i] = 2.0 / ((1.0 - z * z) * dp * dp);
    }
  }
};

const GaussLegendre16 &gl16() {
  static GaussLegendre16 g;
  return g;
}

// integrand with n >= m, written to keep full accuracy as th -> 0
inline double integrand(double th, double m, double n) {
  double sh = std::sin(0.5 * th);
  double x = 2.0 * sh * sh;                  // cosh t - 1
  double sinh_t = std::sqrt(x * (x + 2.0));
  double t = std::log1p(x + sinh_t);         // acosh(1 + x)
  double sm = std::sin(0.5 * m * th);
  double num = 2.0 * sm * sm - std::cos(m * th) * std::expm1(-n * t);
  return num / sinh_t;
}

double lgf_quad(int a, int b) {
  int m = a < b ? a : b;
  int n = a < b ? b : a;
  if (n == 0) return 0.0;
  const GaussLegendre16 &g = gl16();
  int panels = 32 + 2 * n;
  double h = kPi / panels;
  double sum = 0.0;
  for (int p = 0; p < panels; ++p) {
    double mid = (p + 0.5) * h, half = 0.5 * h, ps = 0.0;
    for (int k = 0; k < 16; ++k) ps += g.w[k] * integrand(mid + half * g.x[k], m, n);
    sum += ps * half;
  }
  return sum / (2.0 * kPi);
}

double lgf_far(int a, int b) {
  double m = a, n = b;
  double r2 = m * m + n * n, r = std::sqrt(r2);
  double c2 = m * m / r2, s2 = n * n / r2;
  double cos4 = c2 * c2 - 6.0 * c2 * s2 + s2 * s2;
  double p8 = 43.0 * c2 * c2 * c2 * c2 - 772.0 * c2 * c2 * c2 * s2 +
              1570.0 * c2 * c2 * s2 * s2 - 772.0 * c2 * s2 * s2 * s2 +
              43.0 * s2 * s2 * s2 * s2;
  return (std::log(r) + kEulerGamma + 1.5 * std::log(2.0)) / (2.0 * kPi) -
         cos4 / (24.0 * kPi * r2) - p8 / (480.0 * kPi * r2 * r2);
}

template <class F>
void parallel_for(int count, F &&body) {
  unsigned hw = std::thread::hardware_concurrency();
  int nt = (int)std::min<unsigned>(hw ? hw : 1, 16u);
  if (nt <= 1 || count < 64) {
    for (int i = 0; i < count; ++i) body(i);
    return;
  }
  std::vector<std::thread> th;
  for (int t = 0; t < nt; ++t)
    th.emplace_back([&, t] {
      for (int i = t; i < count; i += nt) body(i);
    });
  for (auto &x : th) x.join();
}

// in-place iterative radix-2 complex FFT (forward), length N = 2^p
void fft_inplace(std::complex<double> *a, int N, const std::complex<double> *tw) {
  for (int i = 1, j = 0; i < N; ++i) {
    int bit = N >> 1;
    for (; j & bit; bit >>= 1) j ^= bit;
    j ^= bit;
    if (i < j) std::swap(a[i], a[j]);
  }
  for (int len = 2; len <= N; len <<= 1) {
    int half = len >> 1, step = N / len;
    for (int i = 0; i < N; i += len)
      for (int k = 0; k < half; ++k) {
        std::complex<double> u = a[i + k], v = a[i + k + half] * tw[k * step];
        a[i + k] = u + v;
        a[i + k + half] = u - v;
      }
  }
}

}  // namespace

void lgf_table_host(int nmax, double *table) {
  const int w = nmax + 1;
  parallel_for(w, [&](int a) {
    for (int b = 0; b <= a; ++b) {
      double v;
      if ((long)a * a + (long)b * b <= (long)kQuadRadius * kQuadRadius)
        v = lgf_quad(a, b);
      else
        v = lgf_far(a, b);
      table[(size_t)a * w + b] = v;
      table[(size_t)b * w + a] = v;
    }
  });
}

double lgf_spectrum_host(int n, const double *table, double *spec) {
  const int N = 2 * n, w = n + 1;
  double c = 0.0;
  const int h = n / 2;
  for (int a = 0; a <= h; ++a)
    for (int b = 0; b <= h; ++b) c += table[(size_t)a * w + b];
  c /= double(h + 1) * double(h + 1);

  std::vector<std::complex<double>> tw(N / 2);
  for (int k = 0; k < N / 2; ++k) {
    double ang = -2.0 * kPi * k / N;
    tw[k] = {std::cos(ang), std::sin(ang)};
  }
  // first axis: R[j][k1] for j in [0, n] (rows j and N-j of K coincide)
  std::vector<double> R((size_t)w * w);
  parallel_for(w, [&](int j) {
    std::vector<std::complex<double>> buf(N);
    for (int i = 0; i < N; ++i) {
      int ii = i <= n ? i : N - i;
      buf[i] = table[(size_t)ii * w + j] - c;
    }
    fft_inplace(buf.data(), N, tw.data());
    for (int k = 0; k <= n; ++k) R[(size_t)j * w + k] = buf[k].real();
  });
  // second axis
  parallel_for(w, [&](int k1) {
    std::vector<std::complex<double>> buf(N);
    for (int j = 0; j < N; ++j) {
      int jj = j <= n ? j : N - j;
      buf[j] = R[(size_t)jj * w + k1];
    }
    fft_inplace(buf.data(), N, tw.data());
    for (int k2 = 0; k2 <= n; ++k2) spec[(size_t)k1 * w + k2] = buf[k2].real();
  });
  return c;
}

}  // namespace gpf
