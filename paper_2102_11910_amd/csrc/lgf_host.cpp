// Host-side lattice Green's function table and its padded spectrum.
//
// G is the lattice Green's function of the unscaled 5-point Laplacian
// (Sec. 2.1: L^-1 by the lattice Green's function), gauge G(0,0) = 0.
// Near the origin (m^2 + n^2 <= 128^2) it is evaluated from the heat
// kernel of the lattice Laplacian: e^{t Delta_h} delta at (m, n) is
// e^{-4t} I_m(2t) I_n(2t) (a product of two one-dimensional kernels), and
// a(m,n) = int_0^inf (p_t(0,0) - p_t(m,n)) dt satisfies Delta_h a = delta
// with a(0,0) = 0, so
//   G(m,n) = 1/2 int_0^inf [i_0(s)^2 - i_m(s) i_n(s)] ds,  i_k = e^{-s} I_k(s),
// by Gauss-Legendre quadrature on doubling intervals up to s = 2^17, the
// scaled Bessel functions from Miller's backward recurrence normalised by
// e^{-s} (I_0 + 2 sum_{k>=1} I_k) = 1, and the large-s expansion of i_k
// for the rest of the integral.  Farther out, the three-term far-field
// expansion.  The spectrum is the 2-D DFT of the even (2n)^2 periodic
// extension K(i,j) = G(min(i,2n-i), min(j,2n-j)) - c, which is real; only
// 0 <= k1,k2 <= n is kept.
#include <algorithm>
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

// n-point Gauss-Legendre nodes and weights on [-1, 1] (Newton on the
// Legendre recurrence)
struct GaussLegendre {
  static constexpr int n = 32;
  double x[n], w[n];
  GaussLegendre() {
    for (int i = 0; i < n; ++i) {
      double z = std::cos(kPi * (i + 0.75) / (n + 0.5)), dp = 1.0;
      for (int it = 0; it < 100; ++it) {
        double p0 = 1.0, p1 = 0.0;
        for (int k = 1; k <= n; ++k) {
          const double p2 = p1;
          p1 = p0;
          p0 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p2) / k;
        }
        dp = n * (z * p0 - p1) / (z * z - 1.0);
        const double dz = p0 / dp;
        z -= dz;
        if (std::fabs(dz) < 1e-16) break;
      }
      double p0 = 1.0, p1 = 0.0;
      for (int k = 1; k <= n; ++k) {
        const double p2 = p1;
        p1 = p0;
        p0 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p2) / k;
      }
      dp = n * (z * p0 - p1) / (z * z - 1.0);
      x[i] = z;
      w[i] = 2.0 / ((1.0 - z * z) * dp * dp);
    }
  }
};

// i_k(s) = e^{-s} I_k(s) for k = 0..K: Miller's backward recurrence
// I_{k-1} = I_{k+1} + (2k/s) I_k from an index where I_k/I_0 is below
// 1e-17 (about 9 sqrt(s) + K), normalised by i_0 + 2 sum i_k = 1 (all terms
// positive), rescaled before it can overflow
void scaled_bessel_i(double s, int K, double *out) {
  const int n0 = K + 40 + (int)(10.0 * std::sqrt(s));
  double yp = 0.0, y = 1.0, norm = 0.0;
  for (int k = n0; k >= 1; --k) {
    if (k <= K) out[k] = y;
    norm += 2.0 * y;
    const double ym = yp + (2.0 * k / s) * y;
    yp = y;
    y = ym;
    if (y > 1e250) {
      y *= 1e-250;
      yp *= 1e-250;
      norm *= 1e-250;
      for (int j = k; j <= K; ++j) out[j] *= 1e-250;
    }
  }
  out[0] = y;
  norm += y;
  for (int k = 0; k <= K; ++k) out[k] /= norm;
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

// G(m, n) for 0 <= m <= n <= kQuadRadius with m^2 + n^2 <= kQuadRadius^2,
// entry m (K+1) + n: computed once per process
const std::vector<double> &lgf_near() {
  static const std::vector<double> table = [] {
    constexpr int K = kQuadRadius, W = K + 1;
    static const GaussLegendre g;
    // intervals [0, 1/2], [1/2, 1], [1, 2], ..., [2^16, 2^17]
    std::vector<std::pair<double, double>> iv{{0.0, 0.5}};
    for (double L = 0.5; L < 131072.0; L *= 2.0) iv.push_back({L, 2.0 * L});
    const double S = iv.back().second;
    const int nodes = (int)iv.size() * GaussLegendre::n;
    // each node's terms into a row of its own (64 nodes at a time), summed
    // over the nodes in a fixed order: the table does not depend on the
    // number of threads
    constexpr int kChunk = 64;
    std::vector<double> part((size_t)kChunk * W * W), t((size_t)W * W, 0.0);
    for (int q0 = 0; q0 < nodes; q0 += kChunk) {
      const int nq = std::min(kChunk, nodes - q0);
      parallel_for(nq, [&](int c) {
        const int q = q0 + c;
        const auto &in = iv[q / GaussLegendre::n];
        const int j = q % GaussLegendre::n;
        const double mid = 0.5 * (in.first + in.second), half = 0.5 * (in.second - in.first);
        const double s = mid + half * g.x[j], wq = g.w[j] * half;
        std::vector<double> I(W);
        scaled_bessel_i(s, K, I.data());
        double *row = part.data() + (size_t)c * W * W;
        for (int m = 0; m <= K; ++m)
          for (int n = m; n <= K; ++n)
            row[m * W + n] = m * m + n * n <= K * K ? wq * (I[0] * I[0] - I[m] * I[n]) : 0.0;
      });
      for (int c = 0; c < nq; ++c)
        for (int m = 0; m <= K; ++m)
          for (int n = m; n <= K; ++n) t[m * W + n] += part[(size_t)c * W * W + m * W + n];
    }
    // beyond S: i_k(s) ~ (2 pi s)^{-1/2} sum_j (-1)^j a_j(k) s^{-j},
    // a_j(k) = a_{j-1}(k) (4k^2 - (2j-1)^2) / (8j), so the integrand is
    // (1 / (2 pi s)) sum_j d_j s^{-j} and its integral from S is
    // (1 / (2 pi)) sum_{j>=1} d_j / (j S^j)
    constexpr int kTerms = 14;
    auto coef = [](int k, double *c) {
      c[0] = 1.0;
      for (int j = 1; j < kTerms; ++j)
        c[j] = -c[j - 1] * (4.0 * k * k - (2.0 * j - 1.0) * (2.0 * j - 1.0)) / (8.0 * j);
    };
    double c0[kTerms], cm[kTerms], cn[kTerms];
    coef(0, c0);
    for (int m = 0; m <= K; ++m) {
      coef(m, cm);
      for (int n = m; n <= K; ++n) {
        if (m * m + n * n > K * K) continue;
        coef(n, cn);
        double tail = 0.0;
        for (int j = 1; j < kTerms; ++j) {
          double dj = 0.0;
          for (int i = 0; i <= j; ++i) dj += c0[i] * c0[j - i] - cm[i] * cn[j - i];
          tail += dj / (j * std::pow(S, j));
        }
        t[m * W + n] = 0.5 * t[m * W + n] + tail / (4.0 * kPi);
      }
    }
    t[0] = 0.0;
    return t;
  }();
  return table;
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
  const std::vector<double> &near = lgf_near();
  parallel_for(w, [&](int a) {
    for (int b = 0; b <= a; ++b) {
      double v;
      if ((long)a * a + (long)b * b <= (long)kQuadRadius * kQuadRadius)
        v = near[(size_t)b * (kQuadRadius + 1) + a];   // b <= a
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
