// Host-side fit of the recursive ramp-filter pair (Sec. 3): the coefficients of eq 9 are chosen
// to minimise the squared error between the filter's impulse response and the causal half h+
// of the band-limited ramp (eq 7, eq 10), with the Nelder-Mead simplex method.  An optional
// variant, not in the paper, fits the pair's frequency response to the ramp's |w| / (2 pi) in
// relative error over [pi / length, pi] instead: the time-domain criterion barely weighs the
// slowly decaying tail of h+, which carries the ramp's low-frequency behaviour.
//
// Parameterisation: the feedback polynomial 1 + a_1 z^-1 + ... + a_K z^-K is built from K
// reflection coefficients k_i = 0.9999 tanh(theta_i) by the step-up recursion, so every
// candidate is stable; for a given a the feed-forward b enters linearly and is the least
// squares solution (optionally under sum(b) = 0, a zero response at zero frequency).  The
// simplex therefore searches only the K parameters theta.  Restarts use a fixed seed.
#include <math.h>
#include <stdint.h>

#include <algorithm>
#include <vector>

#include "../../include/fhtfbp.h"

namespace {

struct Fit {
  int K, L;
  bool dc0;
  bool freq = false;           // fit the pair's frequency response instead (see solve_b_freq)
  std::vector<double> target;  // h+(n), n < L
  double target_norm2;
  std::vector<double> w;       // frequency grid of the frequency-domain fit
  std::vector<double> cw, sw;  // cos(w_k m), sin(w_k m) for m <= K, [k][m]
  double rmax = 1.0;           // bound on the pole radius (frequency-domain fit)
  // scratch
  std::vector<double> a, u, b;

  void step_up(const double* theta) {
    a.assign(K + 1, 0.0);
    a[0] = 1.0;
    std::vector<double> prev(K + 1);
    for (int m = 1; m <= K; ++m) {
      const double km = 0.9999 * tanh(theta[m - 1]);
      prev = a;
      for (int i = 1; i < m; ++i) a[i] = prev[i] + km * prev[m - i];
      a[m] = km;
    }
    // a_k rmax^k: every root of the polynomial scaled by rmax, so |pole| < rmax
    double r = 1.0;
    for (int k = 1; k <= K; ++k) {
      r *= rmax;
      a[k] *= r;
    }
  }

  // least-squares b for the current a; returns the squared error
  double solve_b() {
    u.assign(L, 0.0);
    for (int n = 0; n < L; ++n) {
      double v = (n == 0) ? 1.0 : 0.0;
      for (int k = 1; k <= K && k <= n; ++k) v -= a[k] * u[n - k];
      u[n] = v;
    }
    const int P = dc0 ? K - 1 : K;   // free parameters
    // column m of the design: response to b_m (u delayed by m); with sum(b) = 0 the last
    // coefficient is minus the sum of the others
    auto col = [&](int m, int n) -> double {
      double v = (n - m >= 0) ? u[n - m] : 0.0;
      if (dc0) v -= (n - (K - 1) >= 0) ? u[n - (K - 1)] : 0.0;
      return v;
    };
    std::vector<double> G(P * P, 0.0), r(P, 0.0);
    for (int n = 0; n < L; ++n) {
      double c[8];
      for (int m = 0; m < P; ++m) c[m] = col(m, n);
      for (int i = 0; i < P; ++i) {
        r[i] += c[i] * target[n];
        for (int j = 0; j <= i; ++j) G[i * P + j] += c[i] * c[j];
      }
    }
    double tr = 0;
    for (int i = 0; i < P; ++i) tr += G[i * P + i];
    for (int i = 0; i < P; ++i) G[i * P + i] += 1e-14 * tr + 1e-300;
    // Cholesky (lower)
    for (int j = 0; j < P; ++j) {
      double s = G[j * P + j];
      for (int k = 0; k < j; ++k) s -= G[j * P + k] * G[j * P + k];
      if (!(s > 0)) return INFINITY;
      const double d = sqrt(s);
      G[j * P + j] = d;
      for (int i = j + 1; i < P; ++i) {
        double t = G[i * P + j];
        for (int k = 0; k < j; ++k) t -= G[i * P + k] * G[j * P + k];
        G[i * P + j] = t / d;
      }
    }
    std::vector<double> z(P);
    for (int i = 0; i < P; ++i) {
      double t = r[i];
      for (int k = 0; k < i; ++k) t -= G[i * P + k] * z[k];
      z[i] = t / G[i * P + i];
    }
    for (int i = P - 1; i >= 0; --i) {
      double t = z[i];
      for (int k = i + 1; k < P; ++k) t -= G[k * P + i] * z[k];
      z[i] = t / G[i * P + i];
    }
    b.assign(K, 0.0);
    double sum = 0;
    for (int m = 0; m < P; ++m) {
      b[m] = z[m];
      sum += z[m];
    }
    if (dc0) b[K - 1] = -sum;
    double err = 0;
    for (int n = 0; n < L; ++n) {
      double g = 0;
      for (int m = 0; m < K && m <= n; ++m) g += b[m] * u[n - m];
      const double d = g - target[n];
      err += d * d;
    }
    return err;
  }

  // Frequency-domain variant: the pair (causal plus anticausal half, Sec. 3) has the response
  // G(w) = 2 Re(B(e^{iw}) / A(e^{iw})); the band-limited ramp of eq 7 (unit sample spacing)
  // has |w| / (2 pi).  Least squares on the relative error (G - R) / R over the grid w_k: G is
  // linear in b, so b is again a linear least-squares solution for the current a.
  double solve_b_freq() {
    const int P = dc0 ? K - 1 : K;
    const int M = (int)w.size();
    std::vector<double> G(P * P, 0.0), r(P, 0.0);
    std::vector<double> resp(K);
    auto basis = [&](int kf, double* out) {   // 2 Re(e^{-i w m} / A(e^{i w})), m < K
      const double* c = &cw[(size_t)kf * (K + 1)];
      const double* sn = &sw[(size_t)kf * (K + 1)];
      double ar = 1.0, ai = 0.0;
      for (int k = 1; k <= K; ++k) {
        ar += a[k] * c[k];
        ai -= a[k] * sn[k];
      }
      const double den = ar * ar + ai * ai;
      for (int m = 0; m < K; ++m)
        out[m] = 2.0 * (c[m] * ar - sn[m] * ai) / den;   // Re(z conj(A)) / |A|^2, z = e^{-iwm}
    };
    const double two_pi = 6.283185307179586;
    for (int k = 0; k < M; ++k) {
      basis(k, resp.data());
      const double R = w[k] / two_pi;
      double c[8];
      for (int m = 0; m < P; ++m) c[m] = (resp[m] - (dc0 ? resp[K - 1] : 0.0)) / R;
      for (int i = 0; i < P; ++i) {
        r[i] += c[i];
        for (int j = 0; j <= i; ++j) G[i * P + j] += c[i] * c[j];
      }
    }
    double tr = 0;
    for (int i = 0; i < P; ++i) tr += G[i * P + i];
    for (int i = 0; i < P; ++i) G[i * P + i] += 1e-14 * tr + 1e-300;
    for (int j = 0; j < P; ++j) {
      double sum = G[j * P + j];
      for (int k = 0; k < j; ++k) sum -= G[j * P + k] * G[j * P + k];
      if (!(sum > 0)) return INFINITY;
      const double d = sqrt(sum);
      G[j * P + j] = d;
      for (int i = j + 1; i < P; ++i) {
        double t = G[i * P + j];
        for (int k = 0; k < j; ++k) t -= G[i * P + k] * G[j * P + k];
        G[i * P + j] = t / d;
      }
    }
    std::vector<double> z(P);
    for (int i = 0; i < P; ++i) {
      double t = r[i];
      for (int k = 0; k < i; ++k) t -= G[i * P + k] * z[k];
      z[i] = t / G[i * P + i];
    }
    for (int i = P - 1; i >= 0; --i) {
      double t = z[i];
      for (int k = i + 1; k < P; ++k) t -= G[k * P + i] * z[k];
      z[i] = t / G[i * P + i];
    }
    b.assign(K, 0.0);
    double sum = 0;
    for (int m = 0; m < P; ++m) {
      b[m] = z[m];
      sum += z[m];
    }
    if (dc0) b[K - 1] = -sum;
    double err = 0;
    for (int k = 0; k < M; ++k) {
      basis(k, resp.data());
      double g = 0;
      for (int m = 0; m < K; ++m) g += b[m] * resp[m];
      const double d = g / (w[k] / two_pi) - 1.0;
      err += d * d;
    }
    return err;
  }

  double cost(const double* theta) {
    step_up(theta);
    return freq ? solve_b_freq() : solve_b();
  }
};

uint64_t next_u64(uint64_t& s) {   // splitmix64
  uint64_t z = (s += 0x9E3779B97F4A7C15ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}
double normal(uint64_t& s) {
  const double u1 = ((next_u64(s) >> 11) + 0.5) * (1.0 / 9007199254740992.0);
  const double u2 = ((next_u64(s) >> 11) + 0.5) * (1.0 / 9007199254740992.0);
  return sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2);
}

// Nelder-Mead with the standard coefficients (1, 2, 1/2, 1/2).
double nelder_mead(Fit& f, std::vector<double>& x0, int iters) {
  const int D = (int)x0.size();
  std::vector<std::vector<double>> pts(D + 1, x0);
  std::vector<double> val(D + 1);
  for (int i = 0; i < D; ++i) pts[i + 1][i] += 0.5;
  for (int i = 0; i <= D; ++i) val[i] = f.cost(pts[i].data());
  std::vector<int> ord(D + 1);
  std::vector<double> cen(D), xr(D), xe(D), xc(D);
  for (int it = 0; it < iters; ++it) {
    for (int i = 0; i <= D; ++i) ord[i] = i;
    std::sort(ord.begin(), ord.end(), [&](int p, int q) { return val[p] < val[q]; });
    const int best = ord[0], worst = ord[D], second = ord[D - 1];
    if (fabs(val[worst] - val[best]) <= 1e-18 * (fabs(val[best]) + 1e-300)) break;
    for (int d = 0; d < D; ++d) {
      double s = 0;
      for (int i = 0; i <= D; ++i)
        if (i != worst) s += pts[i][d];
      cen[d] = s / D;
    }
    for (int d = 0; d < D; ++d) xr[d] = cen[d] + (cen[d] - pts[worst][d]);
    const double fr = f.cost(xr.data());
    if (fr < val[best]) {
      for (int d = 0; d < D; ++d) xe[d] = cen[d] + 2.0 * (cen[d] - pts[worst][d]);
      const double fe = f.cost(xe.data());
      if (fe < fr) {
        pts[worst] = xe;
        val[worst] = fe;
      } else {
        pts[worst] = xr;
        val[worst] = fr;
      }
    } else if (fr < val[second]) {
      pts[worst] = xr;
      val[worst] = fr;
    } else {
      const bool outside = fr < val[worst];
      for (int d = 0; d < D; ++d)
        xc[d] = outside ? cen[d] + 0.5 * (xr[d] - cen[d]) : cen[d] + 0.5 * (pts[worst][d] - cen[d]);
      const double fc = f.cost(xc.data());
      if (fc < (outside ? fr : val[worst])) {
        pts[worst] = xc;
        val[worst] = fc;
      } else {
        for (int i = 0; i <= D; ++i) {
          if (i == best) continue;
          for (int d = 0; d < D; ++d) pts[i][d] = pts[best][d] + 0.5 * (pts[i][d] - pts[best][d]);
          val[i] = f.cost(pts[i].data());
        }
      }
    }
  }
  int bi = 0;
  for (int i = 1; i <= D; ++i)
    if (val[i] < val[bi]) bi = i;
  x0 = pts[bi];
  return val[bi];
}

}  // namespace

extern "C" int fbp_fit_ramp_iir(int32_t order, int32_t length, uint32_t flags, double* b,
                                double* a, double* rel_err) {
  if (order < 1 || order > 8 || length < order + 1 || length > (1 << 20) || !b || !a)
    return FBP_EINVAL;
  if (flags & ~3u) return FBP_EINVAL;
  const bool dc0 = (flags & 1u) != 0;
  if (dc0 && order < 2) return FBP_EINVAL;
  Fit f;
  f.K = order;
  f.L = length;
  f.dc0 = dc0;
  f.freq = (flags & 2u) != 0;
  if (f.freq) {
    // 256 frequencies spaced evenly in log w from pi / length (the lowest a row of `length`
    // samples resolves) to pi
    const int M = 256;
    const double lo = log(3.14159265358979323846 / length), hi = log(3.14159265358979323846);
    f.w.resize(M);
    for (int k = 0; k < M; ++k) f.w[k] = exp(lo + (hi - lo) * k / (M - 1));
    f.cw.resize((size_t)M * (order + 1));
    f.sw.resize((size_t)M * (order + 1));
    for (int k = 0; k < M; ++k)
      for (int m = 0; m <= order; ++m) {
        f.cw[(size_t)k * (order + 1) + m] = cos(f.w[k] * m);
        f.sw[(size_t)k * (order + 1) + m] = sin(f.w[k] * m);
      }
    // poles within radius 1 - 2 / length: the recursion's slowest mode decays over about half
    // a row instead of running on past the window (left free, the fit of the lowest
    // frequencies pushes poles onto the unit circle)
    f.rmax = 1.0 - 2.0 / length;
  }
  f.target.assign(length, 0.0);
  const double pi = 3.14159265358979323846;
  f.target[0] = 0.125;   // h(0) / 2
  for (int n = 1; n < length; ++n) f.target[n] = (n % 2) ? -1.0 / ((pi * n) * (pi * n)) : 0.0;
  f.target_norm2 = 0;
  for (double v : f.target) f.target_norm2 += v * v;

  uint64_t seed = 0x5EEDull + (uint64_t)order * 7919u + (uint64_t)dc0;
  const int starts = 12;
  const int iters = 800 * order;
  double best = INFINITY;
  std::vector<double> best_theta;
  for (int s = 0; s < starts; ++s) {
    std::vector<double> th(order);
    for (int i = 0; i < order; ++i) th[i] = normal(seed);
    double v = nelder_mead(f, th, iters);
    v = std::min(v, nelder_mead(f, th, iters));   // one restart from the optimum
    if (v < best) {
      best = v;
      best_theta = th;
    }
  }
  if (!isfinite(best)) return FBP_EUNSTABLE;
  f.cost(best_theta.data());
  for (int k = 0; k < order; ++k) {
    b[k] = f.b[k];
    a[k] = f.a[k + 1];
  }
  if (rel_err) *rel_err = f.freq ? sqrt(best / (double)f.w.size()) : sqrt(best / f.target_norm2);
  return FBP_OK;
}
