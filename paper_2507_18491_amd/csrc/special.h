// special.h -- special functions used by the layered-media dyadic FMM,
// callable from host and device (fp64).  Written from the defining
// recurrences; no vendor math internals.
//
//  * orthonormal associated Legendre functions (Condon-Shortley phase) of a
//    possibly complex angle given by (cos b, sin b) separately, so that the
//    analytic extension used in the spectral integrals (sin b = kr/k,
//    cos b = kz/k, paper Sec. 3.3 and the Chebyshev section) is taken
//    without any square root;
//  * spherical Bessel j_n (real argument) by Miller's downward recurrence,
//    y_n by the (stable) upward recurrence;
//  * Bessel J_q of complex argument by Miller's downward recurrence with a
//    normalisation picked between the two generating-function sums;
//  * Chebyshev polynomials T_l by the three-term recurrence.
#pragma once
#include <hip/hip_runtime.h>
#include <math.h>

#define LM_HD __host__ __device__ inline

// ---------------------------------------------------------------- complex
struct cd {
  double x, y;
};
LM_HD cd mk(double a, double b) { return cd{a, b}; }
LM_HD cd operator+(cd a, cd b) { return cd{a.x + b.x, a.y + b.y}; }
LM_HD cd operator-(cd a, cd b) { return cd{a.x - b.x, a.y - b.y}; }
LM_HD cd operator-(cd a) { return cd{-a.x, -a.y}; }
LM_HD cd operator*(cd a, cd b) { return cd{a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x}; }
LM_HD cd operator*(double s, cd a) { return cd{s * a.x, s * a.y}; }
LM_HD cd operator*(cd a, double s) { return cd{s * a.x, s * a.y}; }
LM_HD cd cconj(cd a) { return cd{a.x, -a.y}; }
LM_HD double cabs2(cd a) { return a.x * a.x + a.y * a.y; }
LM_HD double cabsd(cd a) { return hypot(a.x, a.y); }
LM_HD cd cdivd(cd a, cd b) {
  // Smith's algorithm
  if (fabs(b.x) >= fabs(b.y)) {
    double r = b.y / b.x, den = b.x + b.y * r;
    return cd{(a.x + a.y * r) / den, (a.y - a.x * r) / den};
  } else {
    double r = b.x / b.y, den = b.x * r + b.y;
    return cd{(a.x * r + a.y) / den, (a.y * r - a.x) / den};
  }
}
LM_HD cd operator/(cd a, cd b) { return cdivd(a, b); }
LM_HD cd cexpd(cd a) {
  double e = exp(a.x), s, c;
  s = sin(a.y);
  c = cos(a.y);
  return cd{e * c, e * s};
}
LM_HD cd csqrtd(cd a) {
  // principal square root
  double r = hypot(a.x, a.y);
  if (r == 0.0) return cd{0.0, 0.0};
  double t = sqrt(0.5 * (r + fabs(a.x)));
  if (a.x >= 0.0) return cd{t, a.y / (2.0 * t)};
  return cd{fabs(a.y) / (2.0 * t), a.y >= 0.0 ? t : -t};
}
// vertical wavenumber sqrt(k^2 - kr^2) on the branch Im >= 0
LM_HD cd kz_of(double k, cd kr) {
  cd s = csqrtd(cd{k * k, 0.0} - kr * kr);
  if (s.y < 0.0) s = -s;
  return s;
}
// i^n
LM_HD cd ipow(int n) {
  switch (((n % 4) + 4) % 4) {
    case 0: return cd{1, 0};
    case 1: return cd{0, 1};
    case 2: return cd{-1, 0};
    default: return cd{0, -1};
  }
}

// index of (n, m), -n <= m <= n, in a (p+1)^2 coefficient vector
LM_HD int nm_idx(int n, int m) { return n * n + n + m; }
// index of (n, m>=0) in a triangular table
LM_HD int tri_idx(int n, int m) { return n * (n + 1) / 2 + m; }

// sin and cos of x for |x| < 2^19 (pi/2), as needed by the near field where
// x = k r is a few units: Cody-Waite additive range reduction x = n pi/2 + t
// (W. J. Cody and W. Waite, Software Manual for the Elementary Functions,
// 1980), with pi/2 split into three parts of which the first two carry 33
// significant bits (so n times each is exact for n < 2^20; the split was
// computed from a 100-digit value of pi), followed by the Taylor series of
// sin and cos on |t| <= pi/4 up to t^17 and t^16 (truncation below 1e-17).
// Callers guarantee |x| < LM_SINCOS_RED_MAX (the host selects the library
// routine otherwise).
#define LM_SINCOS_RED_MAX 823549.0   // 2^19 pi/2
__device__ inline void lm_sincos_red(double x, double* sn, double* cs) {
  const double PIO2_1 = 1.5707963267341256, PIO2_2 = 6.077100506303966e-11, PIO2_3 = 2.0222662487959506e-21;
  const double TWO_OVER_PI = 0.6366197723675814;
  double n = rint(x * TWO_OVER_PI);
  double t = fma(-n, PIO2_1, x);
  t = fma(-n, PIO2_2, t);
  t = fma(-n, PIO2_3, t);
  double u = t * t;
  double ps = fma(u, 2.8114572543455206e-15, -7.647163731819816e-13);
  ps = fma(u, ps, 1.6059043836821613e-10);
  ps = fma(u, ps, -2.505210838544172e-08);
  ps = fma(u, ps, 2.7557319223985893e-06);
  ps = fma(u, ps, -0.0001984126984126984);
  ps = fma(u, ps, 0.008333333333333333);
  ps = fma(u, ps, -0.16666666666666666);
  double s = fma(t * u, ps, t);
  double pc = fma(u, 4.779477332387385e-14, -1.1470745597729725e-11);
  pc = fma(u, pc, 2.08767569878681e-09);
  pc = fma(u, pc, -2.755731922398589e-07);
  pc = fma(u, pc, 2.48015873015873e-05);
  pc = fma(u, pc, -0.001388888888888889);
  pc = fma(u, pc, 0.041666666666666664);
  pc = fma(u, pc, -0.5);
  double c = fma(u, pc, 1.0);
  int q = ((int)n) & 3;
  double so = (q & 1) ? c : s, co = (q & 1) ? s : c;
  *sn = (q & 2) ? -so : so;
  *cs = ((q + 1) & 2) ? -co : co;
}

template <bool RED>
__device__ inline void lm_sincos_nf(double x, double* sn, double* cs) {
  if (RED)
    lm_sincos_red(x, sn, cs);
  else
    sincos(x, sn, cs);
}

// 1/sqrt(a) for a > 0 (normal range): hardware estimate refined by two
// Newton steps y <- y + y (1/2 - (a y / 2) y)
__device__ inline double lm_rsqrt(double a) {
  double y = __builtin_amdgcn_rsq(a);
  double h = 0.5 * a * y;
  double e = fma(-h, y, 0.5);
  y = fma(y, e, y);
  h = 0.5 * a * y;
  e = fma(-h, y, 0.5);
  return fma(y, e, y);
}

#define LM_INV_SQRT_4PI 0.28209479177387814347

// Orthonormal associated Legendre functions P^m_n(cos b), 0 <= m <= n <= nmax,
// written into out[tri_idx(n, m)] (real cos/sin version).
LM_HD void legendre_r(int nmax, double c, double s, double* out) {
  out[0] = LM_INV_SQRT_4PI;
  for (int m = 1; m <= nmax; m++)
    out[tri_idx(m, m)] = -sqrt((2.0 * m + 1.0) / (2.0 * m)) * s * out[tri_idx(m - 1, m - 1)];
  for (int m = 0; m <= nmax; m++) {
    if (m + 1 <= nmax) out[tri_idx(m + 1, m)] = sqrt(2.0 * m + 3.0) * c * out[tri_idx(m, m)];
    for (int n = m + 2; n <= nmax; n++) {
      double a = sqrt((4.0 * n * n - 1.0) / ((double)n * n - (double)m * m));
      double b = sqrt(((n - 1.0) * (n - 1.0) - (double)m * m) / (4.0 * (n - 1.0) * (n - 1.0) - 1.0));
      out[tri_idx(n, m)] = a * (c * out[tri_idx(n - 1, m)] - b * out[tri_idx(n - 2, m)]);
    }
  }
}

// same for complex (cos b, sin b)
LM_HD void legendre_c(int nmax, cd c, cd s, cd* out) {
  out[0] = cd{LM_INV_SQRT_4PI, 0.0};
  for (int m = 1; m <= nmax; m++)
    out[tri_idx(m, m)] = (-sqrt((2.0 * m + 1.0) / (2.0 * m))) * (s * out[tri_idx(m - 1, m - 1)]);
  for (int m = 0; m <= nmax; m++) {
    if (m + 1 <= nmax) out[tri_idx(m + 1, m)] = sqrt(2.0 * m + 3.0) * (c * out[tri_idx(m, m)]);
    for (int n = m + 2; n <= nmax; n++) {
      double a = sqrt((4.0 * n * n - 1.0) / ((double)n * n - (double)m * m));
      double b = sqrt(((n - 1.0) * (n - 1.0) - (double)m * m) / (4.0 * (n - 1.0) * (n - 1.0) - 1.0));
      out[tri_idx(n, m)] = a * (c * out[tri_idx(n - 1, m)] - b * out[tri_idx(n - 2, m)]);
    }
  }
}

// Spherical Bessel j_n(x), n = 0..nmax, real x >= 0.  Upward recurrence
// when x > nmax (stable there), otherwise Miller's downward recurrence
// normalised by j_0 or j_1, whichever is larger in magnitude.
LM_HD void sph_jn(int nmax, double x, double* out) {
  if (x < 1e-300) {
    out[0] = 1.0;
    for (int n = 1; n <= nmax; n++) out[n] = 0.0;
    return;
  }
  double sx = sin(x), cx = cos(x);
  double j0 = sx / x;
  double j1 = (x > 0.1) ? (sx / x - cx) / x
                        : x / 3.0 * (1.0 - x * x / 10.0 * (1.0 - x * x / 28.0 * (1.0 - x * x / 54.0 * (1.0 - x * x / 88.0))));
  if (x > (double)nmax) {
    out[0] = j0;
    if (nmax >= 1) out[1] = j1;
    const double ix = 1.0 / x;
    for (int n = 1; n < nmax; n++) out[n + 1] = (2.0 * n + 1.0) * ix * out[n] - out[n - 1];
    return;
  }
  int N = nmax + 16 + (int)(x);
  double fp1 = 0.0, f = 1e-280, scale = 1.0;
  // run down from N to 0, storing n <= nmax
  const double ix = 1.0 / x;
  for (int n = N; n >= 1; n--) {
    double fm1 = (2.0 * n + 1.0) * ix * f - fp1;
    fp1 = f;
    f = fm1;
    if (n - 1 <= nmax) out[n - 1] = f;
    if (n <= nmax) out[n] = fp1;
    if (fabs(f) > 1e250) {
      f *= 1e-250;
      fp1 *= 1e-250;
      for (int q = n - 1; q <= nmax; q++)
        if (q >= 0) out[q] *= 1e-250;
    }
  }
  (void)scale;
  double norm;
  if (fabs(j0) >= fabs(j1) || nmax < 1)
    norm = j0 / out[0];
  else
    norm = j1 / out[1];
  for (int n = 0; n <= nmax; n++) out[n] *= norm;
}

// Spherical Bessel y_n(x), x > 0, n = 0..nmax, by upward recurrence
LM_HD void sph_yn(int nmax, double x, double* out) {
  double sx = sin(x), cx = cos(x);
  out[0] = -cx / x;
  if (nmax >= 1) out[1] = -cx / (x * x) - sx / x;
  for (int n = 1; n < nmax; n++) out[n + 1] = (2.0 * n + 1.0) / x * out[n] - out[n - 1];
}

// Bessel J_q(z), q = 0..qmax, complex z, by Miller's downward recurrence.
// Normalisation uses either  1 = J0 + 2 sum J_2k  or  cos z = J0 + 2 sum (-1)^k J_2k,
// whichever has less cancellation.
LM_HD void bessel_jq(int qmax, cd z, cd* out) {
  double az = cabsd(z);
  if (az < 1e-300) {
    out[0] = cd{1.0, 0.0};
    for (int q = 1; q <= qmax; q++) out[q] = cd{0.0, 0.0};
    return;
  }
  int N = qmax + 20 + (int)(az + 4.0 * sqrt(az + 1.0));
  if (N % 2) N++;
  cd two_over_z = cd{2.0, 0.0} / z;
  cd fp1 = cd{0.0, 0.0}, f = cd{1e-250, 0.0};
  cd s1 = cd{0, 0}, s2 = cd{0, 0};  // sum J0 + 2 sum J_2k, sum with (-1)^k
  double a1 = 0.0, a2 = 0.0;        // sums of magnitudes
  for (int q = 0; q <= qmax; q++) out[q] = cd{0, 0};
  for (int n = N; n >= 0; n--) {
    // f = f_n here
    if (n <= qmax) out[n] = f;
    if ((n % 2) == 0) {
      double w = (n == 0) ? 1.0 : 2.0;
      double sg = ((n / 2) % 2 == 0) ? 1.0 : -1.0;
      s1 = s1 + w * f;
      s2 = s2 + (w * sg) * f;
      a1 += w * cabsd(f);
    }
    if (n == 0) break;
    cd fm1 = (double)n * (two_over_z * f) - fp1;
    fp1 = f;
    f = fm1;
    double mag = fabs(f.x) + fabs(f.y);
    if (mag > 1e200) {
      f = 1e-200 * f;
      fp1 = 1e-200 * fp1;
      s1 = 1e-200 * s1;
      s2 = 1e-200 * s2;
      a1 *= 1e-200;
      for (int q = n; q <= qmax; q++) out[q] = 1e-200 * out[q];
    }
  }
  a2 = a1;
  cd cz = cd{cos(z.x) * cosh(z.y), -sin(z.x) * sinh(z.y)};
  // cancellation ratios: a/|s|
  double r1 = a1 / (cabsd(s1) + 1e-300);
  double r2 = a2 / (cabsd(s2) + 1e-300) * 1.0;
  cd scale;
  if (r1 <= r2 || cabsd(cz) == 0.0)
    scale = cd{1.0, 0.0} / s1;
  else
    scale = cz / s2;
  for (int q = 0; q <= qmax; q++) out[q] = out[q] * scale;
}

// Chebyshev T_l(x), l = 0..lmax, complex x
LM_HD void cheb_t(int lmax, cd x, cd* out) {
  out[0] = cd{1.0, 0.0};
  if (lmax >= 1) out[1] = x;
  for (int l = 1; l < lmax; l++) out[l + 1] = 2.0 * (x * out[l]) - out[l - 1];
}
