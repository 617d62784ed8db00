/*
 * lm_oracle.c -- reference (oracle) evaluation of the layered-media electric
 * dyadic Green's function sum  A(x_i) = sum_j G(x_i, x_j) J_j, and of the
 * magnetic one H(x_i) = sum_j G_H(x_i, x_j) J_j (the J6..J9 form).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, plain, fp64 CPU definition
 * that the GPU fast multipole path is checked against.  Only the test suite,
 * the package smoke check and the CPU-baseline leg of the benchmark may load
 * it.  It shares no code, header, table or constant with the GPU library.
 *
 * What is computed (paper, Sec. 3.1 and Sec. 3.3, problem statement of the
 * layered sums):
 *   * free-space part, only for source and target in the same layer and
 *     x_i != x_j:  G^f = (I + grad grad / k^2) e^{ikR}/(4 pi R)
 *     (paper Sec. 2, the free-space dyadic written via the potential tensor);
 *   * reaction part, for every source/target layer pair: the inverse 2-D
 *     Fourier transform of the spectral dyadic of Sec. 3.1 (the J1..J5 form)
 *     with the free-space term removed.  The scalar coefficients phi, psi
 *     come from the two 1-D interface problems of Sec. 3.1 (TE jump
 *     [[u]] = [[u'/mu]] = 0, TM jump [[u]] = [[u'/eps]] = 0, with relative
 *     permeabilities mu (default 1) and eps proportional to k^2 / mu).
 *     The paper's four-component decomposition, images, effective locations,
 *     Z-functions and sigma densities are deliberately NOT used here: the
 *     reaction field is computed in one piece.
 *
 * Normalisation (reading of Sec. 2/3.1): outgoing e^{+ikR}, Im k_z >= 0, and
 * G = (I + grad grad/k^2) e^{ikR}/(4 pi R) in a homogeneous medium.  With the
 * normalised 1-D field u (u'' + k_z^2 u = -delta(z - z'), free part
 * u^f = i e^{i k_z |z-z'|} / (2 k_z)) the spectral dyadic is
 *   Ghat = (1/k^2) [ k^2 u_TE J1 + g kr^2 u_TM J2 + g d_z u_TM J3 - g d_z' u_TM J4
 *                    + (k^2 u_TE - g d_z d_z' u_TM) J5 / kr^2 ],
 * k the target-layer wavenumber, g = mu_t / mu_s (target over source layer:
 * the paper's TM coefficient carries mu of the target layer and its 1-D
 * source 1/mu of the source layer; g = 1 for mu = 1).  The angular integral over the spectral
 * polar angle is done analytically (integer-order Bessel identity, Sec. 3.4),
 * leaving Sommerfeld integrals in kr with J0, J1, J2.
 *
 * Contour (chosen independently of the paper's Gamma_1/Gamma_2): a half
 * ellipse from 0 to a = 1.5 max_l k_l through the fourth quadrant (passes
 * below the real-axis poles and branch points), Gauss-Legendre panels in the
 * ellipse angle, then the real axis [a, inf) with Gauss-Legendre panels of
 * length min(1, 2.5/rho_max) truncated where the slowest exponential of the
 * pair has decayed below 1e-18.
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef double complex cplx;

#define OR_MAXL 16 /* maximum number of layers */

/* ------------------------------------------------------------------ */
/* Medium: n layers, interfaces d[0] > d[1] > ... > d[n-2], wavenumbers k,
 * relative permeabilities mu (eps proportional to k^2 / mu)               */
typedef struct {
  int n;
  double d[OR_MAXL];
  double k[OR_MAXL];
  double mu[OR_MAXL];
  double kmax;
} or_medium;

static int or_layer_of(const or_medium *m, double z) {
  int l = 0;
  while (l < m->n - 1 && z < m->d[l]) l++;
  return l;
}

/* vertical wavenumber sqrt(k^2 - kr^2) on the branch Im >= 0 (Sec. 3.1) */
static cplx or_kz(double k, cplx kr) {
  cplx s = csqrt(k * k - kr * kr);
  if (cimag(s) < 0.0) s = -s;
  return s;
}

/* ------------------------------------------------------------------ */
/* Gauss-Legendre nodes/weights on [-1,1] by Newton on P_n (Golub-Welsch
 * would do equally; this is the textbook Newton iteration).              */
static void or_gauss_legendre(int n, double *x, double *w) {
  for (int i = 0; i < (n + 1) / 2; i++) {
    double z = cos(M_PI * (i + 0.75) / (n + 0.5)), pp = 0.0;
    for (int it = 0; it < 100; it++) {
      double p1 = 1.0, p2 = 0.0;
      for (int j = 1; j <= n; j++) {
        double p3 = p2;
        p2 = p1;
        p1 = ((2.0 * j - 1.0) * z * p2 - (j - 1.0) * p3) / j;
      }
      pp = n * (z * p1 - p2) / (z * z - 1.0);
      double z1 = z;
      z = z1 - p1 / pp;
      if (fabs(z - z1) < 1e-16) break;
    }
    x[i] = -z;
    x[n - 1 - i] = z;
    w[i] = w[n - 1 - i] = 2.0 / ((1.0 - z * z) * pp * pp);
  }
}

#define OR_GL 16
static double or_glx[OR_GL], or_glw[OR_GL];
static int or_gl_ready = 0;
static void or_init_gl(void) {
  if (!or_gl_ready) {
    or_gauss_legendre(OR_GL, or_glx, or_glw);
    or_gl_ready = 1;
  }
}

/* ------------------------------------------------------------------ */
/* Bessel J0, J1, J2 of complex argument by the trapezoidal rule on the
 * periodic integral J_n(z) = (1/2pi) int_0^{2pi} exp(i(z sin t - n t)) dt,
 * which converges geometrically (aliasing error ~ J_{M+n}(z)).          */
static void or_bessel012_c(cplx z, cplx out[3]) {
  int M = 2 * (int)ceil(cabs(z)) + 40;
  cplx s0 = 0, s1 = 0, s2 = 0;
  for (int j = 0; j < M; j++) {
    double t = 2.0 * M_PI * j / M;
    cplx e = cexp(I * z * sin(t));
    s0 += e;
    s1 += e * cexp(-I * t);
    s2 += e * cexp(-2.0 * I * t);
  }
  out[0] = s0 / M;
  out[1] = s1 / M;
  out[2] = s2 / M;
}

/* real argument: the C library's integer-order Bessel functions */
static void or_bessel012_r(double x, cplx out[3]) {
  out[0] = j0(x);
  out[1] = j1(x);
  out[2] = jn(2, x);
}

/* ------------------------------------------------------------------ */
/* 1-D interface problem (Sec. 3.1, the two Helmholtz interface problems)
 * for source layer s, at horizontal wavenumber kr, polarisation pol
 * (0: TE, beta_m = 1; 1: TM, beta_m = k_m^2).  In layer m the reaction
 * field is  a_m e^{i k_mz (z - d_m)} + b_m e^{-i k_mz (z - d_{m-1})}
 * (a_n-1 = b_0 = 0; every exponential has modulus <= 1).  Two unit
 * excitations: "top" (the free wave of the source reaching d_{s-1} with
 * unit exponential factor) and "bottom" (reaching d_s).  The true field is
 * u^r = S_top(z') (.)^top + S_bot(z') (.)^bot with
 * S_top = e^{i k_sz (d_{s-1} - z')}, S_bot = e^{i k_sz (z' - d_s)}.
 * amp[src][m][0..1] = (a_m, b_m).                                        */
static void or_solve_1d(const or_medium *md, cplx kr, int s, int pol,
                        cplx amp[2][OR_MAXL][2]) {
  int n = md->n, L = n - 1, N = 2 * L;
  cplx kz[OR_MAXL], E[OR_MAXL], beta[OR_MAXL];
  for (int m = 0; m < n; m++) {
    kz[m] = or_kz(md->k[m], kr);
    /* the jump conditions of Sec. 3.1: [[u' / mu]] = 0 (TE), [[u' / eps]] = 0 (TM) */
    beta[m] = pol ? md->k[m] * md->k[m] / md->mu[m] : md->mu[m];
    E[m] = (m >= 1 && m <= L - 1) ? cexp(I * kz[m] * (md->d[m - 1] - md->d[m])) : 0.0;
  }
  for (int src = 0; src < 2; src++)
    for (int m = 0; m < n; m++) amp[src][m][0] = amp[src][m][1] = 0.0;
  if (L == 0) return;
  /* unknown columns: a_m -> m (m = 0..L-1), b_m -> L-1+m (m = 1..L) */
  cplx A[2 * OR_MAXL][2 * OR_MAXL], B[2 * OR_MAXL][2];
  memset(A, 0, sizeof(A));
  memset(B, 0, sizeof(B));
  for (int i = 0; i < L; i++) {
    int up = i, lo = i + 1, r0 = 2 * i, r1 = 2 * i + 1;
    /* upper layer evaluated at its bottom face d_i */
    A[r0][up] += 1.0;
    A[r1][up] += I * kz[up] / beta[up];
    if (up >= 1) {
      A[r0][L - 1 + up] += E[up];
      A[r1][L - 1 + up] += -I * kz[up] * E[up] / beta[up];
    }
    /* lower layer evaluated at its top face d_i (subtracted) */
    if (lo <= L - 1) {
      A[r0][lo] -= E[lo];
      A[r1][lo] -= I * kz[lo] * E[lo] / beta[lo];
    }
    A[r0][L - 1 + lo] -= 1.0;
    A[r1][L - 1 + lo] -= -I * kz[lo] / beta[lo];
  }
  cplx c = I / (2.0 * kz[s]);
  if (s >= 1) { /* top excitation at interface s-1: the free wave is on the lower side */
    B[2 * (s - 1)][0] = c;
    B[2 * (s - 1) + 1][0] = I * kz[s] * c / beta[s];
  }
  if (s <= L - 1) { /* bottom excitation at interface s: free wave on the upper side */
    B[2 * s][1] = -c;
    B[2 * s + 1][1] = I * kz[s] * c / beta[s];
  }
  /* Gaussian elimination with partial pivoting */
  for (int col = 0; col < N; col++) {
    int piv = col;
    for (int r = col + 1; r < N; r++)
      if (cabs(A[r][col]) > cabs(A[piv][col])) piv = r;
    if (piv != col) {
      for (int j = 0; j < N; j++) { cplx t = A[col][j]; A[col][j] = A[piv][j]; A[piv][j] = t; }
      for (int j = 0; j < 2; j++) { cplx t = B[col][j]; B[col][j] = B[piv][j]; B[piv][j] = t; }
    }
    for (int r = col + 1; r < N; r++) {
      cplx f = A[r][col] / A[col][col];
      if (f == 0.0) continue;
      for (int j = col; j < N; j++) A[r][j] -= f * A[col][j];
      for (int j = 0; j < 2; j++) B[r][j] -= f * B[col][j];
    }
  }
  cplx X[2 * OR_MAXL][2];
  for (int r = N - 1; r >= 0; r--)
    for (int j = 0; j < 2; j++) {
      cplx acc = B[r][j];
      for (int q = r + 1; q < N; q++) acc -= A[r][q] * X[q][j];
      X[r][j] = acc / A[r][r];
    }
  for (int src = 0; src < 2; src++) {
    for (int m = 0; m <= L - 1; m++) amp[src][m][0] = X[m][src];
    for (int m = 1; m <= L; m++) amp[src][m][1] = X[L - 1 + m][src];
  }
  if (s < 1)
    for (int m = 0; m < n; m++) amp[0][m][0] = amp[0][m][1] = 0.0;
  if (s > L - 1)
    for (int m = 0; m < n; m++) amp[1][m][0] = amp[1][m][1] = 0.0;
}

/* Reaction scalars at (kr, z in layer t, z' in layer s) for one polarisation:
 * out[0] = R, out[1] = d_z R, out[2] = d_z' R, out[3] = d_z d_z' R.      */
static void or_reaction_scalars(const or_medium *md, cplx kr, int t, int s,
                                const cplx amp[2][OR_MAXL][2], double z, double zp,
                                cplx out[4]) {
  int L = md->n - 1;
  cplx kt = or_kz(md->k[t], kr), ks = or_kz(md->k[s], kr);
  cplx up = (t <= L - 1) ? cexp(I * kt * (z - md->d[t])) : 0.0;
  cplx dn = (t >= 1) ? cexp(-I * kt * (z - md->d[t - 1])) : 0.0;
  cplx St = (s >= 1) ? cexp(I * ks * (md->d[s - 1] - zp)) : 0.0;
  cplx Sb = (s <= L - 1) ? cexp(I * ks * (zp - md->d[s])) : 0.0;
  cplx ft = amp[0][t][0] * up + amp[0][t][1] * dn; /* top excitation, field in t */
  cplx fb = amp[1][t][0] * up + amp[1][t][1] * dn;
  cplx dft = I * kt * (amp[0][t][0] * up - amp[0][t][1] * dn);
  cplx dfb = I * kt * (amp[1][t][0] * up - amp[1][t][1] * dn);
  out[0] = St * ft + Sb * fb;
  out[1] = St * dft + Sb * dfb;
  out[2] = -I * ks * St * ft + I * ks * Sb * fb;
  out[3] = -I * ks * St * dft + I * ks * Sb * dfb;
}

/* Free-space scalars pushed through the same spectral machinery (pin of the
 * contour/Bessel/normalisation: must reproduce the closed form).          */
static void or_free_scalars(double k, cplx kr, double z, double zp, cplx out[4]) {
  cplx kz = or_kz(k, kr);
  double sg = (z >= zp) ? 1.0 : -1.0;
  cplx u = I / (2.0 * kz) * cexp(I * kz * fabs(z - zp));
  out[0] = u;
  out[1] = I * kz * sg * u;
  out[2] = -I * kz * sg * u;
  out[3] = kz * kz * u;
}

/* slowest vertical decay length of the reaction field between z (layer t)
 * and z' (layer s): the shortest up/down path leaving the source and
 * reaching the target after at least one interface interaction.          */
static double or_min_decay(const or_medium *md, int t, int s, double z, double zp) {
  int L = md->n - 1;
  if (t != s) return fabs(z - zp);
  double best = 1e300;
  if (t <= L - 1) best = fmin(best, (z - md->d[t]) + (zp - md->d[t]));
  if (t >= 1) best = fmin(best, (md->d[t - 1] - z) + (md->d[t - 1] - zp));
  return best;
}

/* ------------------------------------------------------------------ */
/* One Sommerfeld pair evaluation: 3x3 reaction dyadic G^r(x, x') (or the
 * free dyadic pushed through the integral when free_only != 0).          */
typedef struct {
  int ne;            /* ellipse panels */
  double depth;      /* ellipse depth */
  double a;          /* ellipse end on the real axis */
  double rho_panel;  /* rho used to size tail panels */
  double decay_stop; /* stop tail when kr * decay > decay_stop */
} or_contour;

static void or_accumulate(cplx G[3][3], cplx wgt, cplx kr, double k, const cplx Sf[4],
                          const cplx Sp[4], const cplx Jb[3], double c1, double s1,
                          double c2, double s2) {
  /* Sf: TE scalars (R, dz R, dz' R, dz dz' R), Sp: TM scalars */
  cplx k2 = k * k;
  cplx C5 = k2 * Sf[0] - Sp[3];
  cplx w = wgt * kr / k2;
  G[0][0] += w * (k2 * Sf[0] * Jb[0] - 0.5 * C5 * (Jb[0] - Jb[2] * c2));
  G[1][1] += w * (k2 * Sf[0] * Jb[0] - 0.5 * C5 * (Jb[0] + Jb[2] * c2));
  G[0][1] += w * (0.5 * C5 * Jb[2] * s2);
  G[1][0] += w * (0.5 * C5 * Jb[2] * s2);
  G[2][2] += w * (kr * kr * Sp[0] * Jb[0]);
  G[0][2] += w * (-kr * Sp[1] * Jb[1] * c1);
  G[1][2] += w * (-kr * Sp[1] * Jb[1] * s1);
  G[2][0] += w * (kr * Sp[2] * Jb[1] * c1);
  G[2][1] += w * (kr * Sp[2] * Jb[1] * s1);
}

/* Magnetic dyadic (Sec. 3.1, the J6..J9 form), normalised as
 * G_H = (1/mu_t) curl_x G_E:
 *   Ghat_H = (1/mu_t) [ u_TE J6 + g u_TM J7 + (d_z u_TE + g d_z' u_TM) J8 / kr^2
 *                       - d_z u_TE J9 ]
 * (g = mu_t/mu_s is already in the TM scalars Sp).  Angular integrals:
 * i k_x, i k_y -> -kr J1 (cos phi, sin phi); k_x k_y, k_y^2, -k_x^2 ->
 * kr^2 (-J2 s2, J0 + J2 c2, -(J0 - J2 c2)) / 2.                          */
static void or_accumulate_h(cplx G[3][3], cplx wgt, cplx kr, double inv_mu, const cplx Sf[4],
                            const cplx Sp[4], const cplx Jb[3], double c1, double s1,
                            double c2, double s2) {
  cplx w = wgt * kr * inv_mu;
  cplx a6 = Sf[0], a7 = Sp[0], a8 = Sf[1] + Sp[2], a9 = -Sf[1];
  /* J6 (row z): (-i k_y, i k_x, 0) */
  G[2][0] += w * (a6 * kr * Jb[1] * s1);
  G[2][1] += w * (-a6 * kr * Jb[1] * c1);
  /* J7 (column z): (i k_y, -i k_x, 0)^T */
  G[0][2] += w * (-a7 * kr * Jb[1] * s1);
  G[1][2] += w * (a7 * kr * Jb[1] * c1);
  /* J8 / kr^2: [[k_x k_y, k_y^2], [-k_x^2, -k_x k_y]] / kr^2 */
  G[0][0] += w * (a8 * (-0.5 * Jb[2] * s2));
  G[0][1] += w * (a8 * 0.5 * (Jb[0] + Jb[2] * c2));
  G[1][0] += w * (a8 * (-0.5) * (Jb[0] - Jb[2] * c2));
  G[1][1] += w * (a8 * 0.5 * Jb[2] * s2);
  /* J9: [[0, 1], [-1, 0]] */
  G[0][1] += w * (a9 * Jb[0]);
  G[1][0] += w * (-a9 * Jb[0]);
}

static void or_sommerfeld_pair(const or_medium *md, const or_contour *ct, const double *x,
                               const double *xp, int free_only, double kfree, int field,
                               cplx G[3][3]) {
  or_init_gl();
  for (int i = 0; i < 3; i++)
    for (int j = 0; j < 3; j++) G[i][j] = 0.0;
  double dx = x[0] - xp[0], dy = x[1] - xp[1], z = x[2], zp = xp[2];
  double rho = hypot(dx, dy);
  double phi = (rho > 0.0) ? atan2(dy, dx) : 0.0;
  double c1 = cos(phi), s1 = sin(phi), c2 = cos(2 * phi), s2 = sin(2 * phi);
  int t = free_only ? 0 : or_layer_of(md, z), s = free_only ? 0 : or_layer_of(md, zp);
  double k = free_only ? kfree : md->k[t];
  /* the TM terms of the spectral dyadic carry mu_t / mu_s (Sec. 3.1: the TM
   * coefficient is scaled by the target layer's mu and its 1-D source by
   * 1 / mu of the source layer); the TE terms carry no mu                  */
  double tm_scale = free_only ? 1.0 : md->mu[t] / md->mu[s];
  double inv_mu = free_only ? 1.0 : 1.0 / md->mu[t];
  cplx ampf[2][OR_MAXL][2], ampp[2][OR_MAXL][2];
  cplx Sf[4], Sp[4], Jb[3];
  /* ellipse: kr(th) = a/2 (1 - cos th) - i depth sin th, th in [0, pi] */
  double a = ct->a, h = ct->depth;
  for (int p = 0; p < ct->ne; p++) {
    double th0 = M_PI * p / ct->ne, th1 = M_PI * (p + 1) / ct->ne;
    for (int g = 0; g < OR_GL; g++) {
      double th = 0.5 * (th0 + th1) + 0.5 * (th1 - th0) * or_glx[g];
      cplx kr = 0.5 * a * (1.0 - cos(th)) - I * h * sin(th);
      cplx dk = 0.5 * a * sin(th) - I * h * cos(th);
      cplx wgt = 0.5 * (th1 - th0) * or_glw[g] * dk;
      if (free_only) {
        or_free_scalars(k, kr, z, zp, Sf);
        for (int q = 0; q < 4; q++) Sp[q] = Sf[q];
      } else {
        or_solve_1d(md, kr, s, 0, ampf);
        or_solve_1d(md, kr, s, 1, ampp);
        or_reaction_scalars(md, kr, t, s, ampf, z, zp, Sf);
        or_reaction_scalars(md, kr, t, s, ampp, z, zp, Sp);
        for (int q = 0; q < 4; q++) Sp[q] *= tm_scale;
      }
      or_bessel012_c(kr * rho, Jb);
      if (field)
        or_accumulate_h(G, wgt, kr, inv_mu, Sf, Sp, Jb, c1, s1, c2, s2);
      else
        or_accumulate(G, wgt, kr, k, Sf, Sp, Jb, c1, s1, c2, s2);
    }
  }
  /* real tail [a, inf) */
  double decay = free_only ? fabs(z - zp) : or_min_decay(md, t, s, z, zp);
  double len = fmin(1.0, 2.5 / fmax(ct->rho_panel, 1e-12));
  double kmax_tail = a + (ct->decay_stop + 3.0 * log(1.0 + ct->decay_stop / fmax(decay, 1e-12))) /
                             fmax(decay, 1e-12);
  int npan = (int)ceil((kmax_tail - a) / len);
  if (npan > 2000000) npan = 2000000;
  for (int p = 0; p < npan; p++) {
    double k0 = a + p * len, k1 = k0 + len;
    for (int g = 0; g < OR_GL; g++) {
      double krr = 0.5 * (k0 + k1) + 0.5 * len * or_glx[g];
      cplx kr = krr;
      cplx wgt = 0.5 * len * or_glw[g];
      if (free_only) {
        or_free_scalars(k, kr, z, zp, Sf);
        for (int q = 0; q < 4; q++) Sp[q] = Sf[q];
      } else {
        or_solve_1d(md, kr, s, 0, ampf);
        or_solve_1d(md, kr, s, 1, ampp);
        or_reaction_scalars(md, kr, t, s, ampf, z, zp, Sf);
        or_reaction_scalars(md, kr, t, s, ampp, z, zp, Sp);
        for (int q = 0; q < 4; q++) Sp[q] *= tm_scale;
      }
      or_bessel012_r(krr * rho, Jb);
      if (field)
        or_accumulate_h(G, wgt, kr, inv_mu, Sf, Sp, Jb, c1, s1, c2, s2);
      else
        or_accumulate(G, wgt, kr, k, Sf, Sp, Jb, c1, s1, c2, s2);
    }
  }
  for (int i = 0; i < 3; i++)
    for (int j = 0; j < 3; j++) G[i][j] /= 2.0 * M_PI;
}

/* textbook free-space dyadic (I + grad grad/k^2) e^{ikr}/(4 pi r) */
static void or_free_dyadic(double k, const double *R, cplx G[3][3]) {
  double r = sqrt(R[0] * R[0] + R[1] * R[1] + R[2] * R[2]);
  cplx g = cexp(I * k * r) / (4.0 * M_PI * r);
  double kr = k * r;
  cplx a = g * (1.0 + I / kr - 1.0 / (kr * kr));
  cplx b = g * (-1.0 - 3.0 * I / kr + 3.0 / (kr * kr));
  for (int i = 0; i < 3; i++)
    for (int j = 0; j < 3; j++) G[i][j] = (i == j ? a : 0.0) + b * (R[i] / r) * (R[j] / r);
}

/* textbook free-space curl: (curl (g I)) q = grad g x q, i.e. the matrix
 * [[0, -g_z, g_y], [g_z, 0, -g_x], [-g_y, g_x, 0]], grad g = g (ik - 1/r) R/r */
static void or_free_curl(double k, const double *R, cplx G[3][3]) {
  double r = sqrt(R[0] * R[0] + R[1] * R[1] + R[2] * R[2]);
  cplx g = cexp(I * k * r) / (4.0 * M_PI * r);
  cplx gp = g * (I * k - 1.0 / r);
  cplx gx = gp * R[0] / r, gy = gp * R[1] / r, gz = gp * R[2] / r;
  G[0][0] = 0.0; G[0][1] = -gz; G[0][2] = gy;
  G[1][0] = gz; G[1][1] = 0.0; G[1][2] = -gx;
  G[2][0] = -gy; G[2][1] = gx; G[2][2] = 0.0;
}

static int or_setup(or_medium *md, int n_layers, const double *d, const double *k, const double *mu) {
  if (n_layers < 1 || n_layers > OR_MAXL) return -1;
  md->n = n_layers;
  md->kmax = 0.0;
  for (int l = 0; l < n_layers; l++) {
    md->k[l] = k[l];
    md->mu[l] = mu ? mu[l] : 1.0;
    if (!(k[l] > 0.0) || !(md->mu[l] > 0.0) || !isfinite(md->mu[l])) return -2;
    if (k[l] > md->kmax) md->kmax = k[l];
  }
  for (int l = 0; l < n_layers - 1; l++) {
    md->d[l] = d[l];
    if (l > 0 && !(d[l] < d[l - 1])) return -2;
  }
  return 0;
}

static void or_default_contour(const or_medium *md, double rho_max, or_contour *ct) {
  ct->a = 1.5 * md->kmax;
  ct->depth = 0.25 * fmin(1.0, md->kmax);
  ct->ne = 16;
  ct->rho_panel = rho_max;
  ct->decay_stop = 41.5; /* e^-41.5 ~ 1e-18 */
}

/* ------------------------------------------------------------------ */
/* exported entry points (ctypes) */

/* 3x3 G(x, x') (row-major complex128 out[9]); quad_scale > 1 refines the
 * contour (more ellipse panels, shorter tail panels) for convergence checks. */
static int or_pair(int field, int n_layers, const double *d, const double *k, const double *mu,
                   const double *x, const double *xp, double quad_scale, double *out) {
  or_medium md;
  int rc = or_setup(&md, n_layers, d, k, mu);
  if (rc) return rc;
  or_contour ct;
  double rho = hypot(x[0] - xp[0], x[1] - xp[1]);
  or_default_contour(&md, rho, &ct);
  if (quad_scale > 1.0) {
    ct.ne = (int)ceil(ct.ne * quad_scale);
    ct.rho_panel *= quad_scale;
    ct.decay_stop += 4.0;
  }
  cplx G[3][3];
  or_sommerfeld_pair(&md, &ct, x, xp, 0, 0.0, field, G);
  int t = or_layer_of(&md, x[2]), s = or_layer_of(&md, xp[2]);
  double R[3] = {x[0] - xp[0], x[1] - xp[1], x[2] - xp[2]};
  if (t == s && (R[0] != 0.0 || R[1] != 0.0 || R[2] != 0.0)) {
    cplx Gf[3][3];
    if (field) {
      or_free_curl(md.k[t], R, Gf);
      for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) Gf[i][j] /= md.mu[t];
    } else {
      or_free_dyadic(md.k[t], R, Gf);
    }
    for (int i = 0; i < 3; i++)
      for (int j = 0; j < 3; j++) G[i][j] += Gf[i][j];
  }
  for (int i = 0; i < 9; i++) {
    out[2 * i] = creal(G[i / 3][i % 3]);
    out[2 * i + 1] = cimag(G[i / 3][i % 3]);
  }
  return 0;
}

int lm_oracle_pair(int n_layers, const double *d, const double *k, const double *mu, const double *x,
                   const double *xp, double quad_scale, double *out) {
  return or_pair(0, n_layers, d, k, mu, x, xp, quad_scale, out);
}

/* magnetic dyadic G_H(x, x') = (1/mu_t) curl_x G(x, x') (J6..J9 form of Sec. 3.1) */
int lm_oracle_pair_h(int n_layers, const double *d, const double *k, const double *mu, const double *x,
                     const double *xp, double quad_scale, double *out) {
  return or_pair(1, n_layers, d, k, mu, x, xp, quad_scale, out);
}

/* reaction part only (no free-space term) */
int lm_oracle_reaction_pair(int n_layers, const double *d, const double *k, const double *mu, const double *x,
                            const double *xp, double quad_scale, double *out) {
  or_medium md;
  int rc = or_setup(&md, n_layers, d, k, mu);
  if (rc) return rc;
  or_contour ct;
  or_default_contour(&md, hypot(x[0] - xp[0], x[1] - xp[1]), &ct);
  if (quad_scale > 1.0) {
    ct.ne = (int)ceil(ct.ne * quad_scale);
    ct.rho_panel *= quad_scale;
    ct.decay_stop += 4.0;
  }
  cplx G[3][3];
  or_sommerfeld_pair(&md, &ct, x, xp, 0, 0.0, 0, G);
  for (int i = 0; i < 9; i++) {
    out[2 * i] = creal(G[i / 3][i % 3]);
    out[2 * i + 1] = cimag(G[i / 3][i % 3]);
  }
  return 0;
}

/* free-space dyadic through the Sommerfeld route (pin of the machinery) and
 * the closed form; out_somm/out_closed are complex128[9].                 */
int lm_oracle_free_check(double k, const double *x, const double *xp, double *out_somm,
                         double *out_closed) {
  or_medium md;
  double kk[1] = {k};
  or_setup(&md, 1, NULL, kk, NULL);
  or_contour ct;
  or_default_contour(&md, hypot(x[0] - xp[0], x[1] - xp[1]), &ct);
  cplx G[3][3], Gf[3][3];
  or_sommerfeld_pair(&md, &ct, x, xp, 1, k, 0, G);
  double R[3] = {x[0] - xp[0], x[1] - xp[1], x[2] - xp[2]};
  or_free_dyadic(k, R, Gf);
  for (int i = 0; i < 9; i++) {
    out_somm[2 * i] = creal(G[i / 3][i % 3]);
    out_somm[2 * i + 1] = cimag(G[i / 3][i % 3]);
    out_closed[2 * i] = creal(Gf[i / 3][i % 3]);
    out_closed[2 * i + 1] = cimag(Gf[i / 3][i % 3]);
  }
  return 0;
}

/* free-space curl through the Sommerfeld route (J6, J7, J9 terms) and the
 * closed form grad g x (.)                                               */
int lm_oracle_free_check_h(double k, const double *x, const double *xp, double *out_somm,
                           double *out_closed) {
  or_medium md;
  double kk[1] = {k};
  or_setup(&md, 1, NULL, kk, NULL);
  or_contour ct;
  or_default_contour(&md, hypot(x[0] - xp[0], x[1] - xp[1]), &ct);
  cplx G[3][3], Gf[3][3];
  or_sommerfeld_pair(&md, &ct, x, xp, 1, k, 1, G);
  double R[3] = {x[0] - xp[0], x[1] - xp[1], x[2] - xp[2]};
  or_free_curl(k, R, Gf);
  for (int i = 0; i < 9; i++) {
    out_somm[2 * i] = creal(G[i / 3][i % 3]);
    out_somm[2 * i + 1] = cimag(G[i / 3][i % 3]);
    out_closed[2 * i] = creal(Gf[i / 3][i % 3]);
    out_closed[2 * i + 1] = cimag(Gf[i / 3][i % 3]);
  }
  return 0;
}

/* spectral reaction scalars for pinning the 1-D solve:
 * out = complex128[2][4]: (TE, TM) x (R, dzR, dz'R, dzdz'R) at real or
 * complex kr = (kr_re, kr_im).                                           */
int lm_oracle_spectral(int n_layers, const double *d, const double *k, const double *mu, double kr_re,
                       double kr_im, double z, double zp, double *out) {
  or_medium md;
  int rc = or_setup(&md, n_layers, d, k, mu);
  if (rc) return rc;
  cplx kr = kr_re + I * kr_im;
  int t = or_layer_of(&md, z), s = or_layer_of(&md, zp);
  cplx amp[2][OR_MAXL][2], S[4];
  for (int pol = 0; pol < 2; pol++) {
    or_solve_1d(&md, kr, s, pol, amp);
    or_reaction_scalars(&md, kr, t, s, amp, z, zp, S);
    for (int q = 0; q < 4; q++) {
      out[2 * (4 * pol + q)] = creal(S[q]);
      out[2 * (4 * pol + q) + 1] = cimag(S[q]);
    }
  }
  return 0;
}

/* Bessel check: J0, J1, J2 of complex z by the oracle's own routine */
void lm_oracle_bessel012(double zr, double zi, double *out) {
  cplx J[3];
  or_bessel012_c(zr + I * zi, J);
  for (int i = 0; i < 3; i++) {
    out[2 * i] = creal(J[i]);
    out[2 * i + 1] = cimag(J[i]);
  }
}

/* Direct sum A_i = sum_j G(x_i, x_j) J_j for n_rhs right-hand sides.
 * J: complex128 [n_rhs][n_src][3], A: complex128 [n_rhs][n_tgt][3].
 * The free-space term is skipped for coincident points; sources with an
 * all-zero current in every right-hand side are skipped (they contribute
 * exactly zero).  OpenMP over targets, fixed order over sources.        */
static int or_direct(int field, int n_layers, const double *d, const double *k, const double *mu,
                     int64_t n_src, const double *src_xyz, int n_rhs, const double *J, int64_t n_tgt,
                     const double *tgt_xyz, double *A, int n_threads) {
  or_medium md;
  int rc = or_setup(&md, n_layers, d, k, mu);
  if (rc) return rc;
  or_init_gl();
  double rho_max = 0.0;
  for (int64_t i = 0; i < n_tgt; i++)
    for (int64_t j = 0; j < n_src; j++) {
      double r = hypot(tgt_xyz[3 * i] - src_xyz[3 * j], tgt_xyz[3 * i + 1] - src_xyz[3 * j + 1]);
      if (r > rho_max) rho_max = r;
    }
  or_contour ct;
  or_default_contour(&md, rho_max, &ct);
  char *active = (char *)malloc(n_src > 0 ? n_src : 1);
  for (int64_t j = 0; j < n_src; j++) {
    active[j] = 0;
    for (int r = 0; r < n_rhs; r++)
      for (int c = 0; c < 6; c++)
        if (J[((size_t)r * n_src + j) * 6 + c] != 0.0) active[j] = 1;
  }
  if (n_threads <= 0) n_threads = 1;
#pragma omp parallel for schedule(dynamic, 1) num_threads(n_threads)
  for (int64_t i = 0; i < n_tgt; i++) {
    const double *x = tgt_xyz + 3 * i;
    int t = or_layer_of(&md, x[2]);
    cplx acc[64][3];
    int nr = n_rhs < 64 ? n_rhs : 64;
    for (int r = 0; r < nr; r++) acc[r][0] = acc[r][1] = acc[r][2] = 0.0;
    for (int64_t j = 0; j < n_src; j++) {
      if (!active[j]) continue;
      const double *xp = src_xyz + 3 * j;
      cplx G[3][3];
      or_sommerfeld_pair(&md, &ct, x, xp, 0, 0.0, field, G);
      int s = or_layer_of(&md, xp[2]);
      double R[3] = {x[0] - xp[0], x[1] - xp[1], x[2] - xp[2]};
      if (t == s && (R[0] != 0.0 || R[1] != 0.0 || R[2] != 0.0)) {
        cplx Gf[3][3];
        if (field) {
          or_free_curl(md.k[t], R, Gf);
          for (int a = 0; a < 3; a++)
            for (int b = 0; b < 3; b++) Gf[a][b] /= md.mu[t];
        } else {
          or_free_dyadic(md.k[t], R, Gf);
        }
        for (int a = 0; a < 3; a++)
          for (int b = 0; b < 3; b++) G[a][b] += Gf[a][b];
      }
      for (int r = 0; r < nr; r++) {
        const double *Jj = J + ((size_t)r * n_src + j) * 6;
        cplx q[3] = {Jj[0] + I * Jj[1], Jj[2] + I * Jj[3], Jj[4] + I * Jj[5]};
        for (int a = 0; a < 3; a++) acc[r][a] += G[a][0] * q[0] + G[a][1] * q[1] + G[a][2] * q[2];
      }
    }
    for (int r = 0; r < nr; r++)
      for (int a = 0; a < 3; a++) {
        A[(((size_t)r * n_tgt + i) * 3 + a) * 2] = creal(acc[r][a]);
        A[(((size_t)r * n_tgt + i) * 3 + a) * 2 + 1] = cimag(acc[r][a]);
      }
  }
  free(active);
  return n_rhs > 64 ? -1 : 0;
}

int lm_oracle_direct(int n_layers, const double *d, const double *k, const double *mu, int64_t n_src,
                     const double *src_xyz, int n_rhs, const double *J, int64_t n_tgt,
                     const double *tgt_xyz, double *A, int n_threads) {
  return or_direct(0, n_layers, d, k, mu, n_src, src_xyz, n_rhs, J, n_tgt, tgt_xyz, A, n_threads);
}

/* H_i = sum_j G_H(x_i, x_j) J_j, same layout and rules as lm_oracle_direct */
int lm_oracle_direct_h(int n_layers, const double *d, const double *k, const double *mu, int64_t n_src,
                       const double *src_xyz, int n_rhs, const double *J, int64_t n_tgt,
                       const double *tgt_xyz, double *A, int n_threads) {
  return or_direct(1, n_layers, d, k, mu, n_src, src_xyz, n_rhs, J, n_tgt, tgt_xyz, A, n_threads);
}

/* free-space part only (closed form, same-layer, x_i != x_j): used for the
 * cheap full-size check of the free-space FMM.                           */
int lm_oracle_direct_free(int n_layers, const double *d, const double *k, const double *mu, int64_t n_src,
                          const double *src_xyz, const double *J, int64_t n_tgt,
                          const double *tgt_xyz, double *A, int n_threads) {
  or_medium md;
  int rc = or_setup(&md, n_layers, d, k, mu);
  if (rc) return rc;
  if (n_threads <= 0) n_threads = 1;
#pragma omp parallel for schedule(static) num_threads(n_threads)
  for (int64_t i = 0; i < n_tgt; i++) {
    const double *x = tgt_xyz + 3 * i;
    int t = or_layer_of(&md, x[2]);
    cplx acc[3] = {0, 0, 0};
    for (int64_t j = 0; j < n_src; j++) {
      const double *xp = src_xyz + 3 * j;
      if (or_layer_of(&md, xp[2]) != t) continue;
      double R[3] = {x[0] - xp[0], x[1] - xp[1], x[2] - xp[2]};
      if (R[0] == 0.0 && R[1] == 0.0 && R[2] == 0.0) continue;
      cplx Gf[3][3];
      or_free_dyadic(md.k[t], R, Gf);
      const double *Jj = J + (size_t)j * 6;
      cplx q[3] = {Jj[0] + I * Jj[1], Jj[2] + I * Jj[3], Jj[4] + I * Jj[5]};
      for (int a = 0; a < 3; a++) acc[a] += Gf[a][0] * q[0] + Gf[a][1] * q[1] + Gf[a][2] * q[2];
    }
    for (int a = 0; a < 3; a++) {
      A[(i * 3 + a) * 2] = creal(acc[a]);
      A[(i * 3 + a) * 2 + 1] = cimag(acc[a]);
    }
  }
  return 0;
}
