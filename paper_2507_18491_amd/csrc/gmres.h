// gmres.h -- host logic of the restarted GMRES solve over the layered sum.
//
// The iteration solves K X = B with K = D - G for several right-hand sides
// in lockstep: every operator application is one call for all columns, and
// the small per-column work (Hessenberg columns, Givens rotations, the
// triangular solve, the stopping tests) runs here on the host.  Vector work
// goes through the KrylovSpace interface, so that the same logic drives the
// device vectors of a built FMM and a dense host matrix used to test it.
//
// Algorithm (Saad and Schultz's GMRES with restarts): per cycle, the true
// residual r = B - K X gives the first basis vector r / |r|; each step
// applies K to the newest basis vector, orthogonalises the result against
// the basis by classical Gram-Schmidt done twice (both passes are sets of
// inner products followed by one combined update, so the vector kernels
// read each basis vector once per pass), normalises it, and updates the QR
// factorisation of the Hessenberg matrix with one complex Givens rotation.
// The rotated right-hand side's last entry is the residual norm of the
// current least-squares iterate; a column stops its cycle when that norm is
// below tol |B| (or its Krylov space became invariant), and the cycle ends
// when every column stopped or the basis is full.  X then moves by the basis
// combination, and the true residual decides whether another cycle runs.
#pragma once
#include <math.h>

#include <algorithm>
#include <vector>

#include "special.h"

// Vectors are numbered: 0..m the basis, then W (work), X, B.
struct KrylovSpace {
  int m = 0;        // basis vectors 0..m
  int n_rhs = 1;
  int vW() const { return m + 1; }
  int vX() const { return m + 2; }
  int vB() const { return m + 3; }
  virtual ~KrylovSpace() {}
  // dst = D src - G src   (src != dst)
  virtual int apply(int src, int dst) = 0;
  // h[i * n_rhs + r] = sum conj(V_{first + i}) * w  over column r, i < count
  virtual int dots(int first, int count, int w, cd* h) = 0;
  // dst += sum_i V_{first + i} c[i * n_rhs + r]  (column r)
  virtual int combine(int first, int count, const cd* c, int dst) = 0;
  // dst = c[r] * src   (column r; dst may equal src)
  virtual int scale(int src, const cd* c, int dst) = 0;
  // w = b - w
  virtual int rsub(int b, int w) = 0;
};

struct GmresResult {
  int iters = 0, matvecs = 0, cycles = 0, converged = 0;
};

// relres: n_rhs final true relative residuals (0 for B = 0 columns).
inline int gmres_drive(KrylovSpace& S, double tol, int max_iter, double* relres, GmresResult* out) {
  const int R = S.n_rhs, m = S.m;
  const int W = S.vW(), X = S.vX(), B = S.vB();
  GmresResult res;
  std::vector<cd> t(R), c(R);
  std::vector<double> bn(R), rn(R);
  int rc = S.dots(B, 1, B, t.data());
  if (rc) return rc;
  for (int r = 0; r < R; r++) bn[r] = sqrt(std::max(0.0, t[r].x));
  // columns with B = 0 have the solution 0
  bool any_zero = false;
  for (int r = 0; r < R; r++) {
    c[r] = cd{bn[r] > 0 ? 1.0 : 0.0, 0.0};
    any_zero |= !(bn[r] > 0);
  }
  if (any_zero && (rc = S.scale(X, c.data(), X))) return rc;

  // per-column Hessenberg (column-major, (m+1) x m), rotations, rotated rhs
  std::vector<cd> H((size_t)R * (m + 1) * m), sn((size_t)R * m), g((size_t)R * (m + 1));
  std::vector<double> cs((size_t)R * m);
  std::vector<int> kr(R), live(R);
  std::vector<cd> h1((size_t)(m + 1) * R), h2((size_t)(m + 1) * R), y((size_t)m * R);
  auto Hc = [&](int r, int i, int j) -> cd& { return H[((size_t)r * m + j) * (m + 1) + i]; };

  for (;;) {
    // true residual W = B - K X and the stopping test
    if ((rc = S.apply(X, W))) return rc;
    res.matvecs++;
    if ((rc = S.rsub(B, W))) return rc;
    if ((rc = S.dots(W, 1, W, t.data()))) return rc;
    bool all = true;
    for (int r = 0; r < R; r++) {
      rn[r] = sqrt(std::max(0.0, t[r].x));
      relres[r] = bn[r] > 0 ? rn[r] / bn[r] : 0.0;
      live[r] = bn[r] > 0 && relres[r] > tol;
      all &= !live[r];
    }
    if (all) {
      res.converged = 1;
      break;
    }
    if (res.iters >= max_iter) break;
    res.cycles++;
    for (int r = 0; r < R; r++) {
      c[r] = cd{live[r] ? 1.0 / rn[r] : 0.0, 0.0};
      kr[r] = 0;
      for (int i = 0; i <= m; i++) g[(size_t)r * (m + 1) + i] = cd{0, 0};
      g[(size_t)r * (m + 1)] = cd{live[r] ? rn[r] : 0.0, 0.0};
    }
    if ((rc = S.scale(W, c.data(), 0))) return rc;
    int kmax = 0;
    for (int j = 0; j < m && res.iters < max_iter; j++) {
      if ((rc = S.apply(j, W))) return rc;
      res.iters++;
      res.matvecs++;
      // Gram-Schmidt, twice
      if ((rc = S.dots(0, j + 1, W, h1.data()))) return rc;
      for (auto& v : h1) v = -v;
      if ((rc = S.combine(0, j + 1, h1.data(), W))) return rc;
      if ((rc = S.dots(0, j + 1, W, h2.data()))) return rc;
      for (auto& v : h2) v = -v;
      if ((rc = S.combine(0, j + 1, h2.data(), W))) return rc;
      if ((rc = S.dots(W, 1, W, t.data()))) return rc;
      bool any_live = false;
      for (int r = 0; r < R; r++) {
        c[r] = cd{0, 0};
        if (!live[r]) continue;
        double eta = sqrt(std::max(0.0, t[r].x));
        for (int i = 0; i <= j; i++) Hc(r, i, j) = -(h1[(size_t)i * R + r] + h2[(size_t)i * R + r]);
        Hc(r, j + 1, j) = cd{eta, 0};
        // previous rotations
        for (int i = 0; i < j; i++) {
          double ci = cs[(size_t)r * m + i];
          cd si = sn[(size_t)r * m + i];
          cd a = Hc(r, i, j), b = Hc(r, i + 1, j);
          Hc(r, i, j) = ci * a + si * b;
          Hc(r, i + 1, j) = ci * b - cconj(si) * a;
        }
        // the new rotation zeroes the subdiagonal entry
        cd a = Hc(r, j, j);
        double bb = eta, aa = cabsd(a), tt = hypot(aa, bb);
        double ci;
        cd si;
        if (tt == 0.0) {  // K V_j = 0 on this column: singular, stop before this step
          live[r] = 0;
          continue;
        }
        if (aa == 0.0) {
          ci = 0.0;
          si = cd{1.0, 0.0};
          Hc(r, j, j) = cd{bb, 0.0};
        } else {
          cd ph = cd{a.x / aa, a.y / aa};
          ci = aa / tt;
          si = ph * (bb / tt);
          Hc(r, j, j) = ph * tt;
        }
        Hc(r, j + 1, j) = cd{0, 0};
        cs[(size_t)r * m + j] = ci;
        sn[(size_t)r * m + j] = si;
        cd gj = g[(size_t)r * (m + 1) + j];
        g[(size_t)r * (m + 1) + j] = ci * gj;
        g[(size_t)r * (m + 1) + j + 1] = -(cconj(si) * gj);
        kr[r] = j + 1;
        kmax = std::max(kmax, j + 1);
        double est = cabsd(g[(size_t)r * (m + 1) + j + 1]);
        if (est <= tol * bn[r] || !(eta > 1e-300)) {
          live[r] = 0;
        } else {
          c[r] = cd{1.0 / eta, 0.0};
          any_live = true;
        }
      }
      if (!any_live) break;
      if ((rc = S.scale(W, c.data(), j + 1))) return rc;
    }
    // least-squares coefficients and the update of X
    for (size_t i = 0; i < y.size(); i++) y[i] = cd{0, 0};
    for (int r = 0; r < R; r++)
      for (int i = kr[r] - 1; i >= 0; i--) {
        cd s = g[(size_t)r * (m + 1) + i];
        for (int l = i + 1; l < kr[r]; l++) s = s - Hc(r, i, l) * y[(size_t)l * R + r];
        y[(size_t)i * R + r] = s / Hc(r, i, i);
      }
    if (kmax > 0 && (rc = S.combine(0, kmax, y.data(), X))) return rc;
  }
  *out = res;
  return 0;
}
