// plan.cpp -- host planner of the layered-media dyadic FMM.
//
// Builds, from the medium and the point sets:
//  * the reaction components (target layer, source layer, arrival and
//    departure directions) with their polarization images and effective
//    locations (paper Sec. 3.1, the images/effective-location definitions
//    and the sign table of the Z functions);
//  * one octree per free-space layer (uniform depth) and, per reaction
//    component, a source tree over the images and a target tree over the
//    effective locations.  The two reaction trees share the x-y lattice and
//    are anchored on the two sides of the gap that always separates images
//    from effective locations (Sec. 3.2), so every box centre of one tree
//    lies strictly on its own side; boxes touching the gap are refined until
//    no adjacent source/target boxes remain (Sec. 3.4, the S2T discussion),
//    hence no direct reaction interactions are needed;
//  * interaction lists, grouped into M2L classes (targets with the same
//    lattice parity and distance to the gap share one list of offsets);
//  * table cases for the reaction M2L (one per distinct (rho, z, z') box
//    geometry and level, Sec. 3.4) and the Sommerfeld quadrature nodes;
//  * Chebyshev coefficients of the associated Legendre functions
//    (Appendix B) and of the affine Chebyshev change of variable
//    (Appendix A), and the Gaunt table of the free-space translations.
#include "plan.h"

#include <stdarg.h>
#include <stdio.h>

#include <algorithm>
#include <array>
#include <climits>
#include <cmath>
#include <cstring>
#include <atomic>
#include <functional>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <unordered_set>

std::string lm_fmt(const char* fmt, ...) {
  char buf[1024];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  return std::string(buf);
}

// ------------------------------------------------------------------ algebra

// Chebyshev coefficients of T_j(a x + b) = sum_s C[j][s] T_s(x), j, s <= jmax
// (Appendix A), from T_{j+1}(y) = 2 y T_j(y) - T_{j-1}(y) and the product rule
// 2 x T_s(x) = T_{s+1}(x) + T_{|s-1|}(x).  Row stride jmax+1.
void lm_cheb_affine(int jmax, double a, double b, std::vector<double>& C) {
  int W = jmax + 1;
  C.assign((size_t)W * W, 0.0);
  C[0] = 1.0;
  if (jmax >= 1) {
    C[W + 0] = b;
    C[W + 1] = a;
  }
  for (int j = 1; j < jmax; j++) {
    double* cj = &C[(size_t)j * W];
    double* cm = &C[(size_t)(j - 1) * W];
    double* cn = &C[(size_t)(j + 1) * W];
    for (int s = 0; s <= j; s++) {
      double v = cj[s];
      if (v == 0.0) continue;
      cn[s] += 2.0 * b * v;
      cn[s + 1] += a * v;
      cn[s == 0 ? 1 : s - 1] += a * v;
    }
    for (int s = 0; s <= j - 1; s++) cn[s] -= cm[s];
  }
}

// K_n of Appendix B: degree in cos(2 theta) of P^m_n / tau_nm
int lm_cheb_K(int n, int m) {
  m = m < 0 ? -m : m;
  if (n % 2 == 0) return n / 2;
  return (m % 2 == 0) ? (n + 1) / 2 : (n - 1) / 2;
}

// tau type: 0 -> 1, 1 -> sec, 2 -> sin, 3 -> tan  (Appendix B)
int lm_tau_type(int n, int m) {
  m = m < 0 ? -m : m;
  bool ne = (n % 2 == 0), me = (m % 2 == 0);
  if (ne && me) return 0;
  if (!ne && me) return 1;
  if (!ne && !me) return 2;
  return 3;
}

// B[tri(n,m)][k]: P^m_n(cos t) = tau_nm(t) sum_k B^k T_k(cos 2t), m >= 0
// (Appendix B).  The coefficients are obtained by exact Chebyshev
// interpolation of the polynomial P^m_n / tau_nm in x = cos 2t at
// Chebyshev-Gauss points (more points than the degree), which reproduces
// the appendix's expansion without its recursion constants.
// Row stride KS = (p+1)/2 + 2.
void lm_legendre_cheb(int p, std::vector<double>& B) {
  int KS = (p + 1) / 2 + 2;
  int ntri = (p + 1) * (p + 2) / 2;
  B.assign((size_t)ntri * KS, 0.0);
  int NC = KS + 6;
  std::vector<double> Pt((size_t)ntri);
  for (int i = 0; i < NC; i++) {
    double x = cos(M_PI * (i + 0.5) / NC);
    double th = 0.5 * acos(x);
    double c = cos(th), s = sin(th);
    legendre_r(p, c, s, Pt.data());
    for (int n = 0; n <= p; n++)
      for (int m = 0; m <= n; m++) {
        double tau;
        switch (lm_tau_type(n, m)) {
          case 0: tau = 1.0; break;
          case 1: tau = 1.0 / c; break;
          case 2: tau = s; break;
          default: tau = s / c; break;
        }
        double f = Pt[tri_idx(n, m)] / tau;
        int K = lm_cheb_K(n, m);
        double tk0 = 1.0, tk1 = x;
        for (int k = 0; k <= K; k++) {
          double tk = (k == 0) ? 1.0 : (k == 1 ? x : 2.0 * x * tk1 - tk0);
          if (k >= 2) {
            tk0 = tk1;
            tk1 = tk;
          }
          B[(size_t)tri_idx(n, m) * KS + k] += (k == 0 ? 1.0 : 2.0) / NC * f * tk;
        }
      }
  }
}

// Gaunt coefficients G(nu,mu; n,m; q, mu-m) = int Y^mu_nu conj(Y^m_n) conj(Y^{mu-m}_q)
// by Gauss-Legendre quadrature (exact: polynomial integrand).
long long lm_gaunt_index(int p, int nu, int mu, int n, int m, int q) {
  long long P = (long long)(p + 1) * (p + 1);
  return (((long long)nm_idx(nu, mu) * P) + nm_idx(n, m)) * (2 * p + 1) + q;
}

static void gauss_legendre(int n, std::vector<double>& x, std::vector<double>& w) {
  x.resize(n);
  w.resize(n);
  for (int i = 0; i < (n + 1) / 2; i++) {
    double z = cos(M_PI * (i + 0.75) / (n + 0.5)), pp = 0;
    for (int it = 0; it < 100; it++) {
      double p1 = 1, p2 = 0;
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

void lm_gaunt_table(int p, std::vector<double>& G) {
  int Q = 2 * p;
  long long P = (long long)(p + 1) * (p + 1);
  G.assign((size_t)(P * P * (2 * p + 1)), 0.0);
  int ng = 2 * p + 2;
  std::vector<double> xg, wg;
  gauss_legendre(ng, xg, wg);
  int ntri = (Q + 1) * (Q + 2) / 2;
  std::vector<double> Pl((size_t)ng * ntri);
  for (int g = 0; g < ng; g++) legendre_r(Q, xg[g], sqrt(1.0 - xg[g] * xg[g]), &Pl[(size_t)g * ntri]);
  auto Ph = [&](int g, int n, int m) {
    double v = Pl[(size_t)g * ntri + tri_idx(n, m < 0 ? -m : m)];
    return (m < 0 && (m % 2)) ? -v : v;
  };
  for (int nu = 0; nu <= p; nu++)
    for (int mu = -nu; mu <= nu; mu++)
      for (int n = 0; n <= p; n++)
        for (int m = -n; m <= n; m++) {
          int s = mu - m;
          for (int q = std::abs(n - nu); q <= n + nu; q++) {
            if (((n + nu + q) & 1) || std::abs(s) > q) continue;
            double acc = 0;
            for (int g = 0; g < ng; g++) acc += wg[g] * Ph(g, nu, mu) * Ph(g, n, m) * Ph(g, q, s);
            G[lm_gaunt_index(p, nu, mu, n, m, q)] = 2.0 * M_PI * acc;
          }
        }
}

// ------------------------------------------------------------ components

// Valid reaction components (Sec. 3.1): a wave arriving at the target going
// down needs an interface above the target layer, going up one below; the
// same for the departure at the source.  Fills lt, ls, up_t, up_s, sgn and the
// image/effective-location maps; returns the count.
int lm_enumerate_components(const Medium& med, std::vector<InstParams>& out) {
  int L = med.n - 1;
  out.clear();
  for (int l = 0; l <= L; l++)
    for (int lp = 0; lp <= L; lp++)
      for (int ut = 1; ut >= 0; ut--)
        for (int us = 1; us >= 0; us--) {
          if (!ut && l < 1) continue;
          if (ut && l > L - 1) continue;
          if (us && lp < 1) continue;
          if (!us && lp > L - 1) continue;
          InstParams ip;
          memset(&ip, 0, sizeof(ip));
          ip.kind = 1;
          ip.lt = l;
          ip.ls = lp;
          ip.up_t = ut;
          ip.up_s = us;
          ip.kt = med.k[l];
          ip.ks = med.k[lp];
          // sign of the Z exponent
          if (!us)
            ip.sgn = (l <= lp) ? 1 : -1;
          else
            ip.sgn = (l < lp) ? 1 : -1;
          // polarization image of the source (z' -> as z' + bs)
          if (!us) {
            if (l <= lp) { ip.as = -1; ip.bs = 2 * med.d[lp]; }
            else { ip.as = 1; ip.bs = 0; }
          } else {
            if (l < lp) { ip.as = 1; ip.bs = 0; }
            else { ip.as = -1; ip.bs = 2 * med.d[lp - 1]; }
          }
          // effective location of the target (z -> at z + bt)
          bool refl;
          if (ut && us) refl = !(l < lp);
          else if (ut && !us) refl = !(l <= lp);
          else if (!ut && us) refl = (l < lp);
          else refl = (l <= lp);
          if (!refl) { ip.at = 1; ip.bt = 0; }
          else if (ut) { ip.at = -1; ip.bt = 2 * med.d[l]; }
          else { ip.at = -1; ip.bt = 2 * med.d[l - 1]; }
          out.push_back(ip);
        }
  return (int)out.size();
}

// ------------------------------------------------------------------ trees

static const int DK = LM_TREE_DK;  // key depth

static inline uint64_t spread3(uint64_t v) {
  v &= 0xFFFFF;
  v = (v | (v << 32)) & 0x1F00000000FFFFull;
  v = (v | (v << 16)) & 0x1F0000FF0000FFull;
  v = (v | (v << 8)) & 0x100F00F00F00F00Full;
  v = (v | (v << 4)) & 0x10C30C30C30C30C3ull;
  v = (v | (v << 2)) & 0x1249249249249249ull;
  return v;
}

struct KeyRec {
  uint64_t key;
  int id;   // point id
  int tag;  // 0 source, 1 target
};

static void radix_sort(std::vector<KeyRec>& a) {
  std::vector<KeyRec> b(a.size());
  for (int pass = 0; pass < 8; pass++) {
    int sh = pass * 8;
    size_t cnt[257] = {0};
    for (auto& r : a) cnt[((r.key >> sh) & 255) + 1]++;
    bool trivial = false;
    for (int i = 0; i < 256; i++)
      if (cnt[i + 1] == a.size()) trivial = true;
    if (trivial) continue;
    for (int i = 0; i < 256; i++) cnt[i + 1] += cnt[i];
    for (auto& r : a) b[cnt[(r.key >> sh) & 255]++] = r;
    a.swap(b);
  }
}

struct HTree {
  double x0, y0, z0, S0;
  int zflip;  // j = iz (0) or j = 2^l - 1 - iz (1)
  // per box
  std::vector<int> lvl, ix, iy, iz, parent, child0, nchild, oct, u0, u1, a0, a1, b0, b1;
  std::vector<int> lvl_start;
  std::vector<KeyRec> recs;    // sorted union
  std::vector<int> permA, permB;
  int nbox() const { return (int)lvl.size(); }
  int j(int b) const { return zflip ? ((1 << lvl[b]) - 1 - iz[b]) : iz[b]; }
  double S(int l) const { return S0 / (double)(1 << l); }
  void centre(int b, double* c) const {
    double s = S(lvl[b]);
    c[0] = x0 + (ix[b] + 0.5) * s;
    c[1] = y0 + (iy[b] + 0.5) * s;
    c[2] = z0 + (iz[b] + 0.5) * s;
  }
};

// An octree over tagged points (positions pos[3*i]): first the records
// sorted by Morton key (tree_sort, or a sorter outside the planner), then the
// boxes (tree_boxes), where split(level, n, j, S) decides whether a box is
// refined.
static void tree_sort(HTree& T, const std::vector<double>& pos, const std::vector<int>& ids,
                      const std::vector<int>& tags) {
  size_t n = ids.size();
  T.recs.resize(n);
  double inv = (double)(1 << DK) / T.S0;
  for (size_t i = 0; i < n; i++) {
    const double* x = &pos[3 * i];
    long long ux = (long long)floor((x[0] - T.x0) * inv);
    long long uy = (long long)floor((x[1] - T.y0) * inv);
    long long uz = (long long)floor((x[2] - T.z0) * inv);
    long long mx = (1 << DK) - 1;
    ux = std::min(std::max(ux, 0LL), mx);
    uy = std::min(std::max(uy, 0LL), mx);
    uz = std::min(std::max(uz, 0LL), mx);
    T.recs[i].key = spread3(ux) | (spread3(uy) << 1) | (spread3(uz) << 2);
    T.recs[i].id = ids[i];
    T.recs[i].tag = tags[i];
  }
  radix_sort(T.recs);
}
template <class Split>
static void tree_boxes(HTree& T, Split split) {
  size_t n = T.recs.size();
  std::vector<int> cntA(n + 1, 0);
  for (size_t i = 0; i < n; i++) cntA[i + 1] = cntA[i] + (T.recs[i].tag == 0);
  T.permA.clear();
  T.permB.clear();
  for (size_t i = 0; i < n; i++) (T.recs[i].tag == 0 ? T.permA : T.permB).push_back(T.recs[i].id);
  auto push_box = [&](int l, int px, int py, int pz, int par, int oc, int u0, int u1) {
    T.lvl.push_back(l);
    T.ix.push_back(px);
    T.iy.push_back(py);
    T.iz.push_back(pz);
    T.parent.push_back(par);
    T.child0.push_back(-1);
    T.nchild.push_back(0);
    T.oct.push_back(oc);
    T.u0.push_back(u0);
    T.u1.push_back(u1);
    T.a0.push_back(cntA[u0]);
    T.a1.push_back(cntA[u1]);
    T.b0.push_back(u0 - cntA[u0]);
    T.b1.push_back(u1 - cntA[u1]);
  };
  T.lvl_start.clear();
  if (n == 0) {
    T.lvl_start.push_back(0);
    return;
  }
  push_box(0, 0, 0, 0, -1, -1, 0, (int)n);
  T.lvl_start.push_back(0);
  for (int l = 0; l < DK; l++) {
    int b0 = T.lvl_start.back(), b1 = T.nbox();
    if (b0 == b1) break;
    T.lvl_start.push_back(b1);
    bool any = false;
    for (int b = b0; b < b1; b++) {
      int cnt = T.u1[b] - T.u0[b];
      if (!split(l, cnt, T.j(b), T.S(l))) continue;
      any = true;
      int sh = 3 * (DK - 1 - l);
      int first = T.nbox();
      int u = T.u0[b];
      while (u < T.u1[b]) {
        int dig = (int)((T.recs[u].key >> sh) & 7);
        int v = u;
        while (v < T.u1[b] && (int)((T.recs[v].key >> sh) & 7) == dig) v++;
        push_box(l + 1, 2 * T.ix[b] + (dig & 1), 2 * T.iy[b] + ((dig >> 1) & 1),
                 2 * T.iz[b] + ((dig >> 2) & 1), b, dig, u, v);
        u = v;
      }
      T.child0[b] = first;
      T.nchild[b] = T.nbox() - first;
    }
    if (!any) break;
  }
  if (T.lvl_start.back() != T.nbox()) T.lvl_start.push_back(T.nbox());
}

// The boxes of a sorted tree from their first records: starts[l] lists, in
// increasing order, the first record of every box at level l (level 0: the
// root).  The same boxes, in the same order, as tree_boxes with the rule the
// starts were formed by: a level's boxes are the runs of equal key prefix
// inside the split boxes of the level above.
static void tree_boxes_from(HTree& T, const std::vector<std::vector<int>>& starts) {
  size_t n = T.recs.size();
  std::vector<int> cntA(n + 1, 0);
  for (size_t i = 0; i < n; i++) cntA[i + 1] = cntA[i] + (T.recs[i].tag == 0);
  T.permA.clear();
  T.permB.clear();
  for (size_t i = 0; i < n; i++) (T.recs[i].tag == 0 ? T.permA : T.permB).push_back(T.recs[i].id);
  auto push_box = [&](int l, int px, int py, int pz, int par, int oc, int u0, int u1) {
    T.lvl.push_back(l);
    T.ix.push_back(px);
    T.iy.push_back(py);
    T.iz.push_back(pz);
    T.parent.push_back(par);
    T.child0.push_back(-1);
    T.nchild.push_back(0);
    T.oct.push_back(oc);
    T.u0.push_back(u0);
    T.u1.push_back(u1);
    T.a0.push_back(cntA[u0]);
    T.a1.push_back(cntA[u1]);
    T.b0.push_back(u0 - cntA[u0]);
    T.b1.push_back(u1 - cntA[u1]);
  };
  T.lvl_start.clear();
  if (n == 0) {
    T.lvl_start.push_back(0);
    return;
  }
  push_box(0, 0, 0, 0, -1, -1, 0, (int)n);
  T.lvl_start.push_back(0);
  for (size_t l = 1; l < starts.size() && (int)l <= DK; l++) {
    const std::vector<int>& v = starts[l];
    if (v.empty()) break;
    const int b0 = T.lvl_start.back(), b1 = T.nbox();  // the parents' level
    T.lvl_start.push_back(b1);
    const int sh = 3 * (DK - (int)l);
    int pb = b0;
    for (size_t i = 0; i < v.size(); i++) {
      const int u = v[i];
      while (pb < b1 && u >= T.u1[pb]) pb++;
      if (pb >= b1 || u < T.u0[pb]) break;  // (not inside a box of the level above)
      const int u1 = (i + 1 < v.size() && v[i + 1] < T.u1[pb]) ? v[i + 1] : T.u1[pb];
      const int dig = (int)((T.recs[u].key >> sh) & 7);
      if (T.child0[pb] < 0) T.child0[pb] = T.nbox();
      T.nchild[pb]++;
      push_box((int)l, 2 * T.ix[pb] + (dig & 1), 2 * T.iy[pb] + ((dig >> 1) & 1), 2 * T.iz[pb] + ((dig >> 2) & 1),
               pb, dig, u, u1);
    }
  }
  if (T.lvl_start.back() != T.nbox()) T.lvl_start.push_back(T.nbox());
}

static inline uint64_t ckey(int x, int y, int z) {
  return (uint64_t)(uint32_t)x | ((uint64_t)(uint32_t)y << 21) | ((uint64_t)(uint32_t)z << 42);
}

// ------------------------------------------------------------------ plan

namespace {

struct MatKey {
  int kind;  // 0 free M2L, 1 M2M, 2 L2L
  long long kq;  // quantised wavenumber
  int p;
  long long sq;  // quantised box size of the level
  int a, b, c;
  bool operator<(const MatKey& o) const {
    return std::tie(kind, kq, p, sq, a, b, c) < std::tie(o.kind, o.kq, o.p, o.sq, o.a, o.b, o.c);
  }
};

// one M2L pair (global box ids) with its class key and offset
struct M2LRec {
  int gid, l, px, py, c3, dx, dy, dz, s, t;
  M2LRec() {}  // fields left unset: the concatenated list is first written by host threads
};
// lattice of an instance: instances with equal keys share M2L classes
struct LatKey {
  int free, lt, ls, up_t, up_s, p;
  long long kq, s0q, tzq, szq, rq;
  bool operator<(const LatKey& o) const {
    return std::tie(free, lt, ls, up_t, up_s, p, kq, s0q, tzq, szq, rq) <
           std::tie(o.free, o.lt, o.ls, o.up_t, o.up_s, o.p, o.kq, o.s0q, o.tzq, o.szq, o.rq);
  }
};
struct LatGroup {
  int inst;  // first instance of the group (its parameters serve the group)
  bool free;
  double S0, Tz0, Sz0, rref;
};

}  // namespace

std::string lm_make_plan(Plan& pl, const Medium& med, const PlanParams& prm, int64_t n_src,
                         const double* src, int64_t n_tgt, const double* tgt) {
  int64_t so[2] = {0, n_src}, to[2] = {0, n_tgt};
  return lm_make_plan_multi(pl, med, prm, 1, so, src, to, tgt);
}

unsigned lm_host_thread_count() {
  const char* e = getenv("LMFMM_HOST_THREADS");
  if (e && *e) {
    char* end = nullptr;
    const long v = strtol(e, &end, 10);
    if (end && *end == 0 && v >= 1 && v <= 256) return (unsigned)v;
  }
  return std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
}

std::string lm_make_plan_multi(Plan& pl, const Medium& med, const PlanParams& prm, int n_geom,
                               const int64_t* src_off, const double* src, const int64_t* tgt_off,
                               const double* tgt, const TreeSorter* sorter) {
  pl = Plan();
  pl.med = med;
  pl.prm = prm;
  pl.p = prm.p;
  pl.pf = prm.p_free > 0 ? prm.p_free : prm.p;
  pl.n_src = src_off[n_geom];
  pl.n_tgt = tgt_off[n_geom];
  int L = med.n - 1;
  int pmax = std::max(pl.p, pl.pf);

  // instances
  std::vector<InstParams> comps;
  lm_enumerate_components(med, comps);
  struct IGeom {
    InstParams ip;
    std::vector<int> sid, tid;      // point ids
    std::vector<double> spos, tpos; // positions in instance coordinates
    double zs0, zs1, zt0, zt1;
    double S0, eps, X0, Y0;         // lattice of the geometry: x-y origin and root size
  };
  std::vector<IGeom> geo;
  // per geometry: its first instance, layer lists, x-y bounds
  struct GeoRange {
    size_t geo0, geo1;
    double xmin, ymin, ext;
  };
  std::vector<GeoRange> granges;
  std::vector<std::vector<std::vector<int>>> src_in_g, tgt_in_g;
  std::vector<int> geo_of;  // geometry of each instance
  for (int gi = 0; gi < n_geom; gi++) {
    const int64_t s_lo = src_off[gi], s_hi = src_off[gi + 1], t_lo = tgt_off[gi], t_hi = tgt_off[gi + 1];
    if (s_hi == s_lo && t_hi == t_lo) continue;
    const int gx = (int)granges.size();
    GeoRange gr;
    gr.geo0 = geo.size();
    // layer membership
    src_in_g.emplace_back(med.n);
    tgt_in_g.emplace_back(med.n);
    std::vector<std::vector<int>>& src_in = src_in_g.back();
    std::vector<std::vector<int>>& tgt_in = tgt_in_g.back();
    for (int64_t i = s_lo; i < s_hi; i++) src_in[med.layer_of(src[3 * i + 2])].push_back((int)i);
    for (int64_t i = t_lo; i < t_hi; i++) tgt_in[med.layer_of(tgt[3 * i + 2])].push_back((int)i);
    // lattice of this geometry: common x-y origin and root size for every tree
    double xmin = 1e300, ymin = 1e300, xmax = -1e300, ymax = -1e300;
    for (int64_t i = s_lo; i < s_hi; i++) {
      xmin = std::min(xmin, src[3 * i]);
      xmax = std::max(xmax, src[3 * i]);
      ymin = std::min(ymin, src[3 * i + 1]);
      ymax = std::max(ymax, src[3 * i + 1]);
    }
    for (int64_t i = t_lo; i < t_hi; i++) {
      xmin = std::min(xmin, tgt[3 * i]);
      xmax = std::max(xmax, tgt[3 * i]);
      ymin = std::min(ymin, tgt[3 * i + 1]);
      ymax = std::max(ymax, tgt[3 * i + 1]);
    }
    gr.xmin = xmin;
    gr.ymin = ymin;
    gr.ext = std::max(xmax - xmin, ymax - ymin);
    if (prm.components & 1) {
      for (int l = 0; l <= L; l++) {
        if (src_in[l].empty() || tgt_in[l].empty()) continue;
        IGeom g;
        memset(&g.ip, 0, sizeof(g.ip));
        g.ip.kind = 0;
        g.ip.lt = g.ip.ls = l;
        g.ip.kt = g.ip.ks = med.k[l];
        g.ip.at = g.ip.as = 1;
        g.ip.sgn = 1;
        geo.push_back(g);
        geo_of.push_back(gx);
      }
    }
    if (prm.components & 2) {
      for (auto& c : comps) {
        if (src_in[c.ls].empty() || tgt_in[c.lt].empty()) continue;
        IGeom g;
        g.ip = c;
        geo.push_back(g);
        geo_of.push_back(gx);
      }
    }
    gr.geo1 = geo.size();
    granges.push_back(gr);
  }
  if (geo.empty()) return "";
  // every instance's points in its own coordinates (images and effective
  // locations of a reaction component), on host threads
  auto fill = [&](size_t q) {
    IGeom& g = geo[q];
    const InstParams& c = g.ip;
    g.sid = src_in_g[geo_of[q]][c.ls];
    g.tid = tgt_in_g[geo_of[q]][c.lt];
    g.spos.resize(3 * g.sid.size());
    g.tpos.resize(3 * g.tid.size());
    g.zs0 = g.zt0 = 1e300;
    g.zs1 = g.zt1 = -1e300;
    for (size_t u = 0; u < g.sid.size(); u++) {
      const int i = g.sid[u];
      const double z = c.kind == 0 ? src[3 * i + 2] : c.as * src[3 * i + 2] + c.bs;
      g.spos[3 * u] = src[3 * i];
      g.spos[3 * u + 1] = src[3 * i + 1];
      g.spos[3 * u + 2] = z;
      g.zs0 = std::min(g.zs0, z);
      g.zs1 = std::max(g.zs1, z);
    }
    for (size_t u = 0; u < g.tid.size(); u++) {
      const int i = g.tid[u];
      const double z = c.kind == 0 ? tgt[3 * i + 2] : c.at * tgt[3 * i + 2] + c.bt;
      g.tpos[3 * u] = tgt[3 * i];
      g.tpos[3 * u + 1] = tgt[3 * i + 1];
      g.tpos[3 * u + 2] = z;
      g.zt0 = std::min(g.zt0, z);
      g.zt1 = std::max(g.zt1, z);
    }
    if (c.kind == 0) {
      // one tree over the layer's sources and targets: one z range
      g.zs0 = g.zt0 = std::min(g.zs0, g.zt0);
      g.zs1 = g.zt1 = std::max(g.zs1, g.zt1);
    }
  };
  auto run_threads = [&](size_t n, const std::function<void(size_t)>& fn) {
    const unsigned nth = lm_host_thread_count();
    std::atomic<size_t> next_i{0};
    auto work = [&]() {
      for (size_t i = next_i++; i < n; i = next_i++) fn(i);
    };
    std::vector<std::thread> pool;
    for (unsigned t = 1; t < nth && t < n; t++) pool.emplace_back(work);
    work();
    for (auto& th : pool) th.join();
  };
  run_threads(geo.size(), fill);
  for (const GeoRange& gr : granges) {
    double ext = gr.ext;
    for (size_t q = gr.geo0; q < gr.geo1; q++) {
      const IGeom& g = geo[q];
      const InstParams& c = g.ip;
      if (c.kind == 0) {
        ext = std::max(ext, g.zs1 - g.zs0);
        continue;
      }
      // images and effective locations must lie on the two sides of a gap
      double gap = c.sgn > 0 ? g.zt0 - g.zs1 : g.zs0 - g.zt1;
      if (!(gap > 0))
        return lm_fmt("reaction component (%d,%d,%s,%s): images and effective locations are not "
                      "separated (a point lies on an interface?)",
                      c.lt, c.ls, c.up_t ? "up" : "down", c.up_s ? "up" : "down");
      ext = std::max(ext, std::max(g.zs1 - g.zs0, g.zt1 - g.zt0));
    }
    // root size: the power of two at or above the extent (with room for the
    // anchor snapping of the reaction trees below), a function of this
    // geometry alone, so that geometries of like size share box sizes level by
    // level (and translation tables) whether built together or apart
    const double need = ext * (1.0 + 1.0 / 256) + 1e-300;
    double S0 = 1.0;
    while (S0 < need) S0 *= 2.0;
    while (S0 * 0.5 >= need) S0 *= 0.5;
    double eps = 1e-9 * S0;
    double X0 = gr.xmin - eps, Y0 = gr.ymin - eps;
    for (size_t q = gr.geo0; q < gr.geo1; q++) {
      geo[q].S0 = S0;
      geo[q].eps = eps;
      geo[q].X0 = X0;
      geo[q].Y0 = Y0;
    }
  }

  auto kquant = [](double k) { return (long long)llround(k * 1e12); };
  std::map<MatKey, long long> matmap;
  auto alloc_mat = [&](const MatKey& key, long long size, const TransJob* job) -> long long {
    auto it = matmap.find(key);
    if (it != matmap.end()) return it->second;
    long long off = pl.mat_size;
    pl.mat_size += size;
    matmap[key] = off;
    if (job) {
      TransJob j = *job;
      j.mat = off;
      pl.trans.push_back(j);
    }
    return off;
  };

  int KB = (pmax + 1) / 2;  // maximal Chebyshev index K_n
  pl.kmaxcheb = KB;
  std::map<std::tuple<int, int, long long, long long, long long>, int> casemap;
  std::vector<double> off_ratio;  // per M2L offset: (r_s + r_t) / |c_t - c_s|
  std::vector<M2LRec> recs;       // M2L pairs of every instance
  std::vector<std::vector<M2LRec>> irecs(geo.size());  // the same, per instance
  std::vector<std::array<int, 3>> irec_base(geo.size());  // per instance: source, target box base, lattice group
  std::map<LatKey, int> latmap;
  std::vector<LatGroup> lat;
  std::vector<double> inst_S0;    // root size of each instance's lattice

  std::vector<double> s2t_rho_of;  // per instance: largest horizontal S2T pair distance, -1 if none
  // every instance's trees first, on host threads: its sort, its depth
  // (cost models) and its boxes depend on its own points alone; the
  // records, lists and tables below are then built in instance order
  struct Prep {
    HTree S, T;
    double Dgap = 0;
    int depth_used = 0;
    std::string err;
  };
  std::vector<Prep> preps(geo.size());
  auto prepare = [&](size_t gi) {
    const IGeom& g = geo[gi];
    Prep& pr = preps[gi];
    const double S0 = g.S0, eps = g.eps, X0 = g.X0, Y0 = g.Y0;
    InstParams ip = g.ip;
    ip.p = ip.kind == 0 ? pl.pf : pl.p;
    ip.P = (ip.p + 1) * (ip.p + 1);
    int P = ip.P;
    HTree& S = pr.S;
    HTree& T = pr.T;
    S.x0 = T.x0 = X0;
    S.y0 = T.y0 = Y0;
    S.S0 = T.S0 = S0;
    std::vector<int> tagS, tagT;
    bool free = ip.kind == 0;
    double Dgap = 0;
    int depth_used = 0;
    if (free) {
      S.z0 = g.zs0 - eps;
      S.zflip = 0;
      std::vector<double> pos = g.spos;
      pos.insert(pos.end(), g.tpos.begin(), g.tpos.end());
      std::vector<int> ids = g.sid;
      ids.insert(ids.end(), g.tid.begin(), g.tid.end());
      std::vector<int> tags(g.sid.size(), 0);
      tags.resize(ids.size(), 1);
      int D = prm.free_depth;
      if (D <= 0) {
        // cost model: exact near-field pair count vs M2L work per depth, with
        // the measured rates of the two kernels (about 1e-11 s per near pair
        // and 1.9e-13 s per complex multiply-add of the M2L GEMM; adaptive
        // orders keep about 2/3 of the dense 3 P^2 work per pair).  Cell
        // occupancies come from a dense grid per level (depth <= 7), so
        // clustered points get deeper trees than uniform ones.
        const double t_pair = 1.0e-11, t_m2l_pair = 3.0 * P * (double)P * 0.67 * 1.9e-13;
        const int DMAXC = 7;
        std::vector<uint32_t> ucell(3 * ids.size());
        double inv = (double)(1 << DMAXC) / S0;
        for (size_t i = 0; i < ids.size(); i++) {
          long long mx = (1 << DMAXC) - 1;
          ucell[3 * i] = (uint32_t)std::min(std::max((long long)floor((pos[3 * i] - S.x0) * inv), 0LL), mx);
          ucell[3 * i + 1] = (uint32_t)std::min(std::max((long long)floor((pos[3 * i + 1] - S.y0) * inv), 0LL), mx);
          ucell[3 * i + 2] = (uint32_t)std::min(std::max((long long)floor((pos[3 * i + 2] - S.z0) * inv), 0LL), mx);
        }
        double best = 1e300, m2l_acc = 0;
        for (int Dc = 2; Dc <= DMAXC; Dc++) {
          int n1 = 1 << Dc, sh = DMAXC - Dc;
          std::vector<int> cs((size_t)n1 * n1 * n1, 0), ct((size_t)n1 * n1 * n1, 0);
          for (size_t i = 0; i < ids.size(); i++) {
            size_t c = ((size_t)(ucell[3 * i + 2] >> sh) * n1 + (ucell[3 * i + 1] >> sh)) * n1 + (ucell[3 * i] >> sh);
            if (tags[i] == 0) cs[c]++; else ct[c]++;
          }
          double pairs = 0, occ_t = 0, nb_occ = 0;
          for (int z = 0; z < n1; z++)
            for (int y = 0; y < n1; y++)
              for (int x = 0; x < n1; x++) {
                size_t c = ((size_t)z * n1 + y) * n1 + x;
                if (!ct[c]) continue;
                occ_t += 1;
                double ns = 0;
                for (int dz = -1; dz <= 1; dz++)
                  for (int dy = -1; dy <= 1; dy++)
                    for (int dx = -1; dx <= 1; dx++) {
                      int xx = x + dx, yy = y + dy, zz = z + dz;
                      if (xx < 0 || yy < 0 || zz < 0 || xx >= n1 || yy >= n1 || zz >= n1) continue;
                      int v = cs[((size_t)zz * n1 + yy) * n1 + xx];
                      ns += v;
                      nb_occ += v > 0;
                    }
                pairs += ct[c] * ns;
              }
          // M2L pairs at this level: occupied target boxes x 189 interaction
          // slots x the occupied fraction of their neighbourhoods
          m2l_acc += occ_t > 0 ? occ_t * 189.0 * (nb_occ / (27.0 * occ_t)) : 0.0;
          double c = pairs * t_pair + m2l_acc * t_m2l_pair;
          if (c < best) {
            best = c;
            D = Dc;
          }
        }
      }
      depth_used = D;
      if (!sorter) tree_sort(S, pos, ids, tags);

    } else {
      // anchors on the two sides of the gap, moved outward to multiples of a
      // power-of-two fraction delta of S0 (at most S0 / 1024 and an eighth of
      // the gap), so that geometries whose points come equally close to the
      // interface share anchors, hence M2L tables and GEMMs
      const double raw = ip.sgn > 0 ? (g.zt0 - eps) - (g.zs1 + eps) : (g.zs0 - eps) - (g.zt1 + eps);
      double delta = S0 / 1024.0;
      while (delta > raw / 8.0) delta *= 0.5;
      if (ip.sgn > 0) {
        const double tb = floor((g.zt0 - eps) / delta) * delta, st = ceil((g.zs1 + eps) / delta) * delta;
        S.z0 = st - S0;
        S.zflip = 1;
        T.z0 = tb;
        T.zflip = 0;
        Dgap = tb - st;
      } else {
        const double sb = floor((g.zs0 - eps) / delta) * delta, tt = ceil((g.zt1 + eps) / delta) * delta;
        S.z0 = sb;
        S.zflip = 0;
        T.z0 = tt - S0;
        T.zflip = 1;
        Dgap = sb - tt;
      }
      // D1: the first level whose boxes are no larger than the gap (no
      // adjacent source/target leaves remain).  With the direct near field
      // enabled, the boxes next to the gap may stop one level earlier when
      // the direct (S2T) pairs of that level cost less than the M2L work of
      // the last level (measured rates: about 2.3e-9 s per S2T pair, 2.9e-8 s
      // per reaction M2L pair at p = 12 with adaptive orders; about 50 M2L
      // pairs per box at the finest level).
      int D1 = 0;
      while (S0 / (double)(1 << D1) > Dgap) D1++;
      if (D1 > prm.max_depth)
      {
        pr.err = lm_fmt("reaction component (%d,%d): points are too close to an interface "
                        "(gap %.3e needs %d tree levels, limit %d)",
                        ip.lt, ip.ls, Dgap, D1, prm.max_depth);
        return;
      }
      int Dmax = D1;
      if (prm.react_s2t && D1 >= 2) {
        // distance of each point from the gap plane of its tree
        auto hz_t = [&](double z) { return T.zflip ? (T.z0 + S0 - z) : (z - T.z0); };
        auto hz_s = [&](double z) { return S.zflip ? (S.z0 + S0 - z) : (z - S.z0); };
        auto cell = [&](double x, double y, double sl) {
          long long cx = (long long)floor((x - X0) / sl), cy = (long long)floor((y - Y0) / sl);
          return (cx << 32) ^ (cy & 0xffffffffLL);
        };
        double s1 = S0 / (double)(1 << D1), sb = 2.0 * s1;
        std::unordered_map<long long, int> tb1;  // occupied level-D1 target boxes next to the gap
        std::unordered_map<long long, long long> ct, cs;  // level D1-1, first layer: counts per x-y cell
        for (size_t i = 0; i < g.tid.size(); i++) {
          double x = g.tpos[3 * i], y = g.tpos[3 * i + 1], h = hz_t(g.tpos[3 * i + 2]);
          if (h < sb) {
            tb1[cell(x, y, s1) * 2 + (h >= s1 ? 1 : 0)] = 1;
            ct[cell(x, y, sb)]++;
          }
        }
        for (size_t i = 0; i < g.sid.size(); i++) {
          double h = hz_s(g.spos[3 * i + 2]);
          if (h < sb) cs[cell(g.spos[3 * i], g.spos[3 * i + 1], sb)]++;
        }
        // direct work in lane rounds: a work item takes up to LM_S2T_CHUNK
        // targets of a leaf against all its near sources, LM_S2T_CHUNK pairs
        // per round, and a round costs about the same however many of its
        // lanes hold a pair
        double rounds = 0, item_max = 0;
        for (auto& kv : ct) {
          long long cx = kv.first >> 32, cy = (long long)(int)(kv.first & 0xffffffffLL);
          long long ns = 0;
          for (int dx = -1; dx <= 1; dx++)
            for (int dy = -1; dy <= 1; dy++) {
              auto it = cs.find(((cx + dx) << 32) ^ ((cy + dy) & 0xffffffffLL));
              if (it != cs.end()) ns += it->second;
            }
          const long long nt = kv.second, CH = LM_S2T_CHUNK;
          rounds += (double)((nt / CH) * ns + ((nt % CH) * ns + CH - 1) / CH);
          item_max = std::max(item_max, (double)((std::min(nt, CH) * ns + CH - 1) / CH));
        }
        // a work item runs its rounds on one wave (about 0.85e-4 s each), so
        // the launch lasts at least as long as its longest item: dense leaves
        // next to the gap make a few long items and the direct path slow
        double c_s2t = std::max(rounds * (double)LM_S2T_CHUNK * 2.3e-9, item_max * 0.85e-4);
        double c_m2l = (double)tb1.size() * 50.0 * 9.0 * (double)P * P * 8.0 * 0.6 / 43e12;
        // the rate holds while every direct pair has a rho <= 7.5 on Gamma_1
        // (J0..J2 by their power series); adjacent level-(D1-1) leaves reach
        // rho = 2 sqrt(2) sb, and beyond that bound the general complex
        // Bessel routine makes a pair many times dearer
        const double a_c = prm.contour_a > 0 ? prm.contour_a : 1.5 * med.kmax;
        const bool series_range = a_c * 2.0 * M_SQRT2 * sb <= 7.5;
        if (prm.react_s2t == 2 || (series_range && c_s2t < c_m2l)) Dmax = D1 - 1;
      }
      // every reaction pair direct: single-box trees, whose one source and
      // one target box are adjacent (the component's Sommerfeld integral for
      // every pair, no expansion and no truncation of the method)
      if (prm.react_s2t == 3) Dmax = 0;
      depth_used = Dmax;
      if (!sorter) {
        tree_sort(S, g.spos, g.sid, std::vector<int>(g.sid.size(), 0));
        tree_sort(T, g.tpos, g.tid, std::vector<int>(g.tid.size(), 1));
      }
    }
    pr.Dgap = Dgap;
    pr.depth_used = depth_used;
  };
  run_threads(geo.size(), prepare);
  // (an instance whose depth failed gets no trees; the loop below returns
  // the first error in instance order)
  std::map<const HTree*, std::vector<std::vector<int>>> tree_starts;  // a sorter's boxes per tree
  if (sorter) {
    // every tree's records keyed and sorted in one call: per instance the
    // source tree (the free-space tree holds the layer's sources, then its
    // targets), then the target tree of a reaction component
    std::vector<TreeJob> jobs;
    std::vector<TreeSeg> segs;
    std::vector<HTree*> trees;
    for (size_t gi = 0; gi < geo.size(); gi++) {
      if (!preps[gi].err.empty()) continue;
      const IGeom& g = geo[gi];
      const InstParams& c = g.ip;
      const auto& sl = src_in_g[geo_of[gi]][c.ls];
      const auto& tl = tgt_in_g[geo_of[gi]][c.lt];
      HTree& S = preps[gi].S;
      HTree& T = preps[gi].T;
      const int D = preps[gi].depth_used;
      if (c.kind == 0) {
        jobs.push_back(TreeJob{S.x0, S.y0, S.z0, S.S0, (int)segs.size(), 2, D, 0, S.zflip});
        segs.push_back(TreeSeg{sl.data(), (int)sl.size(), 0, 0, 1.0, 0.0});
        segs.push_back(TreeSeg{tl.data(), (int)tl.size(), 1, 1, 1.0, 0.0});
        trees.push_back(&S);
      } else {
        jobs.push_back(TreeJob{S.x0, S.y0, S.z0, S.S0, (int)segs.size(), 1, D, 1, S.zflip});
        segs.push_back(TreeSeg{sl.data(), (int)sl.size(), 0, 0, c.as, c.bs});
        trees.push_back(&S);
        jobs.push_back(TreeJob{T.x0, T.y0, T.z0, T.S0, (int)segs.size(), 1, D, 1, T.zflip});
        segs.push_back(TreeSeg{tl.data(), (int)tl.size(), 1, 1, c.at, c.bt});
        trees.push_back(&T);
      }
    }
    std::vector<uint64_t> keys, boxes;
    std::vector<uint32_t> pay;
    std::string e = (*sorter)(jobs, segs, keys, pay, boxes);
    if (!e.empty()) return e;
    std::vector<size_t> r0(jobs.size() + 1, 0);
    for (size_t t = 0; t < jobs.size(); t++) {
      size_t nt = 0;
      for (int q = 0; q < jobs[t].nseg; q++) nt += (size_t)segs[jobs[t].seg0 + q].n;
      r0[t + 1] = r0[t] + nt;
    }
    if (keys.size() != r0.back() || pay.size() != r0.back()) return "tree sorter: wrong record count";
    // the sorter's boxes, if it formed them: per tree, the first records of
    // its boxes level by level (entries are in record order)
    std::vector<size_t> e0(jobs.size() + 1, boxes.size());
    if (!boxes.empty()) {
      size_t q = 0;
      for (size_t t = 0; t < jobs.size(); t++) {
        while (q < boxes.size() && (boxes[q] & 0xffffffffffull) < r0[t]) q++;
        e0[t] = q;
      }
      for (size_t q2 = 1; q2 < boxes.size(); q2++)
        if ((boxes[q2] & 0xffffffffffull) < (boxes[q2 - 1] & 0xffffffffffull) ||
            (boxes[q2] >> 40) > (uint64_t)DK)
          return "tree sorter: boxes out of order";
      for (size_t t = 0; t < jobs.size(); t++) tree_starts[trees[t]].assign(DK + 2, {});  // (threads below only fill)
    }
    run_threads(jobs.size(), [&](size_t t) {
      HTree& T = *trees[t];
      T.recs.resize(r0[t + 1] - r0[t]);
      for (size_t i = 0; i < T.recs.size(); i++) {
        const uint32_t v = pay[r0[t] + i];
        T.recs[i].key = keys[r0[t] + i];
        T.recs[i].id = (int)(v & 0x7fffffffu);
        T.recs[i].tag = (int)(v >> 31);
      }
      if (!boxes.empty()) {
        std::vector<std::vector<int>>& st = tree_starts.at(trees[t]);
        for (size_t q = e0[t]; q < e0[t + 1]; q++) st[boxes[q] >> 40].push_back((int)((boxes[q] & 0xffffffffffull) - r0[t]));
      }
    });
  }
  // the boxes of every tree (from the sorter's boxes when it formed them)
  run_threads(geo.size(), [&](size_t gi) {
    Prep& pr = preps[gi];
    if (!pr.err.empty()) return;
    const int D = pr.depth_used;
    auto sit = tree_starts.find(&pr.S);
    if (sit != tree_starts.end()) {
      tree_boxes_from(pr.S, sit->second);
      if (geo[gi].ip.kind != 0) tree_boxes_from(pr.T, tree_starts.at(&pr.T));
    } else if (geo[gi].ip.kind == 0) {
      tree_boxes(pr.S, [&](int l, int n, int, double) { return n > 0 && l < D; });
    } else {
      auto rule = [&](int l, int n, int j, double) { return n > 0 && l < D && j == 0; };
      tree_boxes(pr.S, rule);
      tree_boxes(pr.T, rule);
    }
  });
  // every instance's interaction lists and M2L pair records (local box
  // ids), on host threads: they depend on the instance's own trees alone
  struct ILists {
    std::vector<int> near_t, near_ptr, near_q;  // free space: leaves with targets, their near source boxes
    long long near_pairs = 0;
    std::vector<std::pair<int, std::vector<int>>> s2t_near;  // reaction: target leaf, near source boxes
    std::vector<M2LRec> recs;                                 // M2L pairs (local s, t; gid unset)
    double rref = 0;                                          // worst separation ratio of the pairs
    std::string err;
  };
  std::vector<ILists> ilists(geo.size());
  run_threads(geo.size(), [&](size_t gi) {
    const Prep& pr = preps[gi];
    if (!pr.err.empty()) return;
    ILists& li = ilists[gi];
    const IGeom& g = geo[gi];
    const InstParams& ip = g.ip;
    const double S0 = g.S0;
    const HTree& S = pr.S;
    const HTree& T = pr.T;
    const bool free = ip.kind == 0;
    const HTree& TT = free ? S : T;
    struct Pair {
      int s, t;  // local box ids
    };
    std::vector<Pair> m2l;
    std::vector<std::unordered_map<uint64_t, int>> smap(DK + 2);
    for (int b = 0; b < S.nbox(); b++) smap[S.lvl[b]][ckey(S.ix[b], S.iy[b], S.iz[b])] = b;
    if (free) {
      int D = S.lvl[S.nbox() - 1];
      li.near_ptr.push_back(0);
      for (int t = 0; t < S.nbox(); t++) {
        if (S.b1[t] <= S.b0[t]) continue;  // no targets
        int l = S.lvl[t];
        if (l < 1) continue;
        int px = S.ix[t] >> 1, py = S.iy[t] >> 1, pz = S.iz[t] >> 1;
        for (int dx = -1; dx <= 1; dx++)
          for (int dy = -1; dy <= 1; dy++)
            for (int dz = -1; dz <= 1; dz++) {
              auto it = smap[l - 1].find(ckey(px + dx, py + dy, pz + dz));
              if (it == smap[l - 1].end()) continue;
              int q = it->second;
              for (int c = S.child0[q]; c >= 0 && c < S.child0[q] + S.nchild[q]; c++) {
                if (S.a1[c] <= S.a0[c]) continue;
                int ddx = S.ix[c] - S.ix[t], ddy = S.iy[c] - S.iy[t], ddz = S.iz[c] - S.iz[t];
                if (std::max(std::abs(ddx), std::max(std::abs(ddy), std::abs(ddz))) >= 2)
                  m2l.push_back({c, t});
              }
            }
        if (l == D) {
          li.near_t.push_back(t);
          for (int dx = -1; dx <= 1; dx++)
            for (int dy = -1; dy <= 1; dy++)
              for (int dz = -1; dz <= 1; dz++) {
                auto it = smap[l].find(ckey(S.ix[t] + dx, S.iy[t] + dy, S.iz[t] + dz));
                if (it == smap[l].end()) continue;
                int q = it->second;
                if (S.a1[q] <= S.a0[q]) continue;
                li.near_q.push_back(q);
                li.near_pairs += (long long)(S.a1[q] - S.a0[q]) * (S.b1[t] - S.b0[t]);
              }
          li.near_ptr.push_back((int)li.near_q.size());
        }
      }
    } else {
      std::vector<std::vector<int>> nearT(T.nbox());
      auto ws = [&](int s, int t) {
        double cs[3], ct[3];
        S.centre(s, cs);
        T.centre(t, ct);
        double sl = S.S(S.lvl[s]) * (2.0 - 1e-9);
        return fabs(cs[0] - ct[0]) >= sl || fabs(cs[1] - ct[1]) >= sl || fabs(cs[2] - ct[2]) >= sl;
      };
      if (S.nbox() > 0 && T.nbox() > 0) {
        if (ws(0, 0))
          m2l.push_back({0, 0});
        else
          nearT[0].push_back(0);
      }
      for (int t = 0; t < T.nbox(); t++) {
        int P0 = T.parent[t];
        if (P0 >= 0) {
          for (int q : nearT[P0]) {
            if (S.nchild[q] == 0) {
              li.err = lm_fmt("reaction component (%d,%d): adjacent source leaf at level %d "
                              "(points too close to an interface)",
                              ip.lt, ip.ls, S.lvl[q]);
              return;
            }
            for (int c = S.child0[q]; c < S.child0[q] + S.nchild[q]; c++) {
              if (ws(c, t))
                m2l.push_back({c, t});
              else
                nearT[t].push_back(c);
            }
          }
        }
        if (T.nchild[t] == 0 && !nearT[t].empty()) {
          if (!prm.react_s2t) {
            li.err = lm_fmt("reaction component (%d,%d): adjacent target leaf at level %d "
                            "(points too close to an interface)",
                            ip.lt, ip.ls, T.lvl[t]);
            return;
          }
          li.s2t_near.push_back({t, nearT[t]});
        }
      }
    }
    li.recs.reserve(m2l.size());
    for (auto& pq : m2l) {
      int t = pq.t;
      int l = TT.lvl[t];
      double Sl = S0 / (double)(1 << l);
      M2LRec rec;
      rec.gid = 0;
      rec.l = l;
      rec.px = TT.ix[t] & 1;
      rec.py = TT.iy[t] & 1;
      rec.c3 = free ? (TT.iz[t] & 1) : TT.j(t);
      rec.dx = S.ix[pq.s] - TT.ix[t];
      rec.dy = S.iy[pq.s] - TT.iy[t];
      rec.dz = free ? S.iz[pq.s] - TT.iz[t] : S.j(pq.s);
      rec.s = pq.s;
      rec.t = t;
      double r;
      if (free) {
        r = sqrt(3.0) / sqrt((double)(rec.dx * rec.dx + rec.dy * rec.dy + rec.dz * rec.dz));
      } else {
        const int jt = rec.c3, js = rec.dz;
        double zt_img = ip.sgn > 0 ? T.z0 + (jt + 0.5) * Sl : T.z0 + S0 - (jt + 0.5) * Sl;
        double zs_img = ip.sgn > 0 ? S.z0 + S0 - (js + 0.5) * Sl : S.z0 + (js + 0.5) * Sl;
        double R = sqrt((double)(rec.dx * rec.dx + rec.dy * rec.dy) * Sl * Sl + (zt_img - zs_img) * (zt_img - zs_img));
        r = sqrt(3.0) * Sl / R;
      }
      li.rref = std::max(li.rref, r);
      li.recs.push_back(rec);
    }
  });
  struct BoxFill {
    int gi, inst, sbase, tbase, sp0, tp0, P;
    long long me0, le0;
    std::vector<std::array<long long, 8>> m2m_at, l2l_at;
  };
  std::vector<BoxFill> box_fills;
  {
    size_t ns = 0, nt = 0, np = 0, nq = 0;
    for (const Prep& pr : preps) {
      ns += pr.S.nbox();
      nt += pr.T.nbox();  // (free instances use S: an upper bound)
      np += pr.S.permA.size();
      nq += pr.T.permB.size() + pr.S.permB.size();
    }
    pl.sbox.reserve(ns);
    pl.sbox_m2m.reserve(ns);
    pl.tbox.reserve(nt + ns);
    pl.tbox_l2l.reserve(nt + ns);
    pl.src_perm.reserve(np);
    pl.tgt_perm.reserve(nq);
  }
  for (size_t gi = 0; gi < geo.size(); gi++) {
    const IGeom& g = geo[gi];
    Prep& pr = preps[gi];
    if (!pr.err.empty()) return pr.err;
    const double S0 = g.S0;
    (void)S0;
    InstParams ip = g.ip;
    int inst = (int)pl.inst.size();
    ip.p = ip.kind == 0 ? pl.pf : pl.p;
    ip.P = (ip.p + 1) * (ip.p + 1);
    int P = ip.P;
    HTree& S = pr.S;
    HTree& T = pr.T;
    bool free = ip.kind == 0;
    double Dgap = pr.Dgap;
    int depth_used = pr.depth_used;
    if (free) pl.free_depth_used.push_back(depth_used);
    ip.Dgap = Dgap;
    (void)depth_used;
    HTree& TT = free ? S : T;  // target tree

    // ---- boxes -> global records: ranges, matrices and offsets here, the
    // records themselves on host threads after the loop
    int sbase = (int)pl.sbox.size(), tbase = (int)pl.tbox.size();
    int sp0 = (int)pl.src_perm.size(), tp0 = (int)pl.tgt_perm.size();
    pl.src_perm.resize(sp0 + S.permA.size());  // (filled with the records below)
    pl.tgt_perm.resize(tp0 + TT.permB.size());
    // translation matrices depend on the level and octant alone within an
    // instance: looked up once per (level, octant), in first-use order
    BoxFill bf;
    bf.gi = (int)gi;
    bf.inst = inst;
    bf.sbase = sbase;
    bf.tbase = tbase;
    bf.sp0 = sp0;
    bf.tp0 = tp0;
    bf.me0 = pl.me_size;
    bf.le0 = pl.le_size;
    bf.P = P;
    for (int b = 0; b < S.nbox(); b++)
      if (S.parent[b] >= 0) {
        const int o = S.oct[b], l = S.lvl[b];
        if ((int)bf.m2m_at.size() <= l) bf.m2m_at.resize(l + 1, {-1, -1, -1, -1, -1, -1, -1, -1});
        if (bf.m2m_at[l][o] >= 0) continue;
        double s = S.S(l);
        TransJob j;
        j.b[0] = ((o & 1) - 0.5) * s;
        j.b[1] = (((o >> 1) & 1) - 0.5) * s;
        j.b[2] = (((o >> 2) & 1) - 0.5) * s;
        j.k = ip.ks;
        j.p = ip.p;
        j.kind = 1;
        bf.m2m_at[l][o] = alloc_mat(MatKey{1, kquant(ip.ks), ip.p, kquant(S.S(l)), o, 0, 0}, (long long)P * P, &j);
      }
    for (int b = 0; b < S.nbox(); b++)
      if (S.nchild[b] == 0 && S.a1[b] > S.a0[b]) pl.p2m_leaves.push_back(sbase + b);
    for (int b = 0; b < TT.nbox(); b++)
      if (TT.parent[b] >= 0) {
        const int o = TT.oct[b], l = TT.lvl[b];
        if ((int)bf.l2l_at.size() <= l) bf.l2l_at.resize(l + 1, {-1, -1, -1, -1, -1, -1, -1, -1});
        if (bf.l2l_at[l][o] >= 0) continue;
        double s = TT.S(l);
        TransJob j;
        j.b[0] = ((o & 1) - 0.5) * s;
        j.b[1] = (((o >> 1) & 1) - 0.5) * s;
        j.b[2] = (((o >> 2) & 1) - 0.5) * s;
        j.k = ip.kt;
        j.p = ip.p;
        j.kind = 2;
        bf.l2l_at[l][o] = alloc_mat(MatKey{2, kquant(ip.kt), ip.p, kquant(TT.S(l)), o, 0, 0}, (long long)P * P, &j);
      }
    pl.me_size += 3LL * P * S.nbox();
    pl.le_size += 3LL * P * TT.nbox();
    pl.sbox.resize(sbase + S.nbox());
    pl.sbox_m2m.resize(sbase + S.nbox());
    pl.tbox.resize(tbase + TT.nbox());  // (zero near-box ranges until the lists below set them)
    pl.tbox_l2l.resize(tbase + TT.nbox());
    box_fills.push_back(std::move(bf));
    // M2M parents / L2L children per level
    for (int b = 0; b < S.nbox(); b++)
      if (S.nchild[b] > 0) {
        int l = S.lvl[b];
        if ((int)pl.m2m_parents.size() <= l) pl.m2m_parents.resize(l + 1);
        pl.m2m_parents[l].push_back(sbase + b);
      }
    for (int b = 0; b < TT.nbox(); b++)
      if (TT.parent[b] >= 0) {
        int l = TT.lvl[b];
        if ((int)pl.l2l_children.size() <= l) pl.l2l_children.resize(l + 1);
        pl.l2l_children[l].push_back(tbase + b);
      }
    pl.l2p_leaves.push_back({});
    for (int b = 0; b < TT.nbox(); b++)
      if (TT.nchild[b] == 0 && TT.b1[b] > TT.b0[b]) pl.l2p_leaves.back().push_back(tbase + b);

    // ---- interaction lists (built per instance on host threads above)
    ILists& li = ilists[gi];
    if (!li.err.empty()) return li.err;
    if (free) {
      for (size_t u = 0; u < li.near_t.size(); u++) {
        TgtBox& tb = pl.tbox[tbase + li.near_t[u]];
        tb.p2p0 = (int)pl.p2p_list.size();
        for (int v = li.near_ptr[u]; v < li.near_ptr[u + 1]; v++) pl.p2p_list.push_back(sbase + li.near_q[v]);
        tb.p2p1 = (int)pl.p2p_list.size();
      }
      pl.n_p2p_pairs += li.near_pairs;
      // near-field work items: (target leaf, chunk of LM_P2P_CHUNK targets),
      // so that leaves holding many points spread over many workgroups
      const int D = S.lvl[S.nbox() - 1];
      pl.p2p_tboxes.push_back({});
      for (int t = 0; t < S.nbox(); t++)
        if (S.lvl[t] == D && S.b1[t] > S.b0[t])
          for (int c = 0; c * LM_P2P_CHUNK < S.b1[t] - S.b0[t]; c++) {
            pl.p2p_tboxes.back().push_back(tbase + t);
            pl.p2p_tboxes.back().push_back(c);
          }
    }
    const auto& s2t_near = li.s2t_near;
    // ---- reaction near field (S2T): target leaves next to the gap and their
    // adjacent source boxes, evaluated by direct Sommerfeld integrals
    double s2t_rho = 0;
    if (!free) {
      for (auto& tn : s2t_near) {
        int t = tn.first;
        TgtBox& tb = pl.tbox[tbase + t];
        tb.p2p0 = (int)pl.p2p_list.size();
        double ct[3];
        T.centre(t, ct);
        for (int q : tn.second) {
          pl.p2p_list.push_back(sbase + q);
          pl.n_s2t_pairs += (long long)(S.a1[q] - S.a0[q]) * (T.b1[t] - T.b0[t]);
          double cs[3];
          S.centre(q, cs);
          double rh = hypot(ct[0] - cs[0], ct[1] - cs[1]) + 0.5 * sqrt(2.0) * (T.S(T.lvl[t]) + S.S(S.lvl[q]));
          s2t_rho = std::max(s2t_rho, rh);
        }
        tb.p2p1 = (int)pl.p2p_list.size();
        for (int c = 0; c * LM_S2T_CHUNK < T.b1[t] - T.b0[t]; c++) {
          pl.s2t_items.push_back(tbase + t);
          pl.s2t_items.push_back(c);
        }
      }
    }
    s2t_rho_of.push_back(s2t_near.empty() ? -1.0 : s2t_rho);
    const long long n_m2l = (long long)li.recs.size();
    pl.n_m2l_pairs += n_m2l;
    (free ? pl.n_m2l_pairs_free : pl.n_m2l_pairs_react) += n_m2l;
    (free ? pl.n_free_inst : pl.n_react_inst)++;

    // ---- M2L pairs of this instance, for the classes formed below across
    // instances (computed with the lists; here their global box ids).  The
    // worst separation ratio of the instance's pairs sets its adaptive
    // orders; instances share classes (and tables) when their lattices
    // agree: same kind and component, order, root size, anchors and worst
    // ratio.
    const double rref = li.rref;
    irecs[gi].swap(li.recs);
    irec_base[gi][0] = sbase;
    irec_base[gi][1] = tbase;
    {
      LatKey key;
      key.free = free ? 1 : 0;
      key.lt = ip.lt;
      key.ls = ip.ls;
      key.up_t = ip.up_t;
      key.up_s = ip.up_s;
      key.p = ip.p;
      key.kq = kquant(ip.kt);
      key.s0q = kquant(S0);
      key.tzq = free ? 0 : kquant(T.z0);
      key.szq = free ? 0 : kquant(S.z0);
      key.rq = kquant(rref);
      auto it = latmap.find(key);
      int gid;
      if (it == latmap.end()) {
        gid = (int)lat.size();
        latmap[key] = gid;
        LatGroup lg;
        lg.inst = inst;
        lg.free = free;
        lg.S0 = S0;
        lg.Tz0 = T.z0;
        lg.Sz0 = S.z0;
        lg.rref = rref;
        lat.push_back(lg);
      } else {
        gid = it->second;
      }
      irec_base[gi][2] = gid;
    }
    inst_S0.push_back(S0);
    pl.inst.push_back(ip);
  }
  {
    // the box records of every instance (pieces of up to 2^16 boxes)
    // and their point permutations
    std::vector<std::array<int, 3>> pieces;  // (instance, kind: source / target boxes, source / target points; first)
    const int piece = 1 << 16;
    for (size_t k = 0; k < box_fills.size(); k++) {
      const Prep& pr = preps[box_fills[k].gi];
      const HTree& TT = pl.inst[box_fills[k].inst].kind == 0 ? pr.S : pr.T;
      for (int b = 0; b < pr.S.nbox(); b += piece) pieces.push_back({(int)k, 0, b});
      for (int b = 0; b < TT.nbox(); b += piece) pieces.push_back({(int)k, 1, b});
      for (int b = 0; b < (int)pr.S.permA.size(); b += 4 * piece) pieces.push_back({(int)k, 2, b});
      for (int b = 0; b < (int)TT.permB.size(); b += 4 * piece) pieces.push_back({(int)k, 3, b});
    }
    run_threads(pieces.size(), [&](size_t pi) {
      const BoxFill& bf = box_fills[pieces[pi][0]];
      const Prep& pr = preps[bf.gi];
      const int kind = pieces[pi][1], first = pieces[pi][2];
      if (kind >= 2) {
        const std::vector<int>& v = kind == 2 ? pr.S.permA : (pl.inst[bf.inst].kind == 0 ? pr.S : pr.T).permB;
        int* out = kind == 2 ? pl.src_perm.data() + bf.sp0 : pl.tgt_perm.data() + bf.tp0;
        const int last = std::min((int)v.size(), first + 4 * piece);
        for (int i = first; i < last; i++) out[i] = v[i];
      } else if (kind == 0) {
        const HTree& S = pr.S;
        for (int b = pieces[pi][2]; b < std::min(S.nbox(), pieces[pi][2] + piece); b++) {
          SrcBox sb;
          memset(&sb, 0, sizeof(sb));
          S.centre(b, sb.c);
          sb.pt0 = bf.sp0 + S.a0[b];
          sb.pt1 = bf.sp0 + S.a1[b];
          sb.inst = bf.inst;
          sb.level = S.lvl[b];
          sb.child0 = S.child0[b] >= 0 ? bf.sbase + S.child0[b] : -1;
          sb.nchild = S.nchild[b];
          sb.octant = S.oct[b];
          sb.parent = S.parent[b] >= 0 ? bf.sbase + S.parent[b] : -1;
          sb.me_off = bf.me0 + 3LL * bf.P * b;
          pl.sbox[bf.sbase + b] = sb;
          pl.sbox_m2m[bf.sbase + b] = S.parent[b] >= 0 ? bf.m2m_at[S.lvl[b]][S.oct[b]] : -1;
        }
      } else {
        const HTree& TT = pl.inst[bf.inst].kind == 0 ? pr.S : pr.T;
        for (int b = pieces[pi][2]; b < std::min(TT.nbox(), pieces[pi][2] + piece); b++) {
          TgtBox tb;
          memset(&tb, 0, sizeof(tb));
          TT.centre(b, tb.c);
          tb.pt0 = bf.tp0 + TT.b0[b];
          tb.pt1 = bf.tp0 + TT.b1[b];
          tb.inst = bf.inst;
          tb.level = TT.lvl[b];
          tb.parent = TT.parent[b] >= 0 ? bf.tbase + TT.parent[b] : -1;
          tb.octant = TT.oct[b];
          tb.leaf = TT.nchild[b] == 0;
          tb.le_off = bf.le0 + 3LL * bf.P * b;
          tb.p2p0 = pl.tbox[bf.tbase + b].p2p0;
          tb.p2p1 = pl.tbox[bf.tbase + b].p2p1;
          pl.tbox[bf.tbase + b] = tb;
          pl.tbox_l2l[bf.tbase + b] = TT.parent[b] >= 0 ? bf.l2l_at[TT.lvl[b]][TT.oct[b]] : -1;
        }
      }
    });
  }
  {
    // every instance's pairs in instance order, with global box ids and the
    // lattice group (pieces of up to 2^18 pairs on host threads)
    std::vector<size_t> r0(geo.size() + 1, 0);
    std::vector<std::array<size_t, 2>> pieces;
    const size_t piece = (size_t)1 << 18;
    for (size_t gi = 0; gi < geo.size(); gi++) {
      r0[gi + 1] = r0[gi] + irecs[gi].size();
      for (size_t u = 0; u < irecs[gi].size(); u += piece) pieces.push_back({gi, u});
    }
    recs.resize(r0.back());
    run_threads(pieces.size(), [&](size_t k) {
      const size_t gi = pieces[k][0], u0 = pieces[k][1], u1 = std::min(irecs[gi].size(), u0 + piece);
      const int sb = irec_base[gi][0], tb = irec_base[gi][1], gid = irec_base[gi][2];
      for (size_t u = u0; u < u1; u++) {
        M2LRec r = irecs[gi][u];
        r.s += sb;
        r.t += tb;
        r.gid = gid;
        recs[r0[gi] + u] = r;
      }
    });
    for (auto& ir : irecs) std::vector<M2LRec>().swap(ir);
  }

  // ---- M2L classes, across instances of one lattice group: key (group,
  // level, parity of ix, iy, and iz parity (free) or gap index j (reaction)).
  // A target's pairs, offsets, matrices and orders are those of its own
  // instance alone, so a geometry in a batch computes exactly what its own
  // build computes; the batch only puts more pairs into each GEMM.
  {
    // pairs grouped by class key (group, level, px, py, c3) in key order,
    // each class's pairs in record order
    // The key packs into 64 bits in the same order (group < 2^25, level <
    // 64, parities one bit each, iz parity or gap index j < 2^30), so the
    // distinct keys of pieces of the list (host threads) are merged by one
    // sort, and each pair's class is its key's rank.
    std::vector<std::tuple<int, int, int, int, int>> ckeys;  // distinct keys, increasing
    std::vector<int> rec_cls(recs.size());                   // each pair's class
    {
      auto pack = [](const M2LRec& r) {
        return ((uint64_t)(uint32_t)r.gid << 38) | ((uint64_t)(uint32_t)r.l << 32) |
               ((uint64_t)(uint32_t)r.px << 31) | ((uint64_t)(uint32_t)r.py << 30) | (uint64_t)(uint32_t)r.c3;
      };
      const size_t piece = (size_t)1 << 18, npc = (recs.size() + piece - 1) / piece;
      std::vector<std::vector<uint64_t>> pkeys(npc);
      std::atomic<bool> bad{false};
      run_threads(npc, [&](size_t k) {
        std::unordered_set<uint64_t> seen;
        for (size_t q = k * piece; q < std::min(recs.size(), (k + 1) * piece); q++) {
          const M2LRec& r = recs[q];
          if (r.gid < 0 || r.gid >= (1 << 25) || r.l < 0 || r.l >= 64 || (r.px | r.py) & ~1 || r.c3 < 0 ||
              r.c3 >= (1 << 30))
            bad = true;
          seen.insert(pack(r));
        }
        pkeys[k].assign(seen.begin(), seen.end());
      });
      if (bad) return "internal: M2L class key out of range";
      std::vector<uint64_t> keys;
      for (const auto& v : pkeys) keys.insert(keys.end(), v.begin(), v.end());
      std::sort(keys.begin(), keys.end());
      keys.erase(std::unique(keys.begin(), keys.end()), keys.end());
      std::unordered_map<uint64_t, int> rank;
      for (size_t c = 0; c < keys.size(); c++) {
        const uint64_t u = keys[c];
        rank[u] = (int)c;
        ckeys.push_back(std::make_tuple((int)(u >> 38), (int)((u >> 32) & 63), (int)((u >> 31) & 1),
                                        (int)((u >> 30) & 1), (int)(u & ((1u << 30) - 1))));
      }
      run_threads(npc, [&](size_t k) {
        for (size_t q = k * piece; q < std::min(recs.size(), (k + 1) * piece); q++) rec_cls[q] = rank.at(pack(recs[q]));
      });
    }
    std::vector<int> cptr(ckeys.size() + 1, 0), cpairs(recs.size());
    for (size_t q = 0; q < recs.size(); q++) cptr[rec_cls[q] + 1]++;
    for (size_t c = 0; c < ckeys.size(); c++) cptr[c + 1] += cptr[c];
    {
      std::vector<int> fillp(cptr.begin(), cptr.end() - 1);
      for (size_t q = 0; q < recs.size(); q++) cpairs[fillp[rec_cls[q]]++] = (int)q;
    }
    // Per class, on host threads: the offsets on a dense grid over their
    // range (occupied cells read in (dx, dy, dz) order) and the targets in
    // order of first appearance.  A target box lies in one class only (the
    // key is made of its own lattice group, level, parities and z index), so
    // the classes write disjoint entries of tslot_of.
    std::vector<int> tslot_of(pl.tbox.size(), -1);  // target box -> slot in its class
    struct ClsPre {
      int lo[3];
      long long ey, ez;
      std::vector<int> offgrid, tlist;
      std::vector<std::tuple<int, int, int>> okeys;
    };
    std::vector<ClsPre> pre(ckeys.size());
    run_threads(ckeys.size(), [&](size_t ci) {
      ClsPre& cp = pre[ci];
      const bool free = lat[std::get<0>(ckeys[ci])].free;
      const int* prs = cpairs.data() + cptr[ci];
      const int nprs = cptr[ci + 1] - cptr[ci];
      int lo[3] = {INT_MAX, INT_MAX, INT_MAX}, hi[3] = {INT_MIN, INT_MIN, INT_MIN};
      for (int u = 0; u < nprs; u++) {
        const M2LRec& r = recs[prs[u]];
        const int v[3] = {r.dx, r.dy, r.dz};
        for (int a = 0; a < 3; a++) {
          lo[a] = std::min(lo[a], v[a]);
          hi[a] = std::max(hi[a], v[a]);
        }
      }
      const long long ex = hi[0] - lo[0] + 1, ey = hi[1] - lo[1] + 1, ez = hi[2] - lo[2] + 1;
      for (int a = 0; a < 3; a++) cp.lo[a] = lo[a];
      cp.ey = ey;
      cp.ez = ez;
      cp.offgrid.assign((size_t)(ex * ey * ez), -1);
      for (int u = 0; u < nprs; u++) {
        const M2LRec& r = recs[prs[u]];
        cp.offgrid[((r.dx - lo[0]) * ey + (r.dy - lo[1])) * ez + (r.dz - lo[2])] = 0;
        if (tslot_of[r.t] < 0) {
          tslot_of[r.t] = (int)cp.tlist.size();
          cp.tlist.push_back(r.t);
        }
      }
      for (long long x = 0; x < ex; x++)
        for (long long y = 0; y < ey; y++)
          for (long long z = 0; z < ez; z++)
            if (cp.offgrid[(x * ey + y) * ez + z] == 0)
              cp.okeys.push_back(std::make_tuple((int)x + lo[0], (int)y + lo[1], (int)z + lo[2]));
      // offset order: reaction offsets with equal horizontal distance and
      // source gap index share one table case (they differ only in the
      // azimuth, which the M2L applies per column), so they are placed next
      // to each other and their pairs form the columns of one GEMM
      if (!free)
        std::stable_sort(cp.okeys.begin(), cp.okeys.end(),
                         [](const std::tuple<int, int, int>& a, const std::tuple<int, int, int>& b) {
                           const int ra = std::get<0>(a) * std::get<0>(a) + std::get<1>(a) * std::get<1>(a);
                           const int rb = std::get<0>(b) * std::get<0>(b) + std::get<1>(b) * std::get<1>(b);
                           return ra != rb ? ra < rb : std::get<2>(a) < std::get<2>(b);
                         });
    });
    {
      std::vector<int> owner(pl.tbox.size(), -1);
      for (size_t ci = 0; ci < pre.size(); ci++)
        for (size_t k = 0; k < pre[ci].tlist.size(); k++) {
          const int t = pre[ci].tlist[k];
          if (owner[t] >= 0 || tslot_of[t] != (int)k) return "internal: target box in two M2L classes";
          owner[t] = (int)ci;
        }
    }
    // offsets, table cases and matrices in class order (serial), then each
    // class's (target, offset) -> source box table on host threads
    std::vector<std::vector<int>> group_offs(lat.size());
    long long srcof_n = 0;
    for (size_t ci = 0; ci < ckeys.size(); ci++) {
      const auto& ckey = ckeys[ci];
      const int gid = std::get<0>(ckey);
      const LatGroup& lg = lat[gid];
      const InstParams& ip = pl.inst[lg.inst];
      const bool free = lg.free;
      const int inst = lg.inst;
      const int P = ip.P;
      const double S0 = lg.S0;
      int l = std::get<1>(ckey);
      double Sl = S0 / (double)(1 << l);
      ClsPre& cp = pre[ci];
      const int* lo = cp.lo;
      const long long ey = cp.ey, ez = cp.ez;
      std::vector<int>& offgrid = cp.offgrid;
      const std::vector<int>& tlist = cp.tlist;
      const std::vector<std::tuple<int, int, int>>& okeys = cp.okeys;
      M2LClass C;
      C.inst = inst;
      C.n_off = (int)okeys.size();
      C.off0 = (int)pl.offs.size();
      C.n_tgt = (int)tlist.size();
      C.tgt0 = (int)pl.cls_tgt.size();
      C.nblk = free ? 1 : 3;
      C.P = P;
      int oi = 0;
      int jt = std::get<4>(ckey);
      for (const auto& okey : okeys) {
        int dx = std::get<0>(okey), dy = std::get<1>(okey), dz = std::get<2>(okey);
        offgrid[((long long)(dx - lo[0]) * ey + (dy - lo[1])) * ez + (dz - lo[2])] = oi++;
        M2LOffset mo;
        group_offs[gid].push_back((int)pl.offs.size());
        if (free) {
          TransJob j;
          j.b[0] = -dx * Sl;
          j.b[1] = -dy * Sl;
          j.b[2] = -dz * Sl;
          j.k = ip.kt;
          j.p = ip.p;
          j.kind = 0;
          long long m = alloc_mat(MatKey{0, kquant(ip.kt), ip.p, kquant(Sl), dx, dy, dz}, (long long)P * P, &j);
          mo.mat[0] = mo.mat[1] = mo.mat[2] = m;
          mo.phi = 0;
          off_ratio.push_back(sqrt(3.0) / sqrt((double)(dx * dx + dy * dy + dz * dz)));
        } else {
          int js = dz;
          int r2 = dx * dx + dy * dy;
          double zt_img = ip.sgn > 0 ? lg.Tz0 + (jt + 0.5) * Sl : lg.Tz0 + S0 - (jt + 0.5) * Sl;
          double zs_img = ip.sgn > 0 ? lg.Sz0 + S0 - (js + 0.5) * Sl : lg.Sz0 + (js + 0.5) * Sl;
          auto ck = std::make_tuple(gid, l, (long long)r2, (long long)jt, (long long)js);
          int cid;
          auto it = casemap.find(ck);
          if (it == casemap.end()) {
            cid = (int)pl.cases.size();
            casemap[ck] = cid;
            TabCase tc;
            memset(&tc, 0, sizeof(tc));
            tc.inst = inst;
            tc.rho = sqrt((double)r2) * Sl;
            // centres: target box with gap index jt, source box with gap index js
            tc.zt_orig = ip.at * (zt_img - ip.bt);
            tc.zs_orig = ip.as * (zs_img - ip.bs);
            tc.node0 = l;  // temporarily the level
            tc.nnode = 0;
            // the even and the odd block of the mirror-adapted M2L tensor
            tc.mat = pl.mat_size;
            pl.mat_size += (long long)lm_sym_dim(ip.p, 0) * lm_sym_dim(ip.p, 0) +
                           (long long)lm_sym_dim(ip.p, 1) * lm_sym_dim(ip.p, 1);
            pl.cases.push_back(tc);
          } else
            cid = it->second;
          long long base = pl.cases[cid].mat;
          double R = sqrt((double)(dx * dx + dy * dy) * Sl * Sl + (zt_img - zs_img) * (zt_img - zs_img));
          off_ratio.push_back(sqrt(3.0) * Sl / R);
          mo.mat[0] = base;                                                  // even block
          mo.mat[1] = base + (long long)lm_sym_dim(ip.p, 0) * lm_sym_dim(ip.p, 0);  // odd block
          mo.mat[2] = base;                                                  // (unused)
          mo.phi = atan2(-(double)dy, -(double)dx);
        }
        mo.pord = ip.p;
        mo.pad_ = 0;
        pl.offs.push_back(mo);
      }
      pl.cls_srcof0.push_back(srcof_n);
      srcof_n += (long long)C.n_tgt * C.n_off;
      pl.cls_tgt.insert(pl.cls_tgt.end(), tlist.begin(), tlist.end());
      pl.cls.push_back(C);
    }
    pl.cls_srcof.assign((size_t)srcof_n, -1);
    run_threads(ckeys.size(), [&](size_t ci) {
      const ClsPre& cp = pre[ci];
      const int n_off = pl.cls[ci].n_off;
      int* so = pl.cls_srcof.data() + pl.cls_srcof0[ci];
      for (int u = cptr[ci]; u < cptr[ci + 1]; u++) {
        const M2LRec& r = recs[cpairs[u]];
        const int o = cp.offgrid[((r.dx - cp.lo[0]) * cp.ey + (r.dy - cp.lo[1])) * cp.ez + (r.dz - cp.lo[2])];
        so[(size_t)tslot_of[r.t] * n_off + o] = r.s;
      }
    });
    // per-offset orders: the truncation error of an M2L pair behaves like
    // rho^(p+1).  Every offset gets the least order whose bound lies
    // m2l_margin decades below the bound of the group's worst admissible
    // pair at order p (the margin accounts for the many better-separated
    // pairs that would otherwise all contribute the worst pair's error).
    if (prm.m2l_adapt)
      for (size_t gid = 0; gid < lat.size(); gid++) {
        const double rr = lat[gid].rref;
        const int p = pl.inst[lat[gid].inst].p;
        double target = (p + 1) * log(rr) - prm.m2l_margin * log(10.0);
        for (int o : group_offs[gid]) {
          double r = off_ratio[o];
          int q = p;
          if (r < rr && rr < 1.0) q = (int)ceil(target / log(r)) - 1;
          pl.offs[o].pord = std::min(p, std::max(2, q));
        }
      }
  }

  // ---- M2L work blocks: targets of a class in groups of at most 2048, pairs
  // sorted by offset (GEMM columns) and per target (reduction).  The blocks'
  // sizes are counted first, then every block fills its own ranges of the
  // pair and target arrays (host threads; the arrays are those of one pass
  // over the blocks in class order).
  {
    const int TB = 512;
    struct BJob {
      int c, t0, t1;
      long long nq, q0, offr0, bt0;
    };
    std::vector<BJob> jobs;
    for (int c = 0; c < (int)pl.cls.size(); c++)
      for (int t0 = 0; t0 < pl.cls[c].n_tgt; t0 += TB) jobs.push_back({c, t0, std::min(pl.cls[c].n_tgt, t0 + TB), 0, 0, 0, 0});
    run_threads(jobs.size(), [&](size_t j) {
      BJob& b = jobs[j];
      const M2LClass& C = pl.cls[b.c];
      const int* so = pl.cls_srcof.data() + pl.cls_srcof0[b.c];
      long long n = 0;
      for (long long e = (long long)b.t0 * C.n_off; e < (long long)b.t1 * C.n_off; e++) n += so[e] >= 0;
      b.nq = n;
    });
    long long nq = 0, noffr = 0, nbt = 0;
    for (BJob& b : jobs) {
      b.q0 = nq;
      b.offr0 = noffr;
      b.bt0 = nbt;
      nq += b.nq;
      noffr += pl.cls[b.c].n_off + 1;
      nbt += b.t1 - b.t0;
    }
    if (nq > INT_MAX || noffr > INT_MAX || nbt > INT_MAX) return "too many M2L pairs";
    pl.offr.resize(noffr);
    pl.pair_src.resize(nq);
    pl.pair_P.resize(nq);
    pl.pair_phi.resize(nq);
    pl.bt_pairs.resize(nq);
    pl.bt_tbox.resize(nbt);
    pl.bt_blk.resize(nbt);
    pl.bt_ptr.resize(nbt + 1);
    pl.blocks.resize(jobs.size());
    run_threads(jobs.size(), [&](size_t j) {
      const BJob& b = jobs[j];
      const M2LClass& C = pl.cls[b.c];
      const long long base = pl.cls_srcof0[b.c];
      M2LBlock B;
      B.cls = b.c;
      B.nt = b.t1 - b.t0;
      B.bt0 = (int)b.bt0;
      B.q0 = (int)b.q0;
      B.offr0 = (int)b.offr0;
      B.nq = (int)b.nq;
      // pair index of (target slot, offset) inside the block
      std::vector<int> qidx((size_t)B.nt * C.n_off, -1);
      int q = B.q0, r = B.offr0;
      for (int o = 0; o < C.n_off; o++) {
        pl.offr[r++] = q;
        const int po = pl.offs[C.off0 + o].pord;
        const double phi = pl.offs[C.off0 + o].phi;
        for (int t = b.t0; t < b.t1; t++) {
          const int sb = pl.cls_srcof[base + (long long)t * C.n_off + o];
          if (sb < 0) continue;
          qidx[(size_t)(t - b.t0) * C.n_off + o] = q;
          pl.pair_src[q] = sb;
          pl.pair_P[q] = (po + 1) * (po + 1);
          pl.pair_phi[q] = phi;
          q++;
        }
      }
      pl.offr[r] = q;
      int bt = B.bt0, bp = B.q0;
      for (int t = b.t0; t < b.t1; t++, bt++) {
        pl.bt_tbox[bt] = pl.cls_tgt[C.tgt0 + t];
        pl.bt_blk[bt] = (int)j;
        pl.bt_ptr[bt] = bp;
        for (int o = 0; o < C.n_off; o++) {
          const int qq = qidx[(size_t)(t - b.t0) * C.n_off + o];
          if (qq >= 0) pl.bt_pairs[bp++] = qq;
        }
      }
      pl.blocks[j] = B;
    });
    pl.bt_ptr[nbt] = (int)nq;
  }

  // ---- quadrature node sets: one per (reaction instance, level)
  {
    double a = prm.contour_a > 0 ? prm.contour_a : 1.5 * med.kmax;
    double kg = med.kmax;
    if (!(a > kg)) return "contour end point must exceed the largest wavenumber";
    // per (lattice group, level): the largest horizontal distance and the
    // smallest vertical centre separation an interaction-list pair of the
    // level can have (offsets up to 3 boxes in x and y; both boxes next to
    // the gap), so that the node set depends on the lattice alone
    std::map<std::pair<int, int>, std::pair<double, double>> lvinfo;  // rho_max, dz_min
    for (size_t ci = 0; ci < pl.cases.size(); ci++) {
      auto& tc = pl.cases[ci];
      const double Sl = inst_S0[tc.inst] / (double)(1 << tc.node0);
      lvinfo[std::make_pair(tc.inst, tc.node0)] = std::make_pair(3.0 * sqrt(2.0) * Sl, pl.inst[tc.inst].Dgap + Sl);
    }
    std::map<std::pair<int, int>, std::pair<int, int>> nodemap;
    std::vector<double> gx, gw;
    gauss_legendre(16, gx, gw);
    double w_im = sqrt(a * a - kg * kg);
    for (auto& kv : lvinfo) {
      int inst = kv.first.first;
      double rho_max = kv.second.first, dzmin = kv.second.second;
      int n0 = (int)pl.node_kr.size();
      // Gamma_1: k'_z runs on a straight line from kg to i*sqrt(a^2-kg^2)
      int np1 = std::max(1, prm.gamma1_panels);
      for (int pnl = 0; pnl < np1; pnl++) {
        double t0 = (double)pnl / np1, t1 = (double)(pnl + 1) / np1;
        for (int gi = 0; gi < 16; gi++) {
          double t = 0.5 * (t0 + t1) + 0.5 * (t1 - t0) * gx[gi];
          cd kzg = cd{kg * (1 - t), w_im * t};
          cd kr = csqrtd(cd{kg * kg, 0} - kzg * kzg);
          cd dkzg = cd{-kg, w_im};
          cd dkr = (-1.0) * (kzg * dkzg) / kr;
          pl.node_kr.push_back(kr);
          pl.node_w.push_back(0.5 * (t1 - t0) * gw[gi] * dkr);
          pl.node_inst.push_back(inst);
        }
      }
      // real tail [a, kcut]
      int pp = pl.inst[inst].p;
      double kcut = a + (3.0 * pp + prm.tail_digits) / dzmin;
      // 16-point Gauss-Legendre panels spanning two periods of J(k rho_max)
      // (error below 3e-16 of the panel's largest integrand value while the
      // decay over half a panel, len h / 2, stays below about 7)
      double len = std::min(4.0 / dzmin, rho_max > 0 ? 4.0 * M_PI / rho_max : 1e300);
      int npan = (int)ceil((kcut - a) / len);
      len = (kcut - a) / npan;
      for (int pnl = 0; pnl < npan; pnl++) {
        double k0 = a + pnl * len;
        for (int gi = 0; gi < 16; gi++) {
          pl.node_kr.push_back(cd{k0 + 0.5 * len * (gx[gi] + 1.0), 0.0});
          pl.node_w.push_back(cd{0.5 * len * gw[gi], 0.0});
          pl.node_inst.push_back(inst);
        }
      }
      nodemap[kv.first] = std::make_pair(n0, (int)pl.node_kr.size() - n0);
    }
    // direct near field (S2T) of a reaction component: Gamma_1 and the real
    // tail up to a + s2t_digits / gap (every pair's vertical transmission
    // distance is at least the gap; each pair stops at its own cut)
    if (s2t_rho_of.size() != pl.inst.size()) return "internal: near-field bookkeeping out of step";
    for (size_t inst = 0; inst < pl.inst.size(); inst++) {
      InstParams& ipr = pl.inst[inst];
      ipr.s2t0 = ipr.s2tn = 0;
      ipr.s2t_rho = s2t_rho_of[inst];
      if (ipr.kind != 1 || s2t_rho_of[inst] < 0) continue;
      double dzmin = ipr.Dgap, rho_max = s2t_rho_of[inst];
      int n0 = (int)pl.node_kr.size();
      // within the series range (|k_rho| rho <= 7.5 on Gamma_1) two panels
      // integrate the direct pairs to within about 2e-9 of the field; the
      // tables (larger rho at coarse levels) keep the full panel count
      int np1 = std::max(1, prm.gamma1_panels);
      if (a * rho_max <= 7.5) np1 = std::min(np1, 2);
      for (int pnl = 0; pnl < np1; pnl++) {
        double t0 = (double)pnl / np1, t1 = (double)(pnl + 1) / np1;
        for (int gi = 0; gi < 16; gi++) {
          double t = 0.5 * (t0 + t1) + 0.5 * (t1 - t0) * gx[gi];
          cd kzg = cd{kg * (1 - t), w_im * t};
          cd kr = csqrtd(cd{kg * kg, 0} - kzg * kzg);
          cd dkzg = cd{-kg, w_im};
          cd dkr = (-1.0) * (kzg * dkzg) / kr;
          pl.node_kr.push_back(kr);
          pl.node_w.push_back(0.5 * (t1 - t0) * gw[gi] * dkr);
          pl.node_inst.push_back((int)inst);
        }
      }
      double kcut = a + LM_S2T_DIGITS / dzmin;
      // 16-point Gauss-Legendre panels spanning two periods of J(k rho_max)
      // (error below 3e-16 of the panel's largest integrand value while the
      // decay over half a panel, len h / 2, stays below about 7)
      double len = std::min(4.0 / dzmin, rho_max > 0 ? 4.0 * M_PI / rho_max : 1e300);
      int npan = (int)ceil((kcut - a) / len);
      len = (kcut - a) / npan;
      for (int pnl = 0; pnl < npan; pnl++) {
        double k0 = a + pnl * len;
        for (int gi = 0; gi < 16; gi++) {
          pl.node_kr.push_back(cd{k0 + 0.5 * len * (gx[gi] + 1.0), 0.0});
          pl.node_w.push_back(cd{0.5 * len * gw[gi], 0.0});
          pl.node_inst.push_back((int)inst);
        }
      }
      ipr.s2t0 = n0;
      ipr.s2tn = (int)pl.node_kr.size() - n0;
    }
    int NQ = 2 * pl.p + 3, NL = pl.p + 2;
    for (auto& tc : pl.cases) {
      auto nm = nodemap[std::make_pair(tc.inst, tc.node0)];
      tc.node0 = nm.first;
      tc.nnode = nm.second;
      tc.ibuf = pl.ibuf_size;
      pl.ibuf_size += 5LL * 16 * NL * NQ;
    }
  }

  // ---- the requested accuracy against the quadrature rules of the plan
  if (prm.tol > 0) {
    if (!pl.cases.empty() && std::exp(-prm.tail_digits) > prm.tol)
      return lm_fmt(LM_PLAN_ACCURACY_PREFIX "the real tail of the M2L tables' Sommerfeld integrals is cut at "
                    "e^-%.1f (tail_digits) beyond the Legendre products' growth, coarser than tol = %.1e",
                    prm.tail_digits, prm.tol);
    if (!pl.cases.empty() && prm.gamma1_panels < 3 && prm.tol < 1e-8)
      return lm_fmt(LM_PLAN_ACCURACY_PREFIX "%d Gauss-Legendre panels on the first contour piece give about "
                    "2e-9 of the M2L tables, coarser than tol = %.1e (use 3 or more)",
                    prm.gamma1_panels, prm.tol);
    if (pl.n_s2t_pairs > 0 && prm.tol < 2.5e-9)
      return lm_fmt(LM_PLAN_ACCURACY_PREFIX "the direct reaction pairs' integrals are cut at %.0f e-folds on "
                    "the real tail with two panels on the first contour piece (about 2.5e-9 of a pair's field), "
                    "coarser than tol = %.1e (react_s2t = 0 refines the trees instead)",
                    (double)LM_S2T_DIGITS, prm.tol);
  }

  // ---- coefficient tables
  lm_legendre_cheb(pmax, pl.Bcoef);
  for (auto& ip : pl.inst) {
    pl.Ccoef0.push_back((long long)pl.Ccoef.size());
    if (ip.kind != 1) continue;
    double ksm = std::min(ip.kt, ip.ks), klg = std::max(ip.kt, ip.ks);
    double aa = (ksm / klg) * (ksm / klg);
    std::vector<double> C;
    lm_cheb_affine(KB + 1, aa, 1.0 - aa, C);
    pl.Ccoef.insert(pl.Ccoef.end(), C.begin(), C.end());
  }
  bool need_gaunt = !pl.trans.empty();
  if (need_gaunt) {
    // the Gaunt table depends only on the order: computed once per process
    static std::mutex mu;
    static std::map<int, std::vector<double>> cache;
    std::lock_guard<std::mutex> lock(mu);
    auto it = cache.find(pmax);
    if (it == cache.end()) {
      std::vector<double> G;
      lm_gaunt_table(pmax, G);
      it = cache.emplace(pmax, std::move(G)).first;
    }
    pl.gaunt = it->second;
    pl.gaunt_p = pmax;
  }
  return "";
}
