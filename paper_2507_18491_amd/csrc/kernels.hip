// kernels.hip -- gfx950 kernels of the layered-media dyadic FMM (fp64).
//
// Passes (paper Sec. 2 and Sec. 3.3): P2M, M2M, M2L, L2L, L2P for the
// free-space part of every layer and for every reaction component, the
// free-space near field P2P, and the table builders: free-space translation
// matrices (addition theorem through Gaunt coefficients), Sommerfeld
// quadrature densities of the reaction components, the Chebyshev-weighted
// Sommerfeld integrals (Sec. 3.4) and their assembly into M2L matrices.
//
// Coefficient vectors are stored per box as [rhs][channel][(p+1)^2], with
// channels in the spin basis (x + i y, x - i y, z).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <mutex>
#include <vector>

#include "bessel_pq.h"
#include "kernels.h"

// Raises a kernel's dynamic LDS limit before its launch.  A failure leaves
// the default limit in place; the launch that follows then fails, and the
// caller's hipGetLastError check reports it (as it reports this call's
// error, which HIP keeps as the last error).
static inline void set_dyn_lds(const void* f, size_t bytes) {
  (void)hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

// RC (template parameter): right-hand sides per block in the point/translation passes (1 or 4)
#define NT 256          // threads per block
static_assert(NT == LM_P2P_CHUNK, "near-field work items hold one block's worth of targets");

// Coefficients of the orthonormal associated Legendre recurrences (uploaded
// once per device): P^m_m = LEG_MM[m] sin P^{m-1}_{m-1}, P^m_{m+1} =
// LEG_M1[m] cos P^m_m, P^m_n = LEG_A[n][m] (cos P^m_{n-1} - LEG_B[n][m] P^m_{n-2}).
#define LEGN (LM_PMAX + 5)
__constant__ double c_leg_a[LEGN * LEGN], c_leg_b[LEGN * LEGN], c_leg_mm[LEGN], c_leg_m1[LEGN];
// 1/k, 1/k^2, 1/(k(k+1)), 1/(k(k+2)) for the Bessel series (index k, 1..64)
#define RCPN 65
__constant__ double c_rk[RCPN], c_rk2[RCPN], c_rkk1[RCPN], c_rkk2[RCPN];

int lm_upload_leg_tables() {
  static bool done[64] = {false};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return -1;
  if (done[dev]) return 0;
  std::vector<double> a(LEGN * LEGN, 0.0), b(LEGN * LEGN, 0.0), mm(LEGN, 0.0), m1(LEGN, 0.0);
  for (int m = 0; m < LEGN; m++) {
    mm[m] = m > 0 ? -std::sqrt((2.0 * m + 1.0) / (2.0 * m)) : 0.0;
    m1[m] = std::sqrt(2.0 * m + 3.0);
    for (int n = m + 2; n < LEGN; n++) {
      a[n * LEGN + m] = std::sqrt((4.0 * n * n - 1.0) / ((double)n * n - (double)m * m));
      b[n * LEGN + m] = std::sqrt(((n - 1.0) * (n - 1.0) - (double)m * m) / (4.0 * (n - 1.0) * (n - 1.0) - 1.0));
    }
  }
  if (hipMemcpyToSymbol(HIP_SYMBOL(c_leg_a), a.data(), a.size() * sizeof(double)) != hipSuccess ||
      hipMemcpyToSymbol(HIP_SYMBOL(c_leg_b), b.data(), b.size() * sizeof(double)) != hipSuccess ||
      hipMemcpyToSymbol(HIP_SYMBOL(c_leg_mm), mm.data(), mm.size() * sizeof(double)) != hipSuccess ||
      hipMemcpyToSymbol(HIP_SYMBOL(c_leg_m1), m1.data(), m1.size() * sizeof(double)) != hipSuccess)
    return -1;
  std::vector<double> rk(RCPN, 0.0), rk2(RCPN, 0.0), rkk1(RCPN, 0.0), rkk2(RCPN, 0.0);
  for (int k = 1; k < RCPN; k++) {
    rk[k] = 1.0 / k;
    rk2[k] = 1.0 / ((double)k * k);
    rkk1[k] = 1.0 / ((double)k * (k + 1));
    rkk2[k] = 1.0 / ((double)k * (k + 2));
  }
  if (hipMemcpyToSymbol(HIP_SYMBOL(c_rk), rk.data(), rk.size() * sizeof(double)) != hipSuccess ||
      hipMemcpyToSymbol(HIP_SYMBOL(c_rk2), rk2.data(), rk2.size() * sizeof(double)) != hipSuccess ||
      hipMemcpyToSymbol(HIP_SYMBOL(c_rkk1), rkk1.data(), rkk1.size() * sizeof(double)) != hipSuccess ||
      hipMemcpyToSymbol(HIP_SYMBOL(c_rkk2), rkk2.data(), rkk2.size() * sizeof(double)) != hipSuccess)
    return -1;
  done[dev] = true;
  return 0;
}

// orthonormal P^m_n(cos t), 0 <= m <= n <= nmax, triangular layout tri_idx(n, m)
__device__ inline void legendre_rt(int nmax, double c, double s, double* out) {
  out[0] = LM_INV_SQRT_4PI;
  for (int m = 1; m <= nmax; m++) out[tri_idx(m, m)] = c_leg_mm[m] * s * out[tri_idx(m - 1, m - 1)];
  for (int m = 0; m <= nmax; m++) {
    if (m + 1 <= nmax) out[tri_idx(m + 1, m)] = c_leg_m1[m] * c * out[tri_idx(m, m)];
    for (int n = m + 2; n <= nmax; n++)
      out[tri_idx(n, m)] =
          c_leg_a[n * LEGN + m] * (c * out[tri_idx(n - 1, m)] - c_leg_b[n * LEGN + m] * out[tri_idx(n - 2, m)]);
  }
}

__device__ inline int n_of(int nm) {
  int n = (int)sqrt((double)nm);
  while (n * n > nm) n--;
  while ((n + 1) * (n + 1) <= nm) n++;
  return n;
}

// Complex products with explicit multiply-adds: the compiler would otherwise
// keep a multiply and an add beside each fused one, and may fuse either real
// product of a complex product -- differently in two instantiations of one
// loop (results that must agree bitwise across the kernels' right-hand-side
// variants use these).
__device__ inline cd cmul_exact(cd a, cd b) {
  return cd{fma(a.x, b.x, -(a.y * b.y)), fma(a.x, b.y, a.y * b.x)};
}
// acc + a b
__device__ inline cd cmac_exact(cd acc, cd a, cd b) {
  return cd{fma(a.x, b.x, fma(-a.y, b.y, acc.x)), fma(a.x, b.y, fma(a.y, b.x, acc.y))};
}

// ------------------------------------------------------------------ fill
__global__ void k_fill(cd* p, long long n) {
  long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  long long st = (long long)gridDim.x * blockDim.x;
  for (; i < n; i += st) p[i] = cd{0.0, 0.0};
}
void launch_fill(cd* p, long long n, hipStream_t s) {
  if (n <= 0) return;
  long long nb = (n + NT - 1) / NT;
  if (nb > 65536) nb = 65536;
  hipLaunchKernelGGL(k_fill, dim3((unsigned)nb), dim3(NT), 0, s, p, n);
}

// ------------------------------------------------------------------ work queues
// Persistent launches of the passes whose work items differ widely in cost
// (near field, direct reaction pairs): as many blocks as the device keeps
// resident, each taking the next item index from a counter in device memory
// until the items run out (items are stored longest first, so the queue
// hands out the long ones first, across every geometry and component of the
// plan).  q[0] hands out indices, q[1] counts the blocks that have left; the
// last block to leave sets both back to zero for the next launch on the
// stream.  The counters start at zero (cleared when the plan is built).
// Launches that share a queue must not overlap in time (they run in stream
// order).  Every item writes outputs of its own, so the order in which the
// blocks take them does not change any result.
struct WorkQueue {
  int* q;  // the counter pair
  int* s;  // an LDS slot of the block
  // the block's next index, once every thread is done with the previous
  // item (taking it ahead, while an item runs, measured slower)
  __device__ int next() {
    __syncthreads();
    if (threadIdx.x == 0) *s = atomicAdd(q, 1);
    __syncthreads();
    return *s;
  }
  __device__ void leave() {
    if (threadIdx.x == 0 && atomicAdd(q + 1, 1) == (int)(gridDim.x * gridDim.y * gridDim.z) - 1) {
      atomicExch(q, 0);
      atomicExch(q + 1, 0);
    }
  }
};
// Blocks of a persistent launch: the kernel's resident blocks per compute
// unit times the compute units, at most `work`.  Cached per (device,
// kernel) in a fixed table (nothing allocated).
static int persistent_grid(const void* f, int nthreads, size_t shm, long long work) {
  struct Ent {
    int dev;
    const void* f;
    int nthreads;
    int blocks;
  };
  static Ent cache[64];
  static int n_cache = 0;
  static std::mutex mu;
  int dev = 0;
  (void)hipGetDevice(&dev);
  int blocks = 0;
  {
    std::lock_guard<std::mutex> lk(mu);
    for (int i = 0; i < n_cache; i++)
      if (cache[i].dev == dev && cache[i].f == f && cache[i].nthreads == nthreads) blocks = cache[i].blocks;
  }
  if (blocks <= 0) {
    int ncu = 0, per = 0;
    if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || ncu <= 0) ncu = 256;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, f, nthreads, shm) != hipSuccess || per <= 0) per = 1;
    blocks = ncu * per;
    std::lock_guard<std::mutex> lk(mu);
    if (n_cache < 64) cache[n_cache++] = Ent{dev, f, nthreads, blocks};
  }
  return (int)std::min<long long>(blocks, work);
}

// ------------------------------------------------------------------ P2M
// M[r][ch][nm] = sum_j q_j^ch j_n(k |d_j|) conj(Y^m_n(d_j)),  d_j = image(x_j) - centre
// (paper Sec. 2, the multipole coefficients, and Sec. 3.3, the reaction ME
// coefficients; the constant 4 pi lives in the M2L tables).
// Work item (leaf, chunk of LM_P2M_CHUNK points, slot): NTB threads, each
// owning H coefficients (P <= NTB H); point records (basis values, charges)
// staged in LDS NPT points at a time.  A leaf of one chunk (slot < 0) writes
// its expansion; each chunk of a larger leaf writes a partial expansion to
// slot `slot` of `part` ([slot][rhs][3][Pg]), summed in chunk order by
// k_p2m_sum.  Reaction leaves hold few points (often one or two near the
// interfaces), so they are run with one-wave blocks and LDS sized for their
// own order.
template <int RC, int NTB, int H, int NPT>
__global__ __launch_bounds__(NTB) void k_p2m(DevPlan d, const int* items, const double* xyz, const cd* J,
                                             long long n_src, int n_rhs, cd* ME, cd* part, int Pg) {
  extern __shared__ double sm[];
  const int b = items[3 * blockIdx.x], chunk = items[3 * blockIdx.x + 1], slot = items[3 * blockIdx.x + 2];
  SrcBox sb = d.sbox[b];
  sb.pt0 += chunk * LM_P2M_CHUNK;
  sb.pt1 = min(sb.pt1, sb.pt0 + LM_P2M_CHUNK);
  InstParams ip = d.inst[sb.inst];
  int p = ip.p, P = ip.P, ntri = (p + 1) * (p + 2) / 2;
  int r0 = blockIdx.y * RC, nr = min(RC, n_rhs - r0);
  int stride = (p + 1) + ntri + 2 * (p + 1) + RC * 6;
  int tid = threadIdx.x;
  cd acc[H][RC][3];
  for (int h = 0; h < H; h++)
    for (int r = 0; r < RC; r++)
      for (int c = 0; c < 3; c++) acc[h][r][c] = cd{0, 0};
  for (int base = sb.pt0; base < sb.pt1; base += NPT) {
    int np = min(NPT, sb.pt1 - base);
    __syncthreads();
    if (tid < np) {
      double* rec = sm + tid * stride;
      int id = d.src_perm[base + tid];
      double dx = xyz[3 * id] - sb.c[0], dy = xyz[3 * id + 1] - sb.c[1];
      double dz = ip.as * xyz[3 * id + 2] + ip.bs - sb.c[2];
      double rxy = sqrt(dx * dx + dy * dy), r = sqrt(dx * dx + dy * dy + dz * dz);
      double ct = r > 0 ? dz / r : 1.0, st = r > 0 ? rxy / r : 0.0;
      double ex = rxy > 0 ? dx / rxy : 1.0, ey = rxy > 0 ? dy / rxy : 0.0;
      sph_jn(p, ip.ks * r, rec);
      legendre_rt(p, ct, st, rec + (p + 1));
      double* e = rec + (p + 1) + ntri;  // e^{-i m phi}
      cd em = cd{1.0, 0.0}, e1 = cd{ex, -ey};
      for (int m = 0; m <= p; m++) {
        e[2 * m] = em.x;
        e[2 * m + 1] = em.y;
        em = em * e1;
      }
      double* q = e + 2 * (p + 1);
      for (int rr = 0; rr < RC; rr++) {
        cd jx = cd{0, 0}, jy = cd{0, 0}, jz = cd{0, 0};
        if (rr < nr) {
          const cd* Jp = J + ((long long)(r0 + rr) * n_src + id) * 3;
          jx = Jp[0];
          jy = Jp[1];
          jz = Jp[2];
        }
        cd up = jx + cd{-jy.y, jy.x};  // jx + i jy
        cd um = jx - cd{-jy.y, jy.x};
        q[rr * 6 + 0] = up.x;
        q[rr * 6 + 1] = up.y;
        q[rr * 6 + 2] = um.x;
        q[rr * 6 + 3] = um.y;
        q[rr * 6 + 4] = jz.x;
        q[rr * 6 + 5] = jz.y;
      }
    }
    __syncthreads();
    for (int h = 0; h < H; h++) {
      int nm = tid + NTB * h;
      if (nm >= P) continue;
      int n = n_of(nm), m = nm - n * n - n, am = m < 0 ? -m : m;
      double sg = (m < 0 && (am & 1)) ? -1.0 : 1.0;
      for (int t = 0; t < np; t++) {
        const double* rec = sm + t * stride;
        double rad = rec[n] * rec[(p + 1) + tri_idx(n, am)] * sg;
        const double* e = rec + (p + 1) + ntri;
        cd ph = cd{e[2 * am], m < 0 ? -e[2 * am + 1] : e[2 * am + 1]};
        cd bas = rad * ph;
        const double* q = e + 2 * (p + 1);
        for (int rr = 0; rr < RC; rr++)
          for (int c = 0; c < 3; c++)
            acc[h][rr][c] = cmac_exact(acc[h][rr][c], cd{q[rr * 6 + 2 * c], q[rr * 6 + 2 * c + 1]}, bas);
      }
    }
  }
  for (int h = 0; h < H; h++) {
    int nm = tid + NTB * h;
    if (nm >= P) continue;
    for (int rr = 0; rr < nr; rr++)
      for (int c = 0; c < 3; c++) {
        if (slot < 0)
          ME[sb.me_off * n_rhs + ((long long)(r0 + rr) * 3 + c) * P + nm] = acc[h][rr][c];
        else
          part[(((long long)slot * n_rhs + r0 + rr) * 3 + c) * Pg + nm] = acc[h][rr][c];
      }
  }
}
// ME of a leaf of several chunks: its partials (slots slot0 .. slot0+nch-1)
// added in chunk order.  Work item (leaf, slot0, nch).
__global__ __launch_bounds__(NT) void k_p2m_sum(DevPlan d, const int* items, int n_rhs, const cd* part, int Pg,
                                                cd* ME) {
  const int b = items[3 * blockIdx.x], slot0 = items[3 * blockIdx.x + 1], nch = items[3 * blockIdx.x + 2];
  const SrcBox sb = d.sbox[b];
  const int P = d.inst[sb.inst].P;
  const int nel = n_rhs * 3 * P;
  for (int e = threadIdx.x; e < nel; e += NT) {
    const int rc = e / P, nm = e - rc * P;  // rc = rhs * 3 + channel
    cd acc = cd{0, 0};
    for (int c = 0; c < nch; c++) acc = acc + part[((long long)(slot0 + c) * n_rhs * 3 + rc) * Pg + nm];
    ME[sb.me_off * n_rhs + (long long)rc * P + nm] = acc;
  }
}
void launch_p2m_sum(const DevPlan& d, const int* items, int n, int n_rhs, const cd* part, int Pg, cd* ME,
                    hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_p2m_sum, dim3(n), dim3(NT), 0, s, d, items, n_rhs, part, Pg, ME);
}
template <int RC, int NTB, int H, int NPT>
static void p2m_go(const DevPlan& d, const int* items, int n, const double* xyz, const cd* J, long long n_src,
                   int n_rhs, cd* ME, cd* part, int pl, hipStream_t s) {
  int ntri = (pl + 1) * (pl + 2) / 2;
  size_t shm = (size_t)NPT * ((pl + 1) + ntri + 2 * (pl + 1) + RC * 6) * sizeof(double);
  set_dyn_lds((const void*)k_p2m<RC, NTB, H, NPT>, shm);
  hipLaunchKernelGGL((k_p2m<RC, NTB, H, NPT>), dim3(n, (n_rhs + RC - 1) / RC), dim3(NTB), shm, s, d, items, xyz, J,
                     n_src, n_rhs, ME, part, (pl + 1) * (pl + 1));
}
// items: n work items (leaf, chunk, slot); pl: the largest order among their
// instances (the slot stride of `part` is (pl+1)^2)
void launch_p2m(const DevPlan& d, const int* items, int n, const double* xyz, const cd* J, long long n_src,
                int n_rhs, cd* ME, cd* part, int pl, hipStream_t s) {
  if (n <= 0) return;
  bool rc1 = n_rhs == 1;
  int P = (pl + 1) * (pl + 1);
  if (P <= 64 * 3 && rc1)
    p2m_go<1, 64, 3, 16>(d, items, n, xyz, J, n_src, n_rhs, ME, part, pl, s);
  else if (P <= 128 * 2 && !rc1)
    p2m_go<4, 128, 2, 16>(d, items, n, xyz, J, n_src, n_rhs, ME, part, pl, s);
  else if (rc1)
    p2m_go<1, NT, 2, 32>(d, items, n, xyz, J, n_src, n_rhs, ME, part, pl, s);
  else
    p2m_go<4, NT, 2, 32>(d, items, n, xyz, J, n_src, n_rhs, ME, part, pl, s);
}

// ------------------------------------------------------------------ M2M
// ME_parent[nm] = sum_children sum_{nu mu} Mat_child[nu mu][nm] ME_child[nu mu]
// (regular-to-regular shift, paper Sec. 2; identical for reaction
// components, Sec. 3.3).  One block per (parent, right-hand side), G groups
// of NT threads: group g translates children g, g + G, ... (each staged in
// the group's LDS), and the groups' sums are added in group order (no
// atomics; the same order for every right-hand side).  Coarse levels hold
// few parents, so there G = 4 spreads a parent's eight children over four
// groups (four times the threads in flight); fine levels run G = 1 at the
// higher occupancy of the smaller LDS.
template <int G>
__global__ __launch_bounds__(NT * G) void k_m2m(DevPlan d, const int* parents, int n_rhs, cd* ME) {
  extern __shared__ cd xs[];  // G x 3P
  const int pb = parents[blockIdx.x];
  const SrcBox sp = d.sbox[pb];
  const int P = d.inst[sp.inst].P;
  const int r = blockIdx.y;
  const int g = threadIdx.x / NT, tid = threadIdx.x - g * NT;
  cd* xg = xs + (long long)g * 3 * P;
  cd acc[2][3];
  for (int h = 0; h < 2; h++)
    for (int c = 0; c < 3; c++) acc[h][c] = cd{0, 0};
  for (int c0 = 0; c0 < sp.nchild; c0 += G) {
    const int ci = c0 + g;
    const bool has = ci < sp.nchild;
    const int cb = sp.child0 + ci;
    __syncthreads();
    if (has) {
      const long long base = d.sbox[cb].me_off * n_rhs + (long long)r * 3 * P;
      for (int e = tid; e < 3 * P; e += NT) xg[e] = ME[base + e];
    }
    __syncthreads();
    if (has) {
      const cd* M = d.mats + d.sbox_m2m[cb];
      for (int h = 0; h < 2; h++) {
        const int nm = tid + NT * h;
        if (nm >= P) continue;
        for (int k = 0; k < P; k++) {
          const cd a = M[(long long)k * P + nm];
          for (int c = 0; c < 3; c++) acc[h][c] = cmac_exact(acc[h][c], a, xg[c * P + k]);
        }
      }
    }
  }
  cd* out = ME + sp.me_off * n_rhs + (long long)r * 3 * P;
  if (G == 1) {
    for (int h = 0; h < 2; h++) {
      const int nm = tid + NT * h;
      if (nm >= P) continue;
      for (int c = 0; c < 3; c++) out[c * P + nm] = acc[h][c];
    }
    return;
  }
  __syncthreads();
  for (int h = 0; h < 2; h++) {
    const int nm = tid + NT * h;
    if (nm >= P) continue;
    for (int c = 0; c < 3; c++) xg[c * P + nm] = acc[h][c];
  }
  __syncthreads();
  for (int e = threadIdx.x; e < 3 * P; e += NT * G) {
    cd v = xs[e];
    for (int q = 1; q < G; q++) v = v + xs[(long long)q * 3 * P + e];
    out[e] = v;
  }
}
// one launch per level; G = 4 where the level has fewer parents than eight
// per compute unit
void launch_m2m(const DevPlan& d, const int* parents, int n, int n_rhs, cd* ME, int pmax, hipStream_t s) {
  if (n <= 0) return;
  const int P = (pmax + 1) * (pmax + 1);
  if (n < 2048) {
    const size_t shm = (size_t)4 * 3 * P * sizeof(cd);
    set_dyn_lds((const void*)k_m2m<4>, shm);
    hipLaunchKernelGGL(k_m2m<4>, dim3(n, n_rhs), dim3(NT * 4), shm, s, d, parents, n_rhs, ME);
  } else {
    const size_t shm = (size_t)3 * P * sizeof(cd);
    set_dyn_lds((const void*)k_m2m<1>, shm);
    hipLaunchKernelGGL(k_m2m<1>, dim3(n, n_rhs), dim3(NT), shm, s, d, parents, n_rhs, ME);
  }
}

// ------------------------------------------------------------------ L2L
// LE_child[nm] += sum_{nu mu} Mat[nu mu][nm] LE_parent[nu mu]
template <int RC>
__global__ __launch_bounds__(NT) void k_l2l(DevPlan d, const int* children, int n_rhs, cd* LE) {
  extern __shared__ cd xs[];
  int cb = children[blockIdx.x];
  TgtBox tc = d.tbox[cb];
  TgtBox tp = d.tbox[tc.parent];
  int P = d.inst[tc.inst].P;
  int r0 = blockIdx.y * RC, nr = min(RC, n_rhs - r0);
  int tid = threadIdx.x;
  const cd* M = d.mats + d.tbox_l2l[cb];
  long long pbase = tp.le_off * n_rhs + (long long)r0 * 3 * P;
  for (int e = tid; e < RC * 3 * P; e += NT) xs[e] = (e < nr * 3 * P) ? LE[pbase + e] : cd{0, 0};
  __syncthreads();
  for (int h = 0; h < 2; h++) {
    int nm = tid + NT * h;
    if (nm >= P) continue;
    cd acc[RC][3];
    for (int r = 0; r < RC; r++)
      for (int c = 0; c < 3; c++) acc[r][c] = cd{0, 0};
    for (int k = 0; k < P; k++) {
      cd a = M[(long long)k * P + nm];
      for (int rr = 0; rr < RC; rr++)
        for (int c = 0; c < 3; c++) acc[rr][c] = acc[rr][c] + a * xs[(rr * 3 + c) * P + k];
    }
    for (int rr = 0; rr < nr; rr++)
      for (int c = 0; c < 3; c++) {
        long long idx = tc.le_off * n_rhs + ((long long)(r0 + rr) * 3 + c) * P + nm;
        LE[idx] = LE[idx] + acc[rr][c];
      }
  }
}
// one block per (child, right-hand side): blocks that each served four
// right-hand sides held 4x the LDS and ran at a quarter of the occupancy,
// 1.7x slower per right-hand side than one at a time
void launch_l2l(const DevPlan& d, const int* children, int n, int n_rhs, cd* LE, int pmax, hipStream_t s) {
  if (n <= 0) return;
  int P = (pmax + 1) * (pmax + 1);
  size_t shm = (size_t)3 * P * sizeof(cd);
  set_dyn_lds((const void*)k_l2l<1>, shm);
  hipLaunchKernelGGL(k_l2l<1>, dim3(n, n_rhs), dim3(NT), shm, s, d, children, n_rhs, LE);
}

// ------------------------------------------------------------------ M2L
// Tiled complex GEMM, one tile per (block, offset o, output part, row tile,
// 64 (pair, rhs) columns).  Free space (one channel per output type, phi =
// 0): Y_q[ot] = A_o X_q[ot].
// Reaction: the spin-basis M2L tensor of Sec. 3.3 maps the channels (u+,
// u-, z) of the source box to the outputs (+, -, z) through blocks
// V(sigma, kappa) with the azimuthal phase e^{i q phi}, q = kappa - m + mu.
// Every block has kappa = a_o - b_c (a = 1, -1, 0 for the outputs +, -, z;
// b = 1, -1, 0 for the channels u+, u-, z), so the tensor is
// e^{i (a_o - m) phi} V e^{i (mu - b_c) phi} with a phase-free core V, and V
// commutes with the mirror S: (S x)_{+,nm} = e_m x_{-,n,-m},
// (S x)_{-,nm} = e_m x_{+,n,-m}, (S x)_{z,nm} = e_m x_{z,n,-m}, e_m =
// (-1)^m, because P^{-m}_n = e_m P^m_n, J_|q| depends on |q| only, and the
// blocks of the - output are the kappa -> -kappa images of those of the +
// output with the same densities (the z output's blocks pair among
// themselves).  V therefore maps the even part (x + S x)/2 and the odd part
// (x - S x)/2 of the phased input x~_c = e^{i (mu - b_c) phi} X_c
// separately: two square GEMMs of dimension lm_sym_dim(q, 0) and
// lm_sym_dim(q, 1) (about 1.5 (q+1)^2 each) in place of the 3 (q+1)^2
// square one, half the multiply-adds.  The even (odd) coordinates are
//   + part:  x~_{u+,nm} + (-) e_m x~_{u-,n,-m}   (every nm),
//   z part:  x~_{z,nm} + (-) e_m x~_{z,n,-m}     (m >= 1; m = 0: x~_{z,n0}, even only),
// and k_tab_sym stores V in these coordinates.  V depends on the horizontal
// distance and the heights only, so the offsets of one table case (equal
// distance, different azimuths) share it: their pairs are the columns of
// one GEMM, each column phased with its own pair's azimuth.  Tiles write
// the phase-free even and odd outputs; k_m2l_reduce recombines them per
// pair and applies e^{i (a_o - m) phi}.  Only pairs whose source box exists
// are columns.  Y is a scratch buffer; the reduction adds, per target, its
// pairs in a fixed order (no atomics).
#define TN 64   // columns per tile (the rows are 32 per wave row: 32 * WR)
typedef double v4d __attribute__((ext_vector_type(4)));

// Shared state of one M2L tile (read by all waves of the block).
struct M2LTileCtx {
  const cd* A;        // free: the offset's P x P matrix; reaction: its even or odd block
  const cd* ME;
  cd* Y;
  long long ybase;    // scratch base of the tile's block
  int P;              // (p+1)^2 of the class
  int R;              // rows = columns used by this offset's order
  int Pb;             // (pord+1)^2: the leading R entries are Pb of the first part, then the second part
  int Kf;             // row pitch of the stored matrix (its full dimension)
  int p, ot, row0, ncol, col0, qo, q0b, n_rhs;
  bool sym;           // reaction: ot 0 = even block, 1 = odd block
};

// complex product with a fixed fused multiply-add order: every tile-shape
// variant must round the phases and source coordinates alike, and the
// compiler's own contraction could differ between instantiations
__device__ __forceinline__ cd cmul_fx(cd a, cd b) {
  return cd{__builtin_fma(a.x, b.x, -(a.y * b.y)), __builtin_fma(a.x, b.y, a.y * b.x)};
}

// stored row / column of the offset's r-th used row / column: the first Pb
// entries, then the second part from position P on
__device__ __forceinline__ int m2l_sidx(const M2LTileCtx& c, int r) { return r < c.Pb ? r : c.P + (r - c.Pb); }

// (n, m) of entry j of the z part of the even (m >= 0) or odd (m >= 1)
// coordinates, as the index n^2 + n + m
__device__ inline int sym_znm(int j, int par) {
  int n = par, base = 0;  // base: first entry of order n
  while (j >= base + n + 1 - par) {
    base += n + 1 - par;
    n++;
  }
  return n * n + n + (j - base) + par;
}

// Operand planes are row-major, [row or column][k], pitch KCV + 1 doubles
// (KCV values of k per chunk, NB chunk buffers): the threads that store one
// row's KCV values write consecutive words, and the MFMA operand reads (16
// lanes on 16 rows, 4 groups of lanes on 4 consecutive k) fall on distinct
// banks (the pitch is odd in doubles).
template <int KCV, int NB, int WR>
struct M2LLds {
  double Ar[NB][32 * WR][KCV + 1], Ai[NB][32 * WR][KCV + 1], Br[NB][TN][KCV + 1], Bi[NB][TN][KCV + 1];
  long long sbase[TN];
  // reaction: powers of each column's e^{i phi}: lo[c][j] = e^{i j phi}
  // (j < 8), hi[c][j] = e^{i 8 j phi} (j < 4), so e^{i e phi} for |e| < 32
  // is lo[e % 8] hi[e / 8] (conjugated for e < 0)
  cd plo[TN][8], phi8[TN][4];
};

// K loop and epilogue of one wave whose 32 x 32 wave tile has NI x NJ active
// 16 x 16 MFMA tiles (NI, NJ in 0..2; rows beyond R and columns beyond the
// pair count are never computed).  Every wave of the block runs the same
// number of barriers whatever its NI, NJ.
// MFMA operand layout (v_mfma_f64_16x16x4f64, one fp64 per lane and
// operand): lane l holds A[l % 16][l / 16] and B[l / 16][l % 16]; the four
// result registers of lane l hold C[4 r + l / 16][l % 16], r = 0..3.  The
// kernel passes the source values (lane l: column l % 16, k = l / 16) as
// the first operand and the matrix (lane l: row l % 16, k = l / 16) as the
// second, so it accumulates the transposed tile.
// Complex product with three real MFMAs per step (Gauss): P1 = sum A_re
// B_re, P2 = sum A_im B_im, P3 = sum (A_re + A_im)(B_re + B_im); then C_re =
// P1 - P2 and C_im = P3 - P1 - P2.  The accumulator chains are interleaved
// so that no MFMA waits on the one issued just before it.
// Tile-shape variants (the same sums in the same order, so bitwise equal
// results): KCV values of k per LDS chunk; NB = 1 stages a chunk, waits,
// multiplies and waits again; NB = 2 loads the next chunk into registers
// while the current one is multiplied and stores it into the other buffer
// (one barrier per chunk).
template <int KCV, int NB, int WR, int NI, int NJ, bool SYM>
__device__ __forceinline__ void m2l_wave(const M2LTileCtx& c, M2LLds<KCV, NB, WR>& L, int tid, int wr, int wc) {
  constexpr int NIx = NI > 0 ? NI : 1, NJx = NJ > 0 ? NJ : 1;
  v4d p1[NIx][NJx], p2[NIx][NJx], p3[NIx][NJx];
#pragma unroll
  for (int i = 0; i < NIx; i++)
#pragma unroll
    for (int j = 0; j < NJx; j++) {
      p1[i][j] = v4d{0, 0, 0, 0};
      p2[i][j] = p1[i][j];
      p3[i][j] = p1[i][j];
    }
  const int lane = tid & 63;
  // rows (matrix) / columns (source vectors) staged per pass: all 128 WR
  // threads stage the 32 WR matrix rows (RPI rows per pass), the first 256
  // the 64 source columns (RPB columns per pass); KCV / 4 of each per thread
  constexpr int NTB = 128 * WR, RPI = NTB / KCV, RPB = 256 / KCV;
  constexpr int NA = 32 * WR / RPI, NB_ = TN / RPB;
  const bool bst = tid < 256;
  // fixed roles of this thread in the chunk loads: k offset kk, and rows
  // r16 + RPI it, columns r16 + RPB it; indices outside the tile are
  // clamped to a valid entry and the value zeroed
  const int kk = tid & (KCV - 1), r16 = tid / KCV;
  int aoff[NA];  // below 2^31: the largest matrix has lm_sym_dim(LM_PMAX, 0)^2 entries
  bool aok[NA];
#pragma unroll
  for (int it = 0; it < NA; it++) {
    int row = c.row0 + r16 + RPI * it;
    aok[it] = row < c.R;
    aoff[it] = m2l_sidx(c, aok[it] ? row : c.R - 1) * c.Kf;
  }
  cd ra[NA], rb[NB_], rm[SYM ? NB_ : 1];
  // source coordinate of this thread's k (reaction): channel entries i1 and
  // i2 (its mirror) with phases e^{i e1 phi} and e^{-i e1 phi}, the mirror
  // term with sign s2 (-1, 0 or 1)
  int e1 = 0, s2 = 0;
  auto load = [&](int k0) {
    const int k = k0 + kk;
    const bool kok = k < c.R;
    const int kc = kok ? k : c.R - 1;
    const int colA = m2l_sidx(c, kc);
#pragma unroll
    for (int it = 0; it < NA; it++) {
      cd v = c.A[aoff[it] + colA];
      ra[it] = (aok[it] && kok) ? v : cd{0, 0};
    }
    if (!bst) return;
    // source columns: base offsets re-read from LDS (fewer live registers);
    // columns without a pair read column 0 and are zeroed
    long long boff[NB_];
    bool bok[NB_];
#pragma unroll
    for (int it = 0; it < NB_; it++) {
      const long long sb = L.sbase[r16 + RPB * it];
      bok[it] = sb >= 0;
      boff[it] = sb >= 0 ? sb : L.sbase[0];
    }
    if (SYM) {
      // (n, mu) of coordinate kc: the + part in nm order, then the z part
      // with mu >= 0 (even) or mu >= 1 (odd), n-major
      const bool zp = kc >= c.Pb;
      int n, mu;
      if (!zp) {
        n = n_of(kc);
        mu = kc - n * n - n;
      } else {
        const int j = kc - c.Pb;
        const double sq = sqrt(8.0 * j + 1.0);
        if (c.ot == 0) {
          n = (int)((sq - 1.0) * 0.5);
          mu = j - n * (n + 1) / 2;
        } else {
          n = (int)((sq + 1.0) * 0.5);
          mu = j - n * (n - 1) / 2 + 1;
        }
      }
      const int nm = n * n + n + mu;
      const int i1 = (zp ? 2 * c.P : 0) + nm;          // u+ or z
      const int i2 = (zp ? 2 * c.P : c.P) + nm - 2 * mu;  // u- or z, order -mu
      e1 = zp ? mu : mu - 1;
      s2 = (zp && mu == 0) ? 0 : ((c.ot ? -1 : 1) * ((mu & 1) ? -1 : 1));
#pragma unroll
      for (int it = 0; it < NB_; it++) {
        cd v = c.ME[boff[it] + i1], w = c.ME[boff[it] + i2];
        rb[it] = (bok[it] && kok) ? v : cd{0, 0};
        rm[it] = (bok[it] && kok) ? w : cd{0, 0};
      }
    } else {
      const long long colB = (long long)c.ot * c.P + kc;
#pragma unroll
      for (int it = 0; it < NB_; it++) {
        cd v = c.ME[boff[it] + colB];
        rb[it] = (bok[it] && kok) ? v : cd{0, 0};
      }
    }
  };
  // registers -> LDS planes of buffer bf (reaction: the even or odd
  // coordinate of the phased source vector, each column with the phase
  // e^{i e1 phi} of its own pair; the phases are read before any store)
  auto store = [&](int bf) {
    cd ph[SYM ? NB_ : 1];
    if (SYM && bst) {
      const int ae = e1 < 0 ? -e1 : e1;
#pragma unroll
      for (int it = 0; it < NB_; it++) {
        const int col = r16 + RPB * it;
        ph[it] = cmul_fx(L.plo[col][ae & 7], L.phi8[col][ae >> 3]);
        if (e1 < 0) ph[it] = cconj(ph[it]);
      }
    }
#pragma unroll
    for (int it = 0; it < NA; it++) {
      L.Ar[bf][r16 + RPI * it][kk] = ra[it].x;
      L.Ai[bf][r16 + RPI * it][kk] = ra[it].y;
    }
    if (!bst) return;
    if (SYM) {
#pragma unroll
      for (int it = 0; it < NB_; it++) {
        const cd u = cmul_fx(ph[it], rb[it]), w = cmul_fx((double)s2 * cconj(ph[it]), rm[it]);
        const cd v = cd{u.x + w.x, u.y + w.y};
        L.Br[bf][r16 + RPB * it][kk] = v.x;
        L.Bi[bf][r16 + RPB * it][kk] = v.y;
      }
    } else {
#pragma unroll
      for (int it = 0; it < NB_; it++) {
        L.Br[bf][r16 + RPB * it][kk] = rb[it].x;
        L.Bi[bf][r16 + RPB * it][kk] = rb[it].y;
      }
    }
  };
  auto mma = [&](int bf) {
    if (NI > 0 && NJ > 0) {
#pragma unroll
      for (int k4 = 0; k4 < KCV; k4 += 4) {
        const int kr = k4 + (lane >> 4), li = lane & 15;
        double a_r[NIx], a_i[NIx], a_s[NIx], b_r[NJx], b_i[NJx], b_s[NJx];
#pragma unroll
        for (int i = 0; i < NIx; i++) {
          a_r[i] = L.Ar[bf][wr * 32 + i * 16 + li][kr];
          a_i[i] = L.Ai[bf][wr * 32 + i * 16 + li][kr];
          a_s[i] = a_r[i] + a_i[i];
        }
#pragma unroll
        for (int j = 0; j < NJx; j++) {
          b_r[j] = L.Br[bf][wc * 32 + j * 16 + li][kr];
          b_i[j] = L.Bi[bf][wc * 32 + j * 16 + li][kr];
          b_s[j] = b_r[j] + b_i[j];
        }
#pragma unroll
        for (int i = 0; i < NIx; i++)
#pragma unroll
          for (int j = 0; j < NJx; j++) p1[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(b_r[j], a_r[i], p1[i][j], 0, 0, 0);
#pragma unroll
        for (int i = 0; i < NIx; i++)
#pragma unroll
          for (int j = 0; j < NJx; j++) p2[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(b_i[j], a_i[i], p2[i][j], 0, 0, 0);
#pragma unroll
        for (int i = 0; i < NIx; i++)
#pragma unroll
          for (int j = 0; j < NJx; j++) p3[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(b_s[j], a_s[i], p3[i][j], 0, 0, 0);
      }
    }
  };
  if (NB == 1) {
    for (int k0 = 0; k0 < c.R; k0 += KCV) {
      load(k0);
      store(0);
      __syncthreads();
      mma(0);
      __syncthreads();
    }
  } else {
    // chunk k0 is in buffer (k0 / KCV) & 1; the loads of the next chunk are
    // in flight during this chunk's MFMAs, and its stores go to the buffer
    // that every wave finished reading before the previous barrier
    load(0);
    store(0);
    __syncthreads();
    for (int k0 = 0; k0 < c.R; k0 += KCV) {
      const int bf = (k0 / KCV) & 1;
      const bool more = k0 + KCV < c.R;
      if (more) load(k0 + KCV);
      mma(bf);
      if (more) store(bf ^ 1);
      __syncthreads();
    }
  }
  if (NI == 0 || NJ == 0) return;
  // epilogue.  The MFMAs take the source values as their first operand and
  // the matrix as their second, so each 16 x 16 accumulator holds the
  // transposed tile: register r of lane l is row lane % 16 of column
  // 4 r + lane / 16, and the 16 lanes of one column write 16 consecutive
  // rows (one contiguous 256-byte run instead of 16 scattered 16-byte
  // stores).  Column j of the tile is (pair, rhs) = (qo + (col0 + j) / n_rhs,
  // (col0 + j) % n_rhs) and goes to that pair's scratch vector: free space
  // [pair][ot][rhs][P], reaction [pair][even: rhs][lm_sym_dim(p, 0)] then
  // [odd: rhs][lm_sym_dim(p, 1)] (3 n_rhs P per pair either way)
  const int li = lane & 15, rq = lane >> 4;
#pragma unroll
  for (int i = 0; i < NIx; i++)
#pragma unroll
    for (int j = 0; j < NJx; j++) {
      const int row = c.row0 + wr * 32 + i * 16 + li;
      const v4d vr = p1[i][j] - p2[i][j], vi = p3[i][j] - p1[i][j] - p2[i][j];
#pragma unroll
      for (int rr = 0; rr < 4; rr++) {
        const int col = wc * 32 + j * 16 + 4 * rr + rq;
        if (col >= c.ncol || row >= c.R) continue;
        const int jj = c.col0 + col;
        const int q = c.qo + jj / c.n_rhs, r = jj % c.n_rhs;
        cd* Yq = SYM ? c.Y + c.ybase + (long long)(q - c.q0b) * 3 * c.n_rhs * c.P +
                             (c.ot ? (long long)c.n_rhs * lm_sym_dim(c.p, 0) : 0) + (long long)r * c.Kf
                       : c.Y + c.ybase + ((long long)((q - c.q0b) * 3 + c.ot) * c.n_rhs + r) * c.P;
        Yq[m2l_sidx(c, row)] = cd{vr[rr], vi[rr]};
      }
    }
}

// One (32 WR) x 64 output tile per block, complex fp64 on the matrix cores.
// The 2 WR waves form a WR x 2 grid of 32 x 32 wave tiles; a wave computes
// only those of its four 16 x 16 MFMA tiles that hold rows below the
// offset's R and columns below the tile's pair count, so partial tiles cost
// little; the choice is made once per tile from a wave-uniform value.  Operands are
// staged through LDS as separate real / imaginary planes, KCV values of k at
// a time (variants above); resident blocks overlap one block's global loads
// with the others' MFMAs.  Consecutive tiles are sent to one XCD (blocks are
// dealt round-robin over the 8 XCDs), so the tiles sharing one offset's
// matrix and source vectors run against one L2.
template <int KCV, int NB, int OCC, int WR>
__global__ __launch_bounds__(128 * WR, OCC) void k_m2l(DevPlan d, const M2LTile* tiles, int n_tiles, int n_rhs,
                                                       const cd* ME, cd* Y) {
  __shared__ M2LLds<KCV, NB, WR> L;
  const int per_xcd = (n_tiles + 7) >> 3;
  const int t_id = (int)(blockIdx.x & 7) * per_xcd + (int)(blockIdx.x >> 3);
  if (t_id >= n_tiles) return;
  const M2LTile tl = tiles[t_id];
  const int tid = threadIdx.x;
  M2LTileCtx c;
  c.P = tl.P;
  c.p = tl.p;
  c.ot = tl.ot;
  c.sym = tl.sym != 0;
  // order used for this offset: free space, the leading Pb rows and columns
  // of the P x P matrix; reaction, the leading entries of both parts
  c.Pb = tl.Pb;
  c.R = tl.R;
  c.Kf = tl.Kf;
  c.row0 = tl.row0;
  c.ncol = tl.ncol;
  c.col0 = tl.col0;
  c.qo = tl.qo;      // first pair of this offset
  c.q0b = tl.q0b;
  c.n_rhs = n_rhs;
  c.ybase = tl.ybase;  // per-block scratch base (blocks differ in P)
  c.A = d.mats + tl.mat;
  c.ME = ME;
  c.Y = Y;
  if (c.sym && tid < TN) {
    // the tile's columns may come from several offsets of one table case:
    // each column takes the azimuth of its own pair (columns past the
    // tile's count: any valid value, their sources are zero)
    const int q = c.qo + (tl.col0 + (tid < tl.ncol ? tid : 0)) / n_rhs;
    const double phi = d.pair_phi[q];
    const cd z = cd{cos(phi), sin(phi)};
    cd w = cd{1, 0};
    for (int j = 0; j < 8; j++) {
      L.plo[tid][j] = w;
      w = cmul_fx(w, z);
    }
    const cd z8 = w;
    w = cd{1, 0};
    for (int j = 0; j < 4; j++) {
      L.phi8[tid][j] = w;
      w = cmul_fx(w, z8);
    }
  }
  if (tid < TN) {
    long long v = -1;
    if (tid < tl.ncol) {
      int j = tl.col0 + tid;
      int q = c.qo + j / n_rhs, r = j % n_rhs;
      v = d.pair_me[q] * n_rhs + (long long)r * 3 * c.P;
    }
    L.sbase[tid] = v;
  }
  __syncthreads();
  // this wave's active MFMA tiles (uniform over the wave, kept in an SGPR)
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wr = wave >> 1, wc = wave & 1;
  const int ni = (c.row0 + wr * 32 < c.R) + (c.row0 + wr * 32 + 16 < c.R);
  const int nj = (wc * 32 < c.ncol) + (wc * 32 + 16 < c.ncol);
  const int pat = __builtin_amdgcn_readfirstlane(ni * 3 + nj);
  if (c.sym) {
    switch (pat) {
      case 4: m2l_wave<KCV, NB, WR, 1, 1, true>(c, L, tid, wr, wc); break;
      case 5: m2l_wave<KCV, NB, WR, 1, 2, true>(c, L, tid, wr, wc); break;
      case 7: m2l_wave<KCV, NB, WR, 2, 1, true>(c, L, tid, wr, wc); break;
      case 8: m2l_wave<KCV, NB, WR, 2, 2, true>(c, L, tid, wr, wc); break;
      default: m2l_wave<KCV, NB, WR, 0, 0, true>(c, L, tid, wr, wc); break;
    }
  } else {
    switch (pat) {
      case 4: m2l_wave<KCV, NB, WR, 1, 1, false>(c, L, tid, wr, wc); break;
      case 5: m2l_wave<KCV, NB, WR, 1, 2, false>(c, L, tid, wr, wc); break;
      case 7: m2l_wave<KCV, NB, WR, 2, 1, false>(c, L, tid, wr, wc); break;
      case 8: m2l_wave<KCV, NB, WR, 2, 2, false>(c, L, tid, wr, wc); break;
      default: m2l_wave<KCV, NB, WR, 0, 0, false>(c, L, tid, wr, wc); break;
    }
  }
}
// variant (tiles of 64 rows, 4 waves; 3 waves per SIMD): 0 = 8 values of k
// per chunk, one buffer; 1 = 4 values, two buffers; 2 = 8 values, two
// buffers (LM_M2L_VARIANTS variants, bitwise equal results).  Tiles of 96
// rows (WR = 3, two blocks of 6 waves per CU) measured 40% slower.
void launch_m2l(const DevPlan& d, const M2LTile* tiles, int n_tiles, int n_rhs, const cd* ME, cd* Y, int pmax,
                int variant, hipStream_t s) {
  if (n_tiles <= 0) return;
  int grid = ((n_tiles + 7) / 8) * 8;
  switch (variant) {
    case 1: hipLaunchKernelGGL((k_m2l<4, 2, 3, 2>), dim3(grid), dim3(256), 0, s, d, tiles, n_tiles, n_rhs, ME, Y); break;
    case 2: hipLaunchKernelGGL((k_m2l<8, 2, 3, 2>), dim3(grid), dim3(256), 0, s, d, tiles, n_tiles, n_rhs, ME, Y); break;
    default: hipLaunchKernelGGL((k_m2l<8, 1, 3, 2>), dim3(grid), dim3(256), 0, s, d, tiles, n_tiles, n_rhs, ME, Y); break;
  }
}

// LE_t[out][rhs] += sum over the target's pairs (fixed offset order) of the
// pair's output.  Free space: Y as written.  Reaction: the pair's even (E)
// and odd (O) outputs recombined and phased (k_m2l), with e_m = (-1)^m and
// the z part indexed by (n, |m|):
//   (+, nm):  e^{i (1 - m) phi} (E_{+,nm} + O_{+,nm})
//   (-, nm):  e^{i (-1 - m) phi} e_m (E_{+,n,-m} - O_{+,n,-m})
//   (z, nm):  e^{-i m phi} (E_{z,n|m|} + O_{z,n|m|}) for m >= 0 (no O at m = 0),
//             e^{-i m phi} e_m (E_{z,n|m|} - O_{z,n|m|}) for m < 0;
// the phases of LM_RED_PAIRS pairs at a time are tabulated in LDS, and each
// such group is added into LE in turn.  (At m = 0 of the z part, O is absent
// and the second output coincides with the first: only the first is kept.)
#define LM_RED_PAIRS 32
#define RED_NT 512  // threads per target: the even part of p = 12 (260 entries) in one pass
__global__ __launch_bounds__(RED_NT) void k_m2l_reduce(DevPlan d, int bt0, int n_rhs, const cd* Y, cd* LE) {
  __shared__ cd ph[LM_RED_PAIRS][2 * LM_PMAX + 5];
  int bt = bt0 + blockIdx.x;
  TgtBox tb = d.tbox[d.bt_tbox[bt]];
  const int P = d.inst[tb.inst].P, p = d.inst[tb.inst].p;
  int blk = d.bt_blk[bt];
  long long ybase = d.blk_ybase[blk];
  int qb = d.blocks[blk].q0;
  int q0 = d.bt_ptr[bt], q1 = d.bt_ptr[bt + 1];
  int nel = 3 * n_rhs * P;
  if (d.cls[d.blocks[blk].cls].nblk != 3) {
    for (int e = threadIdx.x; e < nel; e += RED_NT) {
      int tr_ = e / P, row = e - tr_ * P;   // tr_ = ot * n_rhs + r
      int ot = tr_ / n_rhs, r = tr_ - ot * n_rhs;
      cd s = cd{0, 0};
      for (int qi = q0; qi < q1; qi++) {
        int q = d.bt_pairs[qi];
        if (row < d.pair_P[q]) s = s + Y[ybase + ((long long)(q - qb) * 3 * n_rhs + tr_) * P + row];
      }
      long long idx = tb.le_off * n_rhs + ((long long)r * 3 + ot) * P + row;
      LE[idx] = LE[idx] + s;
    }
    return;
  }
  __shared__ long long yq[LM_RED_PAIRS];  // each pair's scratch vector
  __shared__ int plim[LM_RED_PAIRS];      // and its (pord+1)^2
  const int Re = lm_sym_dim(p, 0), Ro = lm_sym_dim(p, 1), NJ = 2 * p + 5;
  // one thread per (rhs, entry of the even part): the + part entries nm give
  // (+, nm) and (-, n, -m), the z part entries (n, m >= 0) give (z, n, m) and
  // (z, n, -m); both outputs of an entry read the same E and O entries, with
  // conjugate phases
  for (int c0 = q0; c0 < q1; c0 += LM_RED_PAIRS) {
    const int nc = min(LM_RED_PAIRS, q1 - c0);
    __syncthreads();
    for (int e = threadIdx.x; e < nc * NJ; e += RED_NT) {
      const int i = e / NJ, j = e - i * NJ;
      const double a = (j - (p + 2)) * d.pair_phi[d.bt_pairs[c0 + i]];
      ph[i][j] = cd{cos(a), sin(a)};
    }
    if (threadIdx.x < LM_RED_PAIRS) {
      const int i = threadIdx.x;
      const int q = i < nc ? d.bt_pairs[c0 + i] : qb;
      yq[i] = ybase + (long long)(q - qb) * 3 * n_rhs * P;
      plim[i] = i < nc ? d.pair_P[q] : 0;
    }
    __syncthreads();
    for (int u = threadIdx.x; u < n_rhs * Re; u += RED_NT) {
      const int r = u / Re, w = u - r * Re;  // w: entry of the even part
      const bool zp = w >= P;
      int n, m, io, jph;
      if (!zp) {
        n = n_of(w);
        m = w - n * n - n;
        io = w;
        jph = 1 - m;   // e^{i (1 - m) phi} on (+, nm), its conjugate on (-, n, -m)
      } else {
        const int t = w - P;  // (n, m >= 0) in the z part
        n = 0;
        while ((n + 1) * (n + 2) / 2 <= t) n++;
        m = t - n * (n + 1) / 2;
        io = w - n - 1;       // (n, m) in the z part of O (m >= 1)
        jph = -m;             // e^{-i m phi} on (z, nm), its conjugate on (z, n, -m)
      }
      const int nm = n * n + n + m;
      const bool has_o = !zp || m > 0;
      cd s1 = cd{0, 0}, s2 = cd{0, 0};
      const long long oe = (long long)r * Re + w, oo = (long long)n_rhs * Re + (long long)r * Ro + (has_o ? io : w);
#pragma unroll 4
      for (int i = 0; i < nc; i++) {
        // pairs whose order is below n contribute nothing
        const bool ok = nm < plim[i];
        const cd* Yp = Y + yq[i];
        const cd E = ok ? Yp[oe] : cd{0, 0};
        const cd O = (ok && has_o) ? Yp[oo] : cd{0, 0};
        const cd f = ph[i][jph + p + 2];
        s1 = s1 + f * (E + O);
        s2 = s2 + cconj(f) * (E - O);
      }
      const double em = (m & 1) ? -1.0 : 1.0;
      cd* L0 = LE + tb.le_off * n_rhs + (long long)r * 3 * P;
      if (!zp) {
        L0[nm] = L0[nm] + s1;
        L0[P + nm - 2 * m] = L0[P + nm - 2 * m] + em * s2;
      } else {
        L0[2 * P + nm] = L0[2 * P + nm] + s1;
        if (m > 0) L0[2 * P + nm - 2 * m] = L0[2 * P + nm - 2 * m] + em * s2;
      }
    }
  }
}
void launch_m2l_reduce(const DevPlan& d, int bt0, int nbt, int n_rhs, const cd* Y, cd* LE, int pmax,
                       hipStream_t s) {
  if (nbt <= 0) return;
  hipLaunchKernelGGL(k_m2l_reduce, dim3(nbt), dim3(RED_NT), 0, s, d, bt0, n_rhs, Y, LE);
}

// ------------------------------------------------------------------ L2P
// Reaction: Phi(r) = sum l_nm j_n(k|d|) Y^m_n(d), d = effective(r) - centre
// (Sec. 3.3, the LE of a reaction component).  Free space: the LE of the
// vector potential U is turned into the LE of U + grad div U / k^2 with the
// exact ladder relations of the regular wave functions (paper Sec. 2: the
// dyadic operator applied to the local expansion), then evaluated.
__device__ inline double lad_a(int n, int m) {  // z ladder
  if (n < 0 || (m < 0 ? -m : m) > n) return 0.0;
  return sqrt((double)(n + 1 - m) * (n + 1 + m) / ((2.0 * n + 1) * (2.0 * n + 3)));
}
__device__ inline double lad_b1(int n, int m) { return sqrt((double)(n + m + 1) * (n + m + 2) / ((2.0 * n + 1) * (2.0 * n + 3))); }
__device__ inline double lad_b2(int n, int m) {
  double v = (double)(n - m) * (n - m - 1);
  return (n <= 0 || v <= 0) ? 0.0 : sqrt(v / ((2.0 * n - 1) * (2.0 * n + 1)));
}
__device__ inline double lad_c1(int n, int m) { return sqrt((double)(n - m + 1) * (n - m + 2) / ((2.0 * n + 1) * (2.0 * n + 3))); }
__device__ inline double lad_c2(int n, int m) {
  double v = (double)(n + m) * (n + m - 1);
  return (n <= 0 || v <= 0) ? 0.0 : sqrt(v / ((2.0 * n - 1) * (2.0 * n + 1)));
}
// coefficient of order `oi` (vector c, index nm) at (n, m); 0 outside
__device__ inline cd cget(const cd* c, int oi, int n, int m) {
  if (n < 0 || n > oi || m < -n || m > n) return cd{0, 0};
  return c[nm_idx(n, m)];
}
// out (order oi+1) = D c, dir 0: d/dx + i d/dy, 1: d/dx - i d/dy, 2: d/dz (times 1/k)
__device__ inline cd dapply(const cd* c, int oi, int dir, int n, int m) {
  if (dir == 2) return lad_a(n, m) * cget(c, oi, n + 1, m) - lad_a(n - 1, m) * cget(c, oi, n - 1, m);
  if (dir == 0) {
    cd v = cd{0, 0};
    if (n - 1 >= 0 && m - 1 >= -(n - 1) && m - 1 <= n - 1) v = v + lad_b1(n - 1, m - 1) * cget(c, oi, n - 1, m - 1);
    v = v + lad_b2(n + 1, m - 1) * cget(c, oi, n + 1, m - 1);
    return v;
  }
  cd v = cd{0, 0};
  if (n - 1 >= 0 && m + 1 >= -(n - 1) && m + 1 <= n - 1) v = v + lad_c1(n - 1, m + 1) * cget(c, oi, n - 1, m + 1);
  v = v + lad_c2(n + 1, m + 1) * cget(c, oi, n + 1, m + 1);
  return -1.0 * v;
}

// NTB threads per leaf (one point each at a time); the spherical Bessel
// values of each thread's point sit in its own LDS slot.
template <int RC, int NTB>
__global__ __launch_bounds__(NTB) void k_l2p(DevPlan d, const int* leaves, int ch, int kind, const double* xyz,
                                             long long n_tgt, int n_rhs, const cd* LE, cd* A) {
  extern __shared__ cd Ls[];
  // work item: (leaf, chunk of ch points)
  int b = leaves[2 * blockIdx.x];
  const int q0 = d.tbox[b].pt0 + leaves[2 * blockIdx.x + 1] * ch;
  TgtBox tb = d.tbox[b];
  InstParams ip = d.inst[tb.inst];
  int p = ip.p, P = ip.P;
  int pe = (kind == 0) ? p + 2 : p, Pe = (pe + 1) * (pe + 1);
  int r0 = blockIdx.y * RC, nr = min(RC, n_rhs - r0);
  int tid = threadIdx.x;
  double k = ip.kt;
  cd* Lc = Ls;                       // [RC][3][Pe]
  cd* Dv = Ls + RC * 3 * Pe;         // [RC][(p+2)^2] divergence
  for (int e = tid; e < RC * 3 * Pe; e += NTB) {
    int rr = e / (3 * Pe), rem = e - rr * 3 * Pe, c = rem / Pe, nm = rem - c * Pe;
    cd v = cd{0, 0};
    if (rr < nr && nm < P) v = LE[tb.le_off * n_rhs + ((long long)(r0 + rr) * 3 + c) * P + nm];
    Lc[e] = v;
  }
  __syncthreads();
  if (kind == 0) {
    int Pd = (p + 2) * (p + 2);
    for (int e = tid; e < RC * Pd; e += NTB) {
      int rr = e / Pd, nm = e - rr * Pd;
      int n = n_of(nm), m = nm - n * n - n;
      const cd* Lp = Lc + (rr * 3 + 0) * Pe;
      const cd* Lm = Lc + (rr * 3 + 1) * Pe;
      const cd* Lz = Lc + (rr * 3 + 2) * Pe;
      cd v = 0.5 * (dapply(Lm, p, 0, n, m) + dapply(Lp, p, 1, n, m)) + dapply(Lz, p, 2, n, m);
      Dv[e] = k * v;
    }
    __syncthreads();
    // A = U + grad div U / k^2 (order p+2); the gradient only reads Dv
    for (int e = tid; e < RC * 3 * Pe; e += NTB) {
      int rr = e / (3 * Pe), rem = e - rr * 3 * Pe, c = rem / Pe, nm = rem - c * Pe;
      int n = n_of(nm), m = nm - n * n - n;
      Lc[e] = Lc[e] + (1.0 / k) * dapply(Dv + rr * Pd, p + 1, c, n, m);
    }
    __syncthreads();
  }
  const int q1 = min(tb.pt1, q0 + ch);
  for (int t0 = q0; t0 < q1; t0 += NTB) {
    int ti = t0 + tid;
    if (ti >= q1) continue;
    int id = d.tgt_perm[ti];
    double dx = xyz[3 * id] - tb.c[0], dy = xyz[3 * id + 1] - tb.c[1];
    double dz = ip.at * xyz[3 * id + 2] + ip.bt - tb.c[2];
    double rxy = sqrt(dx * dx + dy * dy), r = sqrt(dx * dx + dy * dy + dz * dz);
    double ct = r > 0 ? dz / r : 1.0, st = r > 0 ? rxy / r : 0.0;
    cd e1 = rxy > 0 ? cd{dx / rxy, dy / rxy} : cd{1.0, 0.0};
    double* jn = (double*)(Dv + RC * (p + 2) * (p + 2)) + tid * (pe + 1);
    sph_jn(pe, k * r, jn);
    cd acc[RC][3];
    for (int rr = 0; rr < RC; rr++)
      for (int c = 0; c < 3; c++) acc[rr][c] = cd{0, 0};
    // m-outer recurrence for the orthonormal Legendre functions
    double pmm = LM_INV_SQRT_4PI;
    cd em = cd{1.0, 0.0};
    for (int m = 0; m <= pe; m++) {
      if (m > 0) {
        pmm = c_leg_mm[m] * st * pmm;
        em = em * e1;
      }
      double p2 = 0.0, p1 = pmm;
      for (int n = m; n <= pe; n++) {
        double pn;
        if (n == m)
          pn = pmm;
        else if (n == m + 1)
          pn = c_leg_m1[m] * ct * pmm;
        else
          pn = c_leg_a[n * LEGN + m] * (ct * p1 - c_leg_b[n * LEGN + m] * p2);
        if (n > m) {
          p2 = p1;
          p1 = pn;
        }
        double rad = jn[n] * pn;
        cd bp = rad * em;                       // j_n Y^m_n
        int ip_ = nm_idx(n, m), im_ = nm_idx(n, -m);
        for (int rr = 0; rr < RC; rr++)
          for (int c = 0; c < 3; c++) {
            const cd* L = Lc + (rr * 3 + c) * Pe;
            acc[rr][c] = cmac_exact(acc[rr][c], L[ip_], bp);
            if (m > 0) {
              cd bm = ((m & 1) ? -rad : rad) * cconj(em);  // j_n Y^{-m}_n
              acc[rr][c] = cmac_exact(acc[rr][c], L[im_], bm);
            }
          }
      }
    }
    for (int rr = 0; rr < nr; rr++) {
      cd vp = acc[rr][0], vm = acc[rr][1], vz = acc[rr][2];
      cd ax = 0.5 * (vp + vm);
      cd dd = 0.5 * (vp - vm);
      cd ay = cd{dd.y, -dd.x};  // (vp - vm) / (2i)
      cd* Ap = A + ((long long)(r0 + rr) * n_tgt + id) * 3;
      Ap[0] = Ap[0] + ax;
      Ap[1] = Ap[1] + ay;
      Ap[2] = Ap[2] + vz;
    }
  }
}
template <int RC, int NTB>
static void l2p_go(const DevPlan& d, const int* leaves, int n, int ch, int kind, const double* xyz, long long n_tgt,
                   int n_rhs, const cd* LE, cd* A, int pi, hipStream_t s) {
  int pe = kind == 0 ? pi + 2 : pi;
  int Pe = (pe + 1) * (pe + 1), Pd = (pi + 2) * (pi + 2);
  size_t shm = (size_t)(RC * 3 * Pe + RC * Pd) * sizeof(cd) + (size_t)NTB * (pe + 1) * sizeof(double);
  set_dyn_lds((const void*)k_l2p<RC, NTB>, shm);
  hipLaunchKernelGGL((k_l2p<RC, NTB>), dim3(n, (n_rhs + RC - 1) / RC), dim3(NTB), shm, s, d, leaves, ch, kind, xyz,
                     n_tgt, n_rhs, LE, A);
}
// leaves: n work items (leaf, chunk of LM_L2P_CHUNK(kind) points); pi: the
// instance's expansion order.  Reaction items (kind 1) run with one-wave
// blocks, free-space ones with 256 threads.
void launch_l2p(const DevPlan& d, const int* leaves, int n, int kind, const double* xyz, long long n_tgt,
                int n_rhs, const cd* LE, cd* A, int pi, hipStream_t s) {
  if (n <= 0) return;
  // one right-hand side per block (four per block measured 1.7x slower per
  // right-hand side: 4x the LDS, a quarter of the occupancy)
  int ch = LM_L2P_CHUNK(kind);
  if (kind == 1)
    l2p_go<1, 64>(d, leaves, n, ch, kind, xyz, n_tgt, n_rhs, LE, A, pi, s);
  else
    l2p_go<1, NT>(d, leaves, n, ch, kind, xyz, n_tgt, n_rhs, LE, A, pi, s);
}

// One pair's dyadic contribution, acc_c += a q_c + u_c b (u . q): the dot
// product and b (u . q) formed once, every product folded into a
// multiply-add chain.
__device__ __forceinline__ void p2p_apply(cd* acc, cd a, cd bq, double ux, double uy, double uz, cd qx, cd qy,
                                          cd qz) {
  const double dre = fma(ux, qx.x, fma(uy, qy.x, uz * qz.x));
  const double dim = fma(ux, qx.y, fma(uy, qy.y, uz * qz.y));
  const double bre = fma(bq.x, dre, -(bq.y * dim)), bim = fma(bq.x, dim, bq.y * dre);
  acc[0] = cd{fma(a.x, qx.x, fma(-a.y, qx.y, fma(ux, bre, acc[0].x))),
              fma(a.x, qx.y, fma(a.y, qx.x, fma(ux, bim, acc[0].y)))};
  acc[1] = cd{fma(a.x, qy.x, fma(-a.y, qy.y, fma(uy, bre, acc[1].x))),
              fma(a.x, qy.y, fma(a.y, qy.x, fma(uy, bim, acc[1].y)))};
  acc[2] = cd{fma(a.x, qz.x, fma(-a.y, qz.y, fma(uz, bre, acc[2].x))),
              fma(a.x, qz.y, fma(a.y, qz.x, fma(uz, bim, acc[2].y)))};
}

// ------------------------------------------------------------------ P2P
// free-space near field: A_i += sum_j G^f(x_i - x_j) J_j over same-layer
// sources in adjacent leaves, coincident points skipped (paper Sec. 2 and the
// layered sums of Sec. 3.3)
template <int RC, bool RED>
__global__ __launch_bounds__(NT) void k_p2p(DevPlan d, const int* tboxes, int n_items, const double* sxyz,
                                            const cd* J, long long n_src, const double* txyz, long long n_tgt,
                                            int n_rhs, cd* A) {
  __shared__ double sp[NT][3];
  __shared__ cd sj[NT][RC][3];
  const int ny = (n_rhs + RC - 1) / RC, total = n_items * ny;
  __shared__ int wq_s;
  WorkQueue wq{d.wq + LM_WQ_P2P, &wq_s};
  for (int wi = wq.next(); wi < total; wi = wq.next()) {
  const int bx = wi / ny, by = wi - bx * ny;
  // work item: (target leaf, chunk of NT targets); the wavenumber is that of
  // the leaf's instance (its layer)
  int b = tboxes[2 * bx];
  TgtBox tb = d.tbox[b];
  const double k = d.inst[__builtin_amdgcn_readfirstlane(tb.inst)].kt;
  int r0 = by * RC, nr = min(RC, n_rhs - r0);
  int tid = threadIdx.x;
  const double inv4pi = 0.079577471545947667884;
  const double invk = 1.0 / k;
  {
    int t0 = tb.pt0 + tboxes[2 * bx + 1] * NT;
    int ti = t0 + tid;
    bool act = ti < tb.pt1;
    int id = act ? d.tgt_perm[ti] : 0;
    double x0 = act ? txyz[3 * id] : 0, y0 = act ? txyz[3 * id + 1] : 0, z0 = act ? txyz[3 * id + 2] : 0;
    cd acc[RC][3];
    for (int rr = 0; rr < RC; rr++)
      for (int c = 0; c < 3; c++) acc[rr][c] = cd{0, 0};
    for (int li = tb.p2p0; li < tb.p2p1; li++) {
      SrcBox sb = d.sbox[d.p2p_list[li]];
      for (int s0 = sb.pt0; s0 < sb.pt1; s0 += NT) {
        int ns = min(NT, sb.pt1 - s0);
        __syncthreads();
        if (tid < ns) {
          int sid = d.src_perm[s0 + tid];
          sp[tid][0] = sxyz[3 * sid];
          sp[tid][1] = sxyz[3 * sid + 1];
          sp[tid][2] = sxyz[3 * sid + 2];
          for (int rr = 0; rr < RC; rr++)
            for (int c = 0; c < 3; c++)
              sj[tid][rr][c] = rr < nr ? J[((long long)(r0 + rr) * n_src + sid) * 3 + c] : cd{0, 0};
        }
        __syncthreads();
        if (act) {
          // the coincident point (r = 0) is skipped without a branch: 1/r is
          // set to 0, so that g and every term vanish; the loop body then
          // has no data-dependent control flow and is unrolled
#pragma unroll 4
          for (int j = 0; j < ns; j++) {
            double rx = x0 - sp[j][0], ry = y0 - sp[j][1], rz = z0 - sp[j][2];
            double r2 = rx * rx + ry * ry + rz * rz;
            double ir = r2 > 0.0 ? lm_rsqrt(r2) : 0.0, r = r2 * ir;
            double kr = k * r, ikr = invk * ir, ikr2 = ikr * ikr;
            double sn, cs;
            lm_sincos_nf<RED>(kr, &sn, &cs);
            cd g = cd{cs * inv4pi * ir, sn * inv4pi * ir};
            cd a = g * cd{1.0 - ikr2, ikr};
            cd bq = g * cd{-1.0 + 3.0 * ikr2, -3.0 * ikr};
            double ux = rx * ir, uy = ry * ir, uz = rz * ir;
            for (int rr = 0; rr < RC; rr++) p2p_apply(acc[rr], a, bq, ux, uy, uz, sj[j][rr][0], sj[j][rr][1], sj[j][rr][2]);
          }
        }
      }
    }
    if (act)
      for (int rr = 0; rr < nr; rr++) {
        cd* Ap = A + ((long long)(r0 + rr) * n_tgt + id) * 3;
        for (int c = 0; c < 3; c++) Ap[c] = Ap[c] + acc[rr][c];
      }
  }
  }
  wq.leave();
}
void launch_p2p(const DevPlan& d, const int* tboxes, int n, const double* sxyz, const cd* J, long long n_src,
                const double* txyz, long long n_tgt, int n_rhs, cd* A, bool red, hipStream_t s) {
  if (n <= 0) return;
#define LM_P2P_GO(RC, RED)                                                                                     \
  do {                                                                                                         \
    const void* f = (const void*)k_p2p<RC, RED>;                                                               \
    const int g = persistent_grid(f, NT, 0, (long long)n * ((n_rhs + RC - 1) / RC));                           \
    hipLaunchKernelGGL((k_p2p<RC, RED>), dim3(g), dim3(NT), 0, s, d, tboxes, n, sxyz, J, n_src, txyz, n_tgt,   \
                       n_rhs, A);                                                                              \
  } while (0)
  if (n_rhs == 1) {
    if (red)
      LM_P2P_GO(1, true);
    else
      LM_P2P_GO(1, false);
  } else {
    if (red)
      LM_P2P_GO(4, true);
    else
      LM_P2P_GO(4, false);
  }
#undef LM_P2P_GO
}

// Symmetric free-space near field, for builds whose targets are the
// sources: G^f(x_i - x_j) = G^f(x_j - x_i) (a symmetric dyadic of r), so one
// evaluation of the kernel per unordered pair serves both ends.  A work
// item is (leaf, chunk of NT points): its points interact with their own
// leaf as in k_p2p (every ordered pair, the coincident one skipped) and
// with the adjacent leaves of higher source-box id (the partners), whose
// points receive G J_i back.  Per partner, 64 points at a time: each wave
// holds 64 of the item's points (one per lane) and runs a systolic cycle of
// 64 steps: at step s lane l pairs its point with partner point
// (l - s) mod 64, adds G J_j to its own sum and G J_i to that partner
// point's sum for the wave (in LDS; the 64 lanes of a step touch 64
// different points).  The four waves' sums are added in wave order and written to the item's output slot
// for that point; k_s2t_gather adds each point's slots in item order after
// the item's own sums went into A.  Deterministic, no atomics; one
// right-hand side per block (blockIdx.y).
template <bool RED>
__global__ __launch_bounds__(NT, RED ? 3 : 2) void k_p2p_sym(DevPlan d, const int* items, int n_items, const int* part,
                                                const double* xyz, const cd* J, long long n_pts, int n_rhs, cd* A,
                                                cd* Ys) {
  __shared__ double sp[NT][3];
  __shared__ cd sj[NT][3];
  __shared__ double qx[64], qy[64], qz[64], qj[6][64];  // one block of 64 partner points
  __shared__ cd tw[NT / 64][64][3];                    // per wave: sums for the partner points
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int total = n_items * n_rhs;
  __shared__ int wq_s;
  WorkQueue wq{d.wq + LM_WQ_P2PS, &wq_s};
  for (int wi = wq.next(); wi < total; wi = wq.next()) {
  const int bx = wi / n_rhs;
  // item: (target leaf, chunk, first output slot, partner range, own source box)
  const int* it = items + 6 * bx;
  const int b = __builtin_amdgcn_readfirstlane(it[0]);
  const int chunk = __builtin_amdgcn_readfirstlane(it[1]);
  const long long slot0 = __builtin_amdgcn_readfirstlane(it[2]);
  const int p0 = __builtin_amdgcn_readfirstlane(it[3]), p1 = __builtin_amdgcn_readfirstlane(it[4]);
  const int self = __builtin_amdgcn_readfirstlane(it[5]);
  const TgtBox tb = d.tbox[b];
  const double k = d.inst[__builtin_amdgcn_readfirstlane(tb.inst)].kt;
  const int r = wi - bx * n_rhs;
  const cd* Jr = J + (long long)r * n_pts * 3;
  const double inv4pi = 0.079577471545947667884;
  const double invk = 1.0 / k;
  const int ti = tb.pt0 + chunk * NT + tid;
  const bool act = ti < tb.pt1;
  // lanes past the chunk take the leaf's first point with no current: every
  // lane runs the systolic cycle, their terms vanish
  const int id = d.tgt_perm[act ? ti : tb.pt0];
  const double x0 = xyz[3 * id], y0 = xyz[3 * id + 1], z0 = xyz[3 * id + 2];
  cd ji[3];
  for (int c = 0; c < 3; c++) ji[c] = act ? Jr[(long long)id * 3 + c] : cd{0, 0};
  cd acc[3] = {cd{0, 0}, cd{0, 0}, cd{0, 0}};
  // pair kernel: a = g (1 - 1/(kr)^2 + i/(kr)), b = g (-1 + 3/(kr)^2 - 3i/(kr)),
  // g = e^{ikr} / (4 pi r), unit vector u; r = 0 gives 1/r = 0 and no term
  auto kern = [&](double rx, double ry, double rz, cd& a, cd& bq, double& ux, double& uy, double& uz) {
    const double r2 = rx * rx + ry * ry + rz * rz;
    const double ir = r2 > 0.0 ? lm_rsqrt(r2) : 0.0, rr = r2 * ir;
    const double kr = k * rr, ikr = invk * ir, ikr2 = ikr * ikr;
    double sn, cs;
    lm_sincos_nf<RED>(kr, &sn, &cs);
    const cd g = cd{cs * inv4pi * ir, sn * inv4pi * ir};
    a = g * cd{1.0 - ikr2, ikr};
    bq = g * cd{-1.0 + 3.0 * ikr2, -3.0 * ikr};
    ux = rx * ir;
    uy = ry * ir;
    uz = rz * ir;
  };
  {
    // own leaf: every ordered pair
    const SrcBox sb = d.sbox[self];
    for (int s0 = sb.pt0; s0 < sb.pt1; s0 += NT) {
      const int ns = min(NT, sb.pt1 - s0);
      __syncthreads();
      if (tid < ns) {
        const int sid = d.src_perm[s0 + tid];
        sp[tid][0] = xyz[3 * sid];
        sp[tid][1] = xyz[3 * sid + 1];
        sp[tid][2] = xyz[3 * sid + 2];
        for (int c = 0; c < 3; c++) sj[tid][c] = Jr[(long long)sid * 3 + c];
      }
      __syncthreads();
      if (act) {
#pragma unroll 4
        for (int j = 0; j < ns; j++) {
          cd a, bq;
          double ux, uy, uz;
          kern(x0 - sp[j][0], y0 - sp[j][1], z0 - sp[j][2], a, bq, ux, uy, uz);
          p2p_apply(acc, a, bq, ux, uy, uz, sj[j][0], sj[j][1], sj[j][2]);
        }
      }
    }
  }
  // waves with points of the chunk (the others skip the partner cycles)
  const int nchunk = min(NT, tb.pt1 - (tb.pt0 + chunk * NT));
  const int nwav = (nchunk + 63) >> 6;
  const bool wact = wave < nwav;
  long long so = slot0;
  for (int pi = p0; pi < p1; pi++) {
    const SrcBox sb = d.sbox[part[pi]];
    for (int s0 = sb.pt0; s0 < sb.pt1; s0 += 64) {
      const int nb = min(64, sb.pt1 - s0);
      __syncthreads();
      if (tid < 64) {
        const bool ok = tid < nb;
        const int sid = d.src_perm[ok ? s0 + tid : sb.pt0];
        qx[tid] = xyz[3 * sid];
        qy[tid] = xyz[3 * sid + 1];
        qz[tid] = xyz[3 * sid + 2];
        for (int c = 0; c < 3; c++) {
          const cd v = ok ? Jr[(long long)sid * 3 + c] : cd{0, 0};
          qj[2 * c][tid] = v.x;
          qj[2 * c + 1][tid] = v.y;
        }
      }
      __syncthreads();
      // partner sums of this wave in LDS: at step s lane l adds to point
      // (l - s) mod 64, so the 64 lanes touch 64 different points and each
      // point receives its terms in step order (the wave's LDS operations
      // complete in issue order, so step s + 1 reads what step s wrote)
      // waves holding none of the chunk's points (short leaves) add nothing
      if (wact) {
      for (int c = 0; c < 3; c++) tw[wave][lane][c] = cd{0, 0};
      for (int st = 0; st < 64; st++) {
        const int j = (lane - st) & 63;
        cd a, bq;
        double ux, uy, uz;
        kern(x0 - qx[j], y0 - qy[j], z0 - qz[j], a, bq, ux, uy, uz);
        p2p_apply(acc, a, bq, ux, uy, uz, cd{qj[0][j], qj[1][j]}, cd{qj[2][j], qj[3][j]}, cd{qj[4][j], qj[5][j]});
        // the same kernel at the partner point: G(x_j - x_i) = G(x_i - x_j)
        cd t[3] = {tw[wave][j][0], tw[wave][j][1], tw[wave][j][2]};
        p2p_apply(t, a, bq, ux, uy, uz, ji[0], ji[1], ji[2]);
        tw[wave][j][0] = t[0];
        tw[wave][j][1] = t[1];
        tw[wave][j][2] = t[2];
      }
      }
      __syncthreads();
      if (tid < nb) {
        cd u[3] = {tw[0][tid][0], tw[0][tid][1], tw[0][tid][2]};
        for (int w = 1; w < nwav; w++)
          for (int c = 0; c < 3; c++) u[c] = u[c] + tw[w][tid][c];
        cd* Yp = Ys + ((so + (s0 - sb.pt0) + tid) * n_rhs + r) * 3;
        for (int c = 0; c < 3; c++) Yp[c] = u[c];
      }
    }
    so += sb.pt1 - sb.pt0;
  }
  if (act) {
    cd* Ap = A + ((long long)r * n_pts + id) * 3;
    for (int c = 0; c < 3; c++) Ap[c] = Ap[c] + acc[c];
  }
  }
  wq.leave();
}
void launch_p2p_sym(const DevPlan& d, const int* items, int n, const int* part, const double* xyz, const cd* J,
                    long long n_pts, int n_rhs, cd* A, cd* Ys, bool red, hipStream_t s) {
  if (n <= 0) return;
  const void* f = red ? (const void*)k_p2p_sym<true> : (const void*)k_p2p_sym<false>;
  const int g = persistent_grid(f, NT, 0, (long long)n * n_rhs);
  if (red)
    hipLaunchKernelGGL(k_p2p_sym<true>, dim3(g), dim3(NT), 0, s, d, items, n, part, xyz, J, n_pts, n_rhs, A, Ys);
  else
    hipLaunchKernelGGL(k_p2p_sym<false>, dim3(g), dim3(NT), 0, s, d, items, n, part, xyz, J, n_pts, n_rhs, A, Ys);
}

// ------------------------------------------------------------------ octrees
// The records of every octree of a plan (paper Sec. 3.3: one tree per
// layer's free-space part and per reaction component, over images and
// effective locations), keyed and sorted on the device in one batch: a
// record is (Morton key of its lattice cell, point id | tag << 31, tree);
// an LSD radix sort with 8-bit digits orders them by key (eight passes)
// and then by tree (one pass per byte of the tree count), every pass stable,
// so that each tree's records end up contiguous, in key order, equal keys
// in input order -- the order of the host planner's own sort; then the
// trees' boxes are formed from the sorted keys (k_tree_box_count / emit).

// Morton code of a lattice cell: bits of ux, uy, uz interleaved from the
// lowest (x at bit 3b, y at 3b + 1, z at 3b + 2).
__device__ __forceinline__ uint64_t tree_spread3(uint64_t v) {
  v &= 0xFFFFF;
  v = (v | (v << 32)) & 0x1F00000000FFFFull;
  v = (v | (v << 16)) & 0x1F0000FF0000FFull;
  v = (v | (v << 8)) & 0x100F00F00F00F00Full;
  v = (v | (v << 4)) & 0x10C30C30C30C30C3ull;
  v = (v | (v << 2)) & 0x1249249249249249ull;
  return v;
}
struct TreeSegDev {
  long long r0;   // first record of the segment
  long long ids;  // first id of the segment in the uploaded id lists
  int n, tgt, tag, tree;
  double za, zb;
};
struct TreeLatDev {
  double x0, y0, z0, inv;  // inv = 2^DK / S0
};
__global__ void k_tree_keys(const TreeSegDev* segs, int nseg, const TreeLatDev* lat, const int* ids,
                            const double* sxyz, const double* txyz, long long n, uint64_t* key, uint32_t* pay,
                            int* tree) {
  const long long st = (long long)gridDim.x * blockDim.x;
  for (long long r = (long long)blockIdx.x * blockDim.x + threadIdx.x; r < n; r += st) {
    // the segment holding record r (segments in record order)
    int lo = 0, hi = nseg - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (segs[mid].r0 <= r)
        lo = mid;
      else
        hi = mid - 1;
    }
    const TreeSegDev sg = segs[lo];
    const TreeLatDev L = lat[sg.tree];
    const int id = ids[sg.ids + (r - sg.r0)];
    const double* x = (sg.tgt ? txyz : sxyz) + 3 * (long long)id;
    // the same operations, in the same order and rounding, as the host's
    // (a product and a sum, not fused)
    const double z = __dadd_rn(__dmul_rn(sg.za, x[2]), sg.zb);
    const long long mx = (1LL << LM_TREE_DK) - 1;
    long long u[3] = {(long long)floor((x[0] - L.x0) * L.inv), (long long)floor((x[1] - L.y0) * L.inv),
                      (long long)floor((z - L.z0) * L.inv)};
    for (int a = 0; a < 3; a++) u[a] = u[a] < 0 ? 0 : (u[a] > mx ? mx : u[a]);
    key[r] = tree_spread3((uint64_t)u[0]) | (tree_spread3((uint64_t)u[1]) << 1) | (tree_spread3((uint64_t)u[2]) << 2);
    pay[r] = (uint32_t)id | ((uint32_t)sg.tag << 31);
    tree[r] = sg.tree;
  }
}

#define RS_NT 256                 // threads per radix block
#define RS_ITEMS 8                // records per thread
#define RS_TILE (RS_NT * RS_ITEMS)  // records per block
__device__ __forceinline__ int rs_digit(int pass, uint64_t key, int tree) {
  return pass < 8 ? (int)((key >> (8 * pass)) & 255) : ((tree >> (8 * (pass - 8))) & 255);
}
// per block: how many of its records hold each digit, at cnt[d * nblk + b]
__global__ __launch_bounds__(RS_NT) void k_rs_hist(const uint64_t* key, const int* tree, long long n, int pass,
                                                   int* cnt, int nblk) {
  __shared__ int h[256];
  const int tid = threadIdx.x;
  h[tid] = 0;
  __syncthreads();
  const long long t0 = (long long)blockIdx.x * RS_TILE;
  for (int k = 0; k < RS_ITEMS; k++) {
    const long long r = t0 + k * RS_NT + tid;
    if (r < n) atomicAdd(&h[rs_digit(pass, key[r], tree[r])], 1);
  }
  __syncthreads();
  cnt[(long long)tid * nblk + blockIdx.x] = h[tid];
}
// stable scatter: a record goes to the start of its digit in its block
// (exclusive scan of cnt) plus the number of earlier records of the block
// with the same digit.  Records are taken in RS_ITEMS rounds of RS_NT in
// index order; in a round, the lanes of a wave with equal digits find each
// other by eight ballots (one per digit bit), the waves' counts per digit
// are added in wave order, and a running count per digit carries over the
// rounds.
__global__ __launch_bounds__(RS_NT) void k_rs_scatter(const uint64_t* key, const uint32_t* pay, const int* tree,
                                                      uint64_t* key2, uint32_t* pay2, int* tree2, long long n,
                                                      int pass, const int* off, int nblk) {
  __shared__ int base[256], run[256], wc[RS_NT / 64][256];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  base[tid] = off[(long long)tid * nblk + blockIdx.x];
  run[tid] = 0;
  const long long t0 = (long long)blockIdx.x * RS_TILE;
  const uint64_t below = lane == 0 ? 0ull : (~0ull >> (64 - lane));
  for (int k = 0; k < RS_ITEMS; k++) {
    for (int w = 0; w < RS_NT / 64; w++) wc[w][tid] = 0;
    __syncthreads();
    const long long r = t0 + k * RS_NT + tid;
    const bool ok = r < n;
    uint64_t kv = 0;
    uint32_t pv = 0;
    int tv = 0, d = 0;
    if (ok) {
      kv = key[r];
      pv = pay[r];
      tv = tree[r];
      d = rs_digit(pass, kv, tv);
    }
    uint64_t peers = __ballot(ok);
    for (int b = 0; b < 8; b++) {
      const bool bit = (d >> b) & 1;
      const uint64_t m = __ballot(ok && bit);
      peers &= bit ? m : ~m;
    }
    const int rank = __popcll(peers & below);
    if (ok && rank == 0) wc[wave][d] = __popcll(peers);
    __syncthreads();
    if (ok) {
      int pos = base[d] + run[d] + rank;
      for (int w = 0; w < wave; w++) pos += wc[w][d];
      key2[pos] = kv;
      pay2[pos] = pv;
      tree2[pos] = tv;
    }
    __syncthreads();
    int add = 0;
    for (int w = 0; w < RS_NT / 64; w++) add += wc[w][tid];
    run[tid] += add;
  }
}
// exclusive scan of a[0..m) in tiles of RS_TILE (each tile's total to sums)
__global__ __launch_bounds__(RS_NT) void k_scan_tiles(int* a, long long m, int* sums) {
  __shared__ int sh[RS_NT];
  const int tid = threadIdx.x;
  const long long e0 = (long long)blockIdx.x * RS_TILE + (long long)tid * RS_ITEMS;
  int v[RS_ITEMS], tot = 0;
  for (int k = 0; k < RS_ITEMS; k++) {
    v[k] = e0 + k < m ? a[e0 + k] : 0;
    tot += v[k];
  }
  sh[tid] = tot;
  __syncthreads();
  for (int o = 1; o < RS_NT; o <<= 1) {
    const int x = tid >= o ? sh[tid - o] : 0;
    __syncthreads();
    sh[tid] += x;
    __syncthreads();
  }
  int acc = sh[tid] - tot;  // exclusive prefix of this thread's items
  for (int k = 0; k < RS_ITEMS; k++) {
    if (e0 + k < m) a[e0 + k] = acc;
    acc += v[k];
  }
  if (tid == RS_NT - 1) sums[blockIdx.x] = sh[tid];
}
__global__ void k_scan_add(int* a, long long m, const int* sums) {
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < m) a[e] += sums[e / RS_TILE];
}
// exclusive scan of a[0..m) on the device; scratch holds the tile sums of
// every level (at least m / RS_TILE + 2 entries per level, levels in turn)
static void scan_excl(int* a, long long m, int* scratch, hipStream_t s) {
  const long long nt = (m + RS_TILE - 1) / RS_TILE;
  if (nt <= 0) return;
  hipLaunchKernelGGL(k_scan_tiles, dim3((unsigned)nt), dim3(RS_NT), 0, s, a, m, scratch);
  if (nt > 1) {
    scan_excl(scratch, nt, scratch + nt, s);
    hipLaunchKernelGGL(k_scan_add, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, s, a, m, (const int*)scratch);
  }
}

// The boxes of the sorted trees.  A record lies in a box at every level up
// to its depth: a free-space tree's depth, or, with gap_only, the first
// level whose box has a nonzero gap index (its boxes below that are not
// split), capped at the depth; and it is the first record of its box at
// level l when l is at least the first level at which its key's prefix
// differs from the previous record's (every level for a tree's first
// record).  k_tree_box_count counts the boxes each record starts; after a
// scan k_tree_box_emit writes them, (level << 40) | record, in record and
// level order.
struct TreeRuleDev {
  long long r0;  // first record of the tree in the sorted output
  int depth, gap_only, zflip;
};
__device__ __forceinline__ int tree_z_at(uint64_t key, int l) {
  // the z cell index at level l: bits 3b + 2 of the key's top l levels
  int iz = 0;
  for (int b = LM_TREE_DK - l; b < LM_TREE_DK; b++) iz |= (int)((key >> (3 * b + 2)) & 1) << (b - (LM_TREE_DK - l));
  return iz;
}
__device__ __forceinline__ void tree_box_range(const uint64_t* key, const int* tree, const TreeRuleDev* rule,
                                               long long u, int* lo, int* hi) {
  const TreeRuleDev R = rule[tree[u]];
  int depth = R.depth;
  if (R.gap_only) {
    int dd = 0;
    while (dd < R.depth) {
      const int iz = tree_z_at(key[u], dd);
      const int j = R.zflip ? ((1 << dd) - 1 - iz) : iz;
      if (j != 0) break;
      dd++;
    }
    depth = dd;
  }
  int first = 0;
  if (u > R.r0) {
    const uint64_t x = key[u] ^ key[u - 1];
    if (x == 0) {
      first = LM_TREE_DK + 1;
    } else {
      const int b = 63 - __clzll((long long)x);  // highest differing bit
      first = LM_TREE_DK - b / 3;
    }
  }
  *lo = first;
  *hi = depth;
}
__global__ void k_tree_box_count(const uint64_t* key, const int* tree, const TreeRuleDev* rule, long long n,
                                 int* cnt) {
  const long long st = (long long)gridDim.x * blockDim.x;
  for (long long u = (long long)blockIdx.x * blockDim.x + threadIdx.x; u < n; u += st) {
    int lo, hi;
    tree_box_range(key, tree, rule, u, &lo, &hi);
    cnt[u] = hi >= lo ? hi - lo + 1 : 0;
    if (u == 0) cnt[n] = 0;  // the scan's total lands here
  }
}
__global__ void k_tree_box_emit(const uint64_t* key, const int* tree, const TreeRuleDev* rule, long long n,
                                const int* off, uint64_t* out) {
  const long long st = (long long)gridDim.x * blockDim.x;
  for (long long u = (long long)blockIdx.x * blockDim.x + threadIdx.x; u < n; u += st) {
    int lo, hi;
    tree_box_range(key, tree, rule, u, &lo, &hi);
    for (int l = lo; l <= hi; l++) out[off[u] + (l - lo)] = ((uint64_t)l << 40) | (uint64_t)u;
  }
}

std::string lm_device_tree_sort(const std::vector<TreeJob>& jobs, const std::vector<TreeSeg>& segs,
                                const double* d_src, const double* d_tgt, std::vector<uint64_t>& keys,
                                std::vector<uint32_t>& pay, std::vector<uint64_t>& boxes, float* ms,
                                hipStream_t s) {
  // segments in record order; each distinct host id list uploaded once
  std::vector<TreeSegDev> sd;
  std::vector<TreeLatDev> ld;
  std::vector<int> ids;
  std::vector<std::pair<const int*, long long>> seen;  // (list, its offset in ids)
  long long n = 0;
  for (size_t t = 0; t < jobs.size(); t++) {
    const TreeJob& J = jobs[t];
    ld.push_back(TreeLatDev{J.x0, J.y0, J.z0, (double)(1 << LM_TREE_DK) / J.S0});
    for (int q = 0; q < J.nseg; q++) {
      const TreeSeg& g = segs[J.seg0 + q];
      if (g.n <= 0) continue;
      long long io = -1;
      for (auto& e : seen)
        if (e.first == g.ids) io = e.second;
      if (io < 0) {
        io = (long long)ids.size();
        seen.push_back({g.ids, io});
        ids.insert(ids.end(), g.ids, g.ids + g.n);
      }
      sd.push_back(TreeSegDev{n, io, g.n, g.tgt, g.tag, (int)t, g.za, g.zb});
      n += g.n;
    }
  }
  keys.assign((size_t)n, 0);
  pay.assign((size_t)n, 0);
  boxes.clear();
  if (ms) *ms = 0;
  if (n == 0) return "";
  std::vector<TreeRuleDev> rd(jobs.size());
  {
    long long r = 0;
    for (size_t t = 0; t < jobs.size(); t++) {
      rd[t] = TreeRuleDev{r, jobs[t].depth, jobs[t].gap_only, jobs[t].zflip};
      for (int q = 0; q < jobs[t].nseg; q++) r += segs[jobs[t].seg0 + q].n > 0 ? segs[jobs[t].seg0 + q].n : 0;
    }
  }
  if (n > 0x7fffffffLL) return "tree sort: too many records";
  const int nblk = (int)((n + RS_TILE - 1) / RS_TILE);
  const long long m = 256LL * nblk;
  long long nscr = 0;
  for (long long mm = std::max<long long>(m, n + 1); mm > 1; mm = (mm + RS_TILE - 1) / RS_TILE)
    nscr += (mm + RS_TILE - 1) / RS_TILE + 2;
  std::vector<void*> bufs;
  bool alloc_ok = true;
  auto dmal = [&](size_t bytes) -> void* {
    void* p = nullptr;
    if (hipMalloc(&p, bytes) != hipSuccess || !p) {
      alloc_ok = false;
      return nullptr;
    }
    bufs.push_back(p);
    return p;
  };
  auto done = [&](const std::string& e) {
    for (void* p : bufs) (void)hipFree(p);
    return e;
  };
  TreeSegDev* d_sd = (TreeSegDev*)dmal(sd.size() * sizeof(TreeSegDev));
  TreeLatDev* d_ld = (TreeLatDev*)dmal(ld.size() * sizeof(TreeLatDev));
  int* d_ids = (int*)dmal(ids.size() * sizeof(int));
  uint64_t* k0 = (uint64_t*)dmal((size_t)n * 8);
  uint64_t* k1 = (uint64_t*)dmal((size_t)n * 8);
  uint32_t* p0 = (uint32_t*)dmal((size_t)n * 4);
  uint32_t* p1 = (uint32_t*)dmal((size_t)n * 4);
  int* t0 = (int*)dmal((size_t)n * 4);
  int* t1 = (int*)dmal((size_t)n * 4);
  int* cnt = (int*)dmal((size_t)std::max<long long>(m, n + 1) * 4);
  int* scr = (int*)dmal((size_t)(nscr + 2) * 4);
  TreeRuleDev* d_rd = (TreeRuleDev*)dmal(rd.size() * sizeof(TreeRuleDev));
  if (!alloc_ok) return done("tree sort: device allocation failed");
  if (hipMemcpy(d_sd, sd.data(), sd.size() * sizeof(TreeSegDev), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(d_ld, ld.data(), ld.size() * sizeof(TreeLatDev), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(d_ids, ids.data(), ids.size() * sizeof(int), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(d_rd, rd.data(), rd.size() * sizeof(TreeRuleDev), hipMemcpyHostToDevice) != hipSuccess)
    return done("tree sort: upload failed");
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (ms) {
    (void)hipEventCreate(&e0);
    (void)hipEventCreate(&e1);
    (void)hipEventRecord(e0, s);
  }
  const long long gk = std::min<long long>((n + 255) / 256, 65536);
  hipLaunchKernelGGL(k_tree_keys, dim3((unsigned)gk), dim3(256), 0, s, (const TreeSegDev*)d_sd, (int)sd.size(),
                     (const TreeLatDev*)d_ld, (const int*)d_ids, d_src, d_tgt, n, k0, p0, t0);
  int npass = 8;
  for (size_t nt = jobs.size() - 1; nt > 0; nt >>= 8) npass++;
  for (int pass = 0; pass < npass; pass++) {
    hipLaunchKernelGGL(k_rs_hist, dim3(nblk), dim3(RS_NT), 0, s, (const uint64_t*)k0, (const int*)t0, n, pass, cnt,
                       nblk);
    scan_excl(cnt, m, scr, s);
    hipLaunchKernelGGL(k_rs_scatter, dim3(nblk), dim3(RS_NT), 0, s, (const uint64_t*)k0, (const uint32_t*)p0,
                       (const int*)t0, k1, p1, t1, n, pass, (const int*)cnt, nblk);
    std::swap(k0, k1);
    std::swap(p0, p1);
    std::swap(t0, t1);
  }
  // (the time reported is that of the keys and the sort)
  if (ms) (void)hipEventRecord(e1, s);
  auto drop_events = [&]() {
    if (!ms) return;
    (void)hipEventSynchronize(e1);
    (void)hipEventElapsedTime(ms, e0, e1);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
  };
  // the boxes: per record the count of boxes it starts, their offsets (an
  // exclusive scan over n + 1 entries gives the total last), the entries
  const long long gb = std::min<long long>((n + 255) / 256, 65536);
  hipLaunchKernelGGL(k_tree_box_count, dim3((unsigned)gb), dim3(256), 0, s, (const uint64_t*)k0, (const int*)t0,
                     (const TreeRuleDev*)d_rd, n, cnt);
  scan_excl(cnt, n + 1, scr, s);
  int nbox = 0;
  if (hipMemcpyAsync(&nbox, cnt + n, sizeof(int), hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess) {
    drop_events();
    return done("tree sort: box count download failed");
  }
  uint64_t* d_box = nbox > 0 ? (uint64_t*)dmal((size_t)nbox * 8) : nullptr;
  if (!alloc_ok) {
    drop_events();
    return done("tree sort: device allocation failed");
  }
  if (nbox > 0)
    hipLaunchKernelGGL(k_tree_box_emit, dim3((unsigned)gb), dim3(256), 0, s, (const uint64_t*)k0, (const int*)t0,
                       (const TreeRuleDev*)d_rd, n, (const int*)cnt, d_box);
  drop_events();
  hipError_t err = hipGetLastError();
  if (err != hipSuccess) return done(std::string("tree sort: ") + hipGetErrorString(err));
  boxes.assign((size_t)nbox, 0);
  if (hipMemcpyAsync(keys.data(), k0, (size_t)n * 8, hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipMemcpyAsync(pay.data(), p0, (size_t)n * 4, hipMemcpyDeviceToHost, s) != hipSuccess ||
      (nbox > 0 && hipMemcpyAsync(boxes.data(), d_box, (size_t)nbox * 8, hipMemcpyDeviceToHost, s) != hipSuccess) ||
      hipStreamSynchronize(s) != hipSuccess)
    return done("tree sort: download failed");
  return done("");
}

// ------------------------------------------------------------------ self-test
// out[4 i .. 4 i + 3] = (sin, cos) by the near-field routine (library beyond
// its range), then
// 1/sqrt(x_i^2 + 1e-300) by the refined estimate, then by the library.
// J0 and J1 of a real argument x >= 0, ix = 1 / x (read only from
// LM_BPQ_X0 up): fixed-degree polynomials, so every lane of a wave runs the
// same steps.  Below LM_BPQ_X0 the power series S(w) in w = x^2 / 4 and
// J1 = -(x/2) S'(w); above, the Hankel modulus/phase form with P and Q / t as
// polynomials in u = t^2, t = X0 / x, and J1 = -J0' from their derivatives
// (coefficients and their accuracy: gen_bessel_pq.py).  The coefficients are
// read through an offset the compiler cannot fold, so that they are loaded
// per call instead of being held in registers across the caller's loop.
__constant__ double c_bpq[LM_BPQ_N] = {LM_BPQ_COEFFS};
// a b + c with c a wave-uniform value read from scalar registers (the
// three-operand form; the compiler otherwise copies c to vector registers
// for the two-address form, two moves per coefficient)
__device__ __forceinline__ double fma_s(double a, double b, double c) {
  double r;
  asm("v_fma_f64 %0, %1, %2, %3" : "=v"(r) : "v"(a), "v"(b), "s"(c));
  return r;
}
__device__ inline void bessel01_real(double x, double ix, double* j0v, double* j1v) {
  int z = 0;
  asm volatile("" : "+s"(z));
  const double* c = c_bpq + z;
  if (x < LM_BPQ_X0) {
    const double w = 0.25 * x * x;
    double b = c[LM_BPQ_NSER - 1], d = 0.0;
#pragma unroll
    for (int k = LM_BPQ_NSER - 2; k >= 0; k--) {
      d = fma(d, w, b);
      b = fma_s(b, w, c[k]);
    }
    *j0v = b;
    *j1v = -0.5 * x * d;
    return;
  }
  const double* cp = c + LM_BPQ_NSERC;
  const double* cq = cp + LM_BPQ_DEG + 1;
  const double t = LM_BPQ_X0 * ix, u = t * t;
  double P = cp[LM_BPQ_DEG], dP = 0.0, Qt = cq[LM_BPQ_DEG], dQt = 0.0;
#pragma unroll
  for (int k = LM_BPQ_DEG - 1; k >= 0; k--) {
    dP = fma(dP, u, P);
    P = fma_s(P, u, cp[k]);
    dQt = fma(dQt, u, Qt);
    Qt = fma_s(Qt, u, cq[k]);
  }
  const double Q = t * Qt;
  const double dPx = -2.0 * u * ix * dP;                // dP / dx
  const double dQx = -(t * ix) * fma(2.0 * u, dQt, Qt);  // dQ / dx
  double sn, cs;
  lm_sincos_red(x - 0.78539816339744830962, &sn, &cs);  // chi = x - pi/4
  const double A = sqrt(0.63661977236758134308 * ix);   // sqrt(2 / (pi x))
  const double j0 = A * (P * cs - Q * sn);
  *j0v = j0;
  // J1 = -J0' = J0 / (2x) + A ((Q - P') cos chi + (P + Q') sin chi)
  *j1v = 0.5 * ix * j0 + A * ((Q - dPx) * cs + (P + dQx) * sn);
}

// J0, J1, J2 of a complex argument by the power series S(w) = sum_k
// (-w)^k / (k!)^2, w = z^2 / 4, with n terms: J0 = S, J1 = -J0' =
// -(z/2) S'(w) and J2 = J0'' - J0'/z = w S''(w) (Bessel's equation), from one
// pass of Horner's rule carrying both derivatives: no division, exact at
// z = 0.  Coefficients as in bessel01_real (n <= LM_BPQ_NSERC).
__device__ inline void bessel012_horner(cd z, int n, cd* j0, cd* j1, cd* j2) {
  const cd w = 0.25 * (z * z);
  int zo = 0;
  asm volatile("" : "+s"(zo));
  const double* c = c_bpq + zo;
  cd v = cd{c[n - 1], 0.0}, d1 = cd{0, 0}, d2 = cd{0, 0};
  for (int k = n - 2; k >= 0; k--) {
    d2 = d2 * w + d1;
    d1 = d1 * w + v;
    v = cd{fma(v.x, w.x, fma_s(-v.y, w.y, c[k])), fma(v.x, w.y, v.y * w.x)};
  }
  *j0 = v;
  *j1 = -0.5 * (z * d1);
  *j2 = 2.0 * (w * d2);
}

// J0 and J1 alone: the same pass without the second derivative (the direct
// pairs take J2 from the recurrence), every complex product written out with
// explicit multiply-adds.
__device__ inline void bessel01_horner(cd z, int n, cd* j0, cd* j1) {
  const cd zz = cmul_exact(z, z);
  const cd w = cd{0.25 * zz.x, 0.25 * zz.y};
  int zo = 0;
  asm volatile("" : "+s"(zo));
  const double* c = c_bpq + zo;
  cd v = cd{c[n - 1], 0.0}, d1 = cd{0, 0};
  for (int k = n - 2; k >= 0; k--) {
    d1 = cd{fma(d1.x, w.x, fma(-d1.y, w.y, v.x)), fma(d1.x, w.y, fma(d1.y, w.x, v.y))};
    v = cd{fma(v.x, w.x, fma_s(-v.y, w.y, c[k])), fma(v.x, w.y, v.y * w.x)};
  }
  *j0 = v;
  const cd zd = cmul_exact(z, d1);
  *j1 = cd{-0.5 * zd.x, -0.5 * zd.y};
}

__global__ void k_selftest_math(const double* x, long long n, double* out) {
  long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double sn, cs;
  if (fabs(x[i]) < LM_SINCOS_RED_MAX)
    lm_sincos_red(x[i], &sn, &cs);
  else
    sincos(x[i], &sn, &cs);
  double a = x[i] * x[i] + 1e-300;
  double ax = fabs(x[i]), j0, j1;
  bessel01_real(ax, ax > 0 ? 1.0 / ax : 0.0, &j0, &j1);
  out[6 * i] = sn;
  out[6 * i + 1] = cs;
  out[6 * i + 2] = lm_rsqrt(a);
  out[6 * i + 3] = 1.0 / sqrt(a);
  out[6 * i + 4] = j0;
  out[6 * i + 5] = j1;
}
void launch_selftest_math(const double* x, long long n, double* out, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_selftest_math, dim3((unsigned)((n + NT - 1) / NT)), dim3(NT), 0, s, x, n, out);
}

// ------------------------------------------------------------------ gradients
// Source-position gradients use reciprocity, G(x, y) = G(y, x)^T (the
// reciprocity of the layered Green's function, Sec. 3.3): with the currents
// conj(gA) placed at the targets, the field B(y) = sum_i G(y, x_i) conj(gA_i)
// is evaluated with its gradient at the source points and contracted with
// the source currents,  gX_j = Re sum_b J_j^b grad B_b(x_j).  The kernels
// below evaluate that contraction for the far field (from the local
// expansions) and for the free-space near field.  Each point is owned by one
// thread of one block per launch, and right-hand sides are taken in order,
// so the accumulation into gX is deterministic.

// out = conj(in)
__global__ void k_conj(cd* out, const cd* in, long long n) {
  long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  long long st = (long long)gridDim.x * blockDim.x;
  for (; i < n; i += st) out[i] = cconj(in[i]);
}
__device__ inline double mu_pow(const MediumDev& md, double z, int pw) {
  int l = 0;
  while (l < md.n - 1 && z < md.d[l]) l++;
  return pw > 0 ? md.mu[l] : 1.0 / md.mu[l];
}
__global__ void k_conj_mu(cd* out, const cd* in, long long n, long long total, const double* xyz, MediumDev md,
                          int pw) {
  long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  long long st = (long long)gridDim.x * blockDim.x;
  for (; e < total; e += st) {
    const long long i = (e / 3) % n;
    out[e] = cconj(in[e]) * mu_pow(md, xyz[3 * i + 2], pw);
  }
}
void launch_conj_mu(cd* out, const cd* in, long long n, int n_rhs, const double* xyz, MediumDev md, int pw,
                    hipStream_t s) {
  const long long total = 3 * n * n_rhs;
  if (total <= 0) return;
  long long nb = std::min<long long>((total + NT - 1) / NT, 65536);
  hipLaunchKernelGGL(k_conj_mu, dim3((unsigned)nb), dim3(NT), 0, s, out, in, n, total, xyz, md, pw);
}
__global__ void k_scale_mu(cd* v, long long n, long long total, const double* xyz, MediumDev md, int pw) {
  long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  long long st = (long long)gridDim.x * blockDim.x;
  for (; e < total; e += st) {
    const long long i = (e / 3) % n;
    v[e] = v[e] * mu_pow(md, xyz[3 * i + 2], pw);
  }
}
void launch_scale_mu(cd* v, long long n, int n_rhs, const double* xyz, MediumDev md, int pw, hipStream_t s) {
  const long long total = 3 * n * n_rhs;
  if (total <= 0) return;
  long long nb = std::min<long long>((total + NT - 1) / NT, 65536);
  hipLaunchKernelGGL(k_scale_mu, dim3((unsigned)nb), dim3(NT), 0, s, v, n, total, xyz, md, pw);
}
__global__ void k_scale_mu_d(double* g, long long n, const double* xyz, MediumDev md, int pw) {
  long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  long long st = (long long)gridDim.x * blockDim.x;
  for (; i < n; i += st) {
    const double f = mu_pow(md, xyz[3 * i + 2], pw);
    for (int c = 0; c < 3; c++) g[3 * i + c] *= f;
  }
}
void launch_scale_mu_d(double* g, long long n, const double* xyz, MediumDev md, int pw, hipStream_t s) {
  if (n <= 0) return;
  long long nb = std::min<long long>((n + NT - 1) / NT, 65536);
  hipLaunchKernelGGL(k_scale_mu_d, dim3((unsigned)nb), dim3(NT), 0, s, g, n, xyz, md, pw);
}
__global__ void k_fill_d(double* p, long long n) {
  long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  long long st = (long long)gridDim.x * blockDim.x;
  for (; i < n; i += st) p[i] = 0.0;
}
void launch_fill_d(double* p, long long n, hipStream_t s) {
  if (n <= 0) return;
  long long nb = std::min<long long>((n + NT - 1) / NT, 65536);
  hipLaunchKernelGGL(k_fill_d, dim3((unsigned)nb), dim3(NT), 0, s, p, n);
}
void launch_conj(cd* out, const cd* in, long long n, hipStream_t s) {
  if (n <= 0) return;
  long long nb = std::min<long long>((n + NT - 1) / NT, 65536);
  hipLaunchKernelGGL(k_conj, dim3((unsigned)nb), dim3(NT), 0, s, out, in, n);
}

// Far field: the local expansion (3 spin channels) is turned into the
// expansion of the field (free space: U + grad div U / k^2, order p + 2;
// reaction: the LE itself, order p), then the three derivatives
// (d/dx + i d/dy, d/dx - i d/dy, d/dz, exact ladder relations of the regular
// wave functions) give 9 expansions of one order more, evaluated at every
// point of the leaf.  For a reaction component the evaluation point is the
// effective location zhat = at z + bt, so d/dz = at d/dzhat.
// CURL: instead of contracting the derivatives with W into gX, the curl of
// the field is added to Hc [rhs][point][3] (the magnetic field's far part,
// Faraday's law, before the 1/mu of the point's layer).
template <int NTB, bool CURL>
__global__ __launch_bounds__(NTB) void k_l2p_grad(DevPlan d, const int* leaves, int ch, int kind, const double* xyz,
                                                  long long n_pts, int n_rhs, const cd* LE, const cd* W,
                                                  double* gX, cd* Hc) {
  extern __shared__ cd Ls[];
  // work item: (leaf, chunk of ch points)
  int b = leaves[2 * blockIdx.x];
  const int q0 = d.tbox[b].pt0 + leaves[2 * blockIdx.x + 1] * ch;
  TgtBox tb = d.tbox[b];
  InstParams ip = d.inst[tb.inst];
  int p = ip.p, P = ip.P;
  int pa = (kind == 0) ? p + 2 : p;  // order of the field expansion
  int pg = pa + 1, Pg = (pg + 1) * (pg + 1);
  int Pd = (p + 2) * (p + 2);
  int tid = threadIdx.x;
  double k = ip.kt;
  cd* Lc = Ls;            // [3][Pg]   field expansion (order pa)
  cd* Dv = Ls + 3 * Pg;   // [Pd]      k x divergence (free space)
  cd* Gc = Dv + Pd;       // [9][Pg]   (channel, direction) derivative expansions
  for (int r = 0; r < n_rhs; r++) {
    __syncthreads();
    for (int e = tid; e < 3 * Pg; e += NTB) {
      int c = e / Pg, nm = e - c * Pg;
      Lc[e] = nm < P ? LE[tb.le_off * n_rhs + ((long long)r * 3 + c) * P + nm] : cd{0, 0};
    }
    __syncthreads();
    if (kind == 0) {
      for (int nm = tid; nm < Pd; nm += NTB) {
        int n = n_of(nm), m = nm - n * n - n;
        cd v = 0.5 * (dapply(Lc + Pg, p, 0, n, m) + dapply(Lc, p, 1, n, m)) + dapply(Lc + 2 * Pg, p, 2, n, m);
        Dv[nm] = k * v;
      }
      __syncthreads();
      int Pa = (pa + 1) * (pa + 1);
      for (int e = tid; e < 3 * Pa; e += NTB) {
        int c = e / Pa, nm = e - c * Pa;
        int n = n_of(nm), m = nm - n * n - n;
        Lc[c * Pg + nm] = Lc[c * Pg + nm] + (1.0 / k) * dapply(Dv, p + 1, c, n, m);
      }
      __syncthreads();
    }
    for (int e = tid; e < 9 * Pg; e += NTB) {
      int cd_ = e / Pg, nm = e - cd_ * Pg;
      int c = cd_ / 3, dir = cd_ - 3 * c;
      int n = n_of(nm), m = nm - n * n - n;
      Gc[e] = dapply(Lc + c * Pg, pa, dir, n, m);
    }
    __syncthreads();
    const int q1 = min(tb.pt1, q0 + ch);
    for (int t0 = q0; t0 < q1; t0 += NTB) {
      int ti = t0 + tid;
      if (ti >= q1) continue;
      int id = d.tgt_perm[ti];
      double dx = xyz[3 * id] - tb.c[0], dy = xyz[3 * id + 1] - tb.c[1];
      double dz = ip.at * xyz[3 * id + 2] + ip.bt - tb.c[2];
      double rxy = sqrt(dx * dx + dy * dy), rr_ = sqrt(dx * dx + dy * dy + dz * dz);
      double ct = rr_ > 0 ? dz / rr_ : 1.0, st = rr_ > 0 ? rxy / rr_ : 0.0;
      cd e1 = rxy > 0 ? cd{dx / rxy, dy / rxy} : cd{1.0, 0.0};
      double* jn = (double*)(Gc + 9 * Pg) + tid * (pg + 1);
      sph_jn(pg, k * rr_, jn);
      cd acc[9];
      for (int q = 0; q < 9; q++) acc[q] = cd{0, 0};
      double pmm = LM_INV_SQRT_4PI;
      cd em = cd{1.0, 0.0};
      for (int m = 0; m <= pg; m++) {
        if (m > 0) {
          pmm = c_leg_mm[m] * st * pmm;
          em = em * e1;
        }
        double p2 = 0.0, p1 = pmm;
        for (int n = m; n <= pg; n++) {
          double pn;
          if (n == m)
            pn = pmm;
          else if (n == m + 1)
            pn = c_leg_m1[m] * ct * pmm;
          else
            pn = c_leg_a[n * LEGN + m] * (ct * p1 - c_leg_b[n * LEGN + m] * p2);
          if (n > m) {
            p2 = p1;
            p1 = pn;
          }
          double rad = jn[n] * pn;
          cd bp = rad * em;
          cd bm = ((m & 1) ? -rad : rad) * cconj(em);
          int ip_ = nm_idx(n, m), im_ = nm_idx(n, -m);
          for (int q = 0; q < 9; q++) {
            acc[q] = acc[q] + Gc[q * Pg + ip_] * bp;
            if (m > 0) acc[q] = acc[q] + Gc[q * Pg + im_] * bm;
          }
        }
      }
      // derivatives of the spin channels: D+ = d/dx + i d/dy, D- = d/dx - i d/dy
      // (both times 1/k in acc), d/dz (times 1/k, in zhat)
      cd dB[3][3];  // [cartesian direction][spin channel]
      for (int c = 0; c < 3; c++) {
        cd dp = k * acc[c * 3 + 0], dm = k * acc[c * 3 + 1], dzv = (k * ip.at) * acc[c * 3 + 2];
        dB[0][c] = 0.5 * (dp + dm);
        cd h = 0.5 * (dp - dm);
        dB[1][c] = cd{h.y, -h.x};  // (dp - dm) / (2i)
        dB[2][c] = dzv;
      }
      cd jac[3][3];  // [direction][cartesian field component]
      for (int a = 0; a < 3; a++) {
        // cartesian field components from the spin channels
        jac[a][0] = 0.5 * (dB[a][0] + dB[a][1]);
        cd h = 0.5 * (dB[a][0] - dB[a][1]);
        jac[a][1] = cd{h.y, -h.x};
        jac[a][2] = dB[a][2];
      }
      if (CURL) {
        cd* o = Hc + ((long long)r * n_pts + id) * 3;
        o[0] = o[0] + (jac[1][2] - jac[2][1]);
        o[1] = o[1] + (jac[2][0] - jac[0][2]);
        o[2] = o[2] + (jac[0][1] - jac[1][0]);
      } else {
        const cd* w = W + ((long long)r * n_pts + id) * 3;
        cd wx = w[0], wy = w[1], wz = w[2];
        for (int a = 0; a < 3; a++) {
          cd v = wx * jac[a][0] + wy * jac[a][1] + wz * jac[a][2];
          gX[3 * id + a] += v.x;
        }
      }
    }
  }
}
template <int NTB, bool CURL>
static void l2p_grad_go(const DevPlan& d, const int* leaves, int n, int kind, const double* xyz, long long n_pts,
                        int n_rhs, const cd* LE, const cd* W, double* gX, cd* Hc, int pi, hipStream_t s) {
  int pg = (kind == 0 ? pi + 2 : pi) + 1;
  int Pg = (pg + 1) * (pg + 1), Pd = (pi + 2) * (pi + 2);
  size_t shm = (size_t)(12 * Pg + Pd) * sizeof(cd) + (size_t)NTB * (pg + 1) * sizeof(double);
  set_dyn_lds((const void*)k_l2p_grad<NTB, CURL>, shm);
  hipLaunchKernelGGL((k_l2p_grad<NTB, CURL>), dim3(n), dim3(NTB), shm, s, d, leaves, LM_L2P_CHUNK(kind), kind, xyz,
                     n_pts, n_rhs, LE, W, gX, Hc);
}
// pi: the instance's expansion order; reaction items with one-wave blocks,
// free-space items with 128 threads (LDS of order p + 3 expansions)
void launch_l2p_grad(const DevPlan& d, const int* leaves, int n, int kind, const double* xyz, long long n_pts,
                     int n_rhs, const cd* LE, const cd* W, double* gX, int pi, hipStream_t s) {
  if (n <= 0) return;
  if (kind == 1)
    l2p_grad_go<64, false>(d, leaves, n, kind, xyz, n_pts, n_rhs, LE, W, gX, nullptr, pi, s);
  else
    l2p_grad_go<128, false>(d, leaves, n, kind, xyz, n_pts, n_rhs, LE, W, gX, nullptr, pi, s);
}
void launch_l2p_curl(const DevPlan& d, const int* leaves, int n, int kind, const double* xyz, long long n_pts,
                     int n_rhs, const cd* LE, cd* Hc, int pi, hipStream_t s) {
  if (n <= 0) return;
  if (kind == 1)
    l2p_grad_go<64, true>(d, leaves, n, kind, xyz, n_pts, n_rhs, LE, nullptr, nullptr, Hc, pi, s);
  else
    l2p_grad_go<128, true>(d, leaves, n, kind, xyz, n_pts, n_rhs, LE, nullptr, nullptr, Hc, pi, s);
}

// Free-space near field: for the target point x_i (here a source point of
// the original problem, weights w = its currents) and near sources x_j with
// currents s_j:  G_bc(R) = a(r) delta_bc + b(r) u_b u_c, R = x_i - x_j,
// u = R / r, and
//   sum_bc w_b d_alpha G_bc s_c = u_alpha [a' (w.s) + (b' - 2 b / r)(w.u)(u.s)]
//                                  + (b / r) [w_alpha (u.s) + s_alpha (w.u)].
template <bool RED>
__global__ __launch_bounds__(NT) void k_p2p_grad(DevPlan d, const int* tboxes, const double* sxyz, const cd* Jsrc,
                                                 long long n_src, const double* txyz, const cd* W,
                                                 long long n_tgt, int n_rhs, double* gX) {
  __shared__ double sp[NT][3];
  __shared__ cd sj[NT][3];
  // work item: (target leaf, chunk of NT targets); wavenumber of its instance
  int b = tboxes[2 * blockIdx.x];
  TgtBox tb = d.tbox[b];
  const double k = d.inst[__builtin_amdgcn_readfirstlane(tb.inst)].kt;
  int tid = threadIdx.x;
  const double inv4pi = 0.079577471545947667884;
  const double invk = 1.0 / k;
  for (int r = 0; r < n_rhs; r++) {
    {
      int t0 = tb.pt0 + tboxes[2 * blockIdx.x + 1] * NT;
      int ti = t0 + tid;
      bool act = ti < tb.pt1;
      int id = act ? d.tgt_perm[ti] : 0;
      double x0 = act ? txyz[3 * id] : 0, y0 = act ? txyz[3 * id + 1] : 0, z0 = act ? txyz[3 * id + 2] : 0;
      cd wx = cd{0, 0}, wy = cd{0, 0}, wz = cd{0, 0};
      if (act) {
        const cd* w = W + ((long long)r * n_tgt + id) * 3;
        wx = w[0];
        wy = w[1];
        wz = w[2];
      }
      double g0 = 0, g1 = 0, g2 = 0;
      for (int li = tb.p2p0; li < tb.p2p1; li++) {
        SrcBox sb = d.sbox[d.p2p_list[li]];
        for (int s0 = sb.pt0; s0 < sb.pt1; s0 += NT) {
          int ns = min(NT, sb.pt1 - s0);
          __syncthreads();
          if (tid < ns) {
            int sid = d.src_perm[s0 + tid];
            sp[tid][0] = sxyz[3 * sid];
            sp[tid][1] = sxyz[3 * sid + 1];
            sp[tid][2] = sxyz[3 * sid + 2];
            for (int c = 0; c < 3; c++) sj[tid][c] = Jsrc[((long long)r * n_src + sid) * 3 + c];
          }
          __syncthreads();
          if (act) {
            for (int j = 0; j < ns; j++) {
              double rx = x0 - sp[j][0], ry = y0 - sp[j][1], rz = z0 - sp[j][2];
              double r2 = rx * rx + ry * ry + rz * rz;
              if (r2 == 0.0) continue;
              double ir = lm_rsqrt(r2), rd = r2 * ir;
              double kr = k * rd, ikr = invk * ir, ikr2 = ikr * ikr, ikr3 = ikr2 * ikr;
              double sn, cs;
              lm_sincos_nf<RED>(kr, &sn, &cs);
              cd g = cd{cs * inv4pi * ir, sn * inv4pi * ir};
              cd gp = g * cd{-ir, k};                          // g' = g (ik - 1/r)
              cd fa = cd{1.0 - ikr2, ikr}, fb = cd{-1.0 + 3.0 * ikr2, -3.0 * ikr};
              cd dfa = k * cd{2.0 * ikr3, -ikr2};              // d fa / dr
              cd dfb = k * cd{-6.0 * ikr3, 3.0 * ikr2};        // d fb / dr
              cd bq = g * fb;
              cd ap = gp * fa + g * dfa, bp = gp * fb + g * dfb;
              double ux = rx * ir, uy = ry * ir, uz = rz * ir;
              cd sx = sj[j][0], sy = sj[j][1], sz = sj[j][2];
              cd ws = wx * sx + wy * sy + wz * sz;
              cd wu = ux * wx + uy * wy + uz * wz;
              cd us = ux * sx + uy * sy + uz * sz;
              cd radial = ap * ws + (bp - (2.0 * ir) * bq) * (wu * us);
              cd br = ir * bq;
              cd v0 = ux * radial + br * (wx * us + sx * wu);
              cd v1 = uy * radial + br * (wy * us + sy * wu);
              cd v2 = uz * radial + br * (wz * us + sz * wu);
              g0 += v0.x;
              g1 += v1.x;
              g2 += v2.x;
            }
          }
        }
      }
      if (act) {
        gX[3 * id] += g0;
        gX[3 * id + 1] += g1;
        gX[3 * id + 2] += g2;
      }
    }
  }
}
void launch_p2p_grad(const DevPlan& d, const int* tboxes, int n, const double* sxyz, const cd* Jsrc,
                     long long n_src, const double* txyz, const cd* W, long long n_tgt, int n_rhs, double* gX,
                     bool red, hipStream_t s) {
  if (n <= 0) return;
  if (red)
    hipLaunchKernelGGL(k_p2p_grad<true>, dim3(n), dim3(NT), 0, s, d, tboxes, sxyz, Jsrc, n_src, txyz, W, n_tgt, n_rhs,
                       gX);
  else
    hipLaunchKernelGGL(k_p2p_grad<false>, dim3(n), dim3(NT), 0, s, d, tboxes, sxyz, Jsrc, n_src, txyz, W, n_tgt,
                       n_rhs, gX);
}

// Free-space near field of the magnetic field (Faraday's law): the curl of
// the free dyadic's field is grad g x q (the grad grad / k^2 part has no
// curl), with grad g = g (ik - 1/r) R / r, R = x_i - x_j; coincident points
// are skipped as in the electric near field.  Added to Hc [rhs][point][3].
template <bool RED>
__global__ __launch_bounds__(NT) void k_p2p_curl(DevPlan d, const int* tboxes, const double* sxyz, const cd* J,
                                                 long long n_src, const double* txyz, long long n_tgt, int n_rhs,
                                                 cd* Hc) {
  __shared__ double sp[NT][3];
  __shared__ cd sj[NT][3];
  int b = tboxes[2 * blockIdx.x];
  TgtBox tb = d.tbox[b];
  const double k = d.inst[__builtin_amdgcn_readfirstlane(tb.inst)].kt;
  const int tid = threadIdx.x;
  const double inv4pi = 0.079577471545947667884;
  for (int r = 0; r < n_rhs; r++) {
    int ti = tb.pt0 + tboxes[2 * blockIdx.x + 1] * NT + tid;
    bool act = ti < tb.pt1;
    int id = act ? d.tgt_perm[ti] : 0;
    double x0 = act ? txyz[3 * id] : 0, y0 = act ? txyz[3 * id + 1] : 0, z0 = act ? txyz[3 * id + 2] : 0;
    cd h0 = cd{0, 0}, h1 = cd{0, 0}, h2 = cd{0, 0};
    for (int li = tb.p2p0; li < tb.p2p1; li++) {
      SrcBox sb = d.sbox[d.p2p_list[li]];
      for (int s0 = sb.pt0; s0 < sb.pt1; s0 += NT) {
        int ns = min(NT, sb.pt1 - s0);
        __syncthreads();
        if (tid < ns) {
          int sid = d.src_perm[s0 + tid];
          sp[tid][0] = sxyz[3 * sid];
          sp[tid][1] = sxyz[3 * sid + 1];
          sp[tid][2] = sxyz[3 * sid + 2];
          for (int c = 0; c < 3; c++) sj[tid][c] = J[((long long)r * n_src + sid) * 3 + c];
        }
        __syncthreads();
        if (act) {
          for (int j = 0; j < ns; j++) {
            double rx = x0 - sp[j][0], ry = y0 - sp[j][1], rz = z0 - sp[j][2];
            double r2 = rx * rx + ry * ry + rz * rz;
            if (r2 == 0.0) continue;
            double ir = lm_rsqrt(r2), rd = r2 * ir;
            double sn, cs;
            lm_sincos_nf<RED>(k * rd, &sn, &cs);
            cd g = cd{cs * inv4pi * ir, sn * inv4pi * ir};
            cd gr = (g * cd{-ir, k}) * ir;  // g' / r
            cd gx = rx * gr, gy = ry * gr, gz = rz * gr;
            cd qx = sj[j][0], qy = sj[j][1], qz = sj[j][2];
            h0 = h0 + (gy * qz - gz * qy);
            h1 = h1 + (gz * qx - gx * qz);
            h2 = h2 + (gx * qy - gy * qx);
          }
        }
      }
    }
    if (act) {
      cd* o = Hc + ((long long)r * n_tgt + id) * 3;
      o[0] = o[0] + h0;
      o[1] = o[1] + h1;
      o[2] = o[2] + h2;
    }
  }
}
void launch_p2p_curl(const DevPlan& d, const int* tboxes, int n, const double* sxyz, const cd* J, long long n_src,
                     const double* txyz, long long n_tgt, int n_rhs, cd* Hc, bool red, hipStream_t s) {
  if (n <= 0) return;
  if (red)
    hipLaunchKernelGGL(k_p2p_curl<true>, dim3(n), dim3(NT), 0, s, d, tboxes, sxyz, J, n_src, txyz, n_tgt, n_rhs, Hc);
  else
    hipLaunchKernelGGL(k_p2p_curl<false>, dim3(n), dim3(NT), 0, s, d, tboxes, sxyz, J, n_src, txyz, n_tgt, n_rhs,
                       Hc);
}

// ------------------------------------------------------------------ S2T
// Reaction near field of one component between adjacent leaves next to the
// gap (Sec. 3.3: the component's Sommerfeld integral evaluated directly).
// For a target x and a source x' (horizontal offset rho at angle phi):
//   I_sigma,|kappa| = sum_nodes w kr Z F_sigma J_|kappa|(kr rho),
//   Z = exp(i (k_z t(z) + k'_z u(z'))),
//   W(kappa, sigma) = e^{i kappa phi} i^{1+|kappa|} I_sigma,|kappa|,
// combined in the spin basis exactly as the M2L tensor (the order-0 case of
// P2M -> M2L -> L2P at the pair itself, hence the factor 1/(4 pi)):
//   out+ = W(0,s1) u+/2 - W(2,s3) u-/2 + W(1,s2) m_z
//   out- = W(0,s1) u-/2 - W(-2,s3) u+/2 + W(-1,s2) m_z
//   out_z = W(1,s4) u-/2 + W(-1,s4) u+/2 + W(0,s5) m_z.
// The nodes are Gamma_1 (complex k_rho) then the real tail in increasing
// order; each pair stops at its own cut a + LM_S2T_DIGITS / (t + u).  Each
// target is owned by one thread of one work item and the launches go
// component by component, so the accumulation into A is deterministic.
// One work item: a chunk of up to 64 targets of a reaction leaf against the
// sources of all its near boxes, taken as one concatenated list (segments of
// up to LM_S2T_SEG boxes).  Pair q = i ns + j (target i, source j of the
// segment) is one lane per round of 64 pairs; each lane loads its own source
// and runs the node loop of the component's Sommerfeld integrals (Gamma_1,
// then the real tail up to its own cut).  Nodes are staged through LDS 64 at
// a time and read in a wave-uniform loop.  A target adds its pairs in q order
// (no atomics).  The integrals depend on the pair only: a block applies them
// to RS right-hand sides (blockIdx.y: the group of RS).
// HF: the curl of the field instead (mu_t times the magnetic field, the
// J6..J9 form, with the node densities FH in the same five slots):
//   out+ as above, out- negated, out_z = W(-1,s4) u+/2 - W(1,s4) u-/2.
template <bool SMALLZ, int RS, bool HF>
__global__ __launch_bounds__(LM_S2T_CHUNK, 2) void k_s2t(DevPlan d, MediumDev md, const int* items, int n_items,
                                                                     const int* tlist, const int* slist,
                                                                     const double* sxyz, const cd* J,
                                                                     long long n_src, const double* txyz,
                                                                     long long n_tgt, int n_rhs, double a,
                                                                     cd* Ys) {
  __shared__ double tp[LM_S2T_CHUNK][3];  // targets: x, y, t
  __shared__ cd res[LM_S2T_CHUNK][RS][3];  // per pair of the round and rhs: out+, out-, out_z
  __shared__ cd nk[LM_S2T_CHUNK][10];     // node chunk: kr, w, kz_t, kz_s, F_1..F_5, 1 / kr (tail)
  const int tid = threadIdx.x;
  const int ny = (n_rhs + RS - 1) / RS, total = n_items * ny;
  __shared__ int wq_s;
  WorkQueue wq{d.wq + LM_WQ_S2T, &wq_s};
  for (int wi = wq.next(); wi < total; wi = wq.next()) {
  const int bx = wi / ny, by = wi - bx * ny;
  // work item, component and node range are uniform over the block
  const int* it6 = items + 6 * bx;
  const int b = __builtin_amdgcn_readfirstlane(it6[0]);
  const int chunk = __builtin_amdgcn_readfirstlane(it6[1]);
  const long long slot0 = __builtin_amdgcn_readfirstlane(it6[2]);
  const int* tl = tlist + __builtin_amdgcn_readfirstlane(it6[3]);  // chunk positions, sorted by t
  const int* sl = slist + __builtin_amdgcn_readfirstlane(it6[4]);  // near source points, sorted by u
  const int ns = __builtin_amdgcn_readfirstlane(it6[5]);
  const TgtBox tb = d.tbox[b];
  const InstParams ip = d.inst[__builtin_amdgcn_readfirstlane(tb.inst)];
  const int r0 = by * RS, nr = min(RS, n_rhs - r0);
  const int t0 = tb.pt0 + chunk * LM_S2T_CHUNK;
  const int nt = min(LM_S2T_CHUNK, tb.pt1 - t0);
  const int n0 = __builtin_amdgcn_readfirstlane(ip.s2t0), nn = __builtin_amdgcn_readfirstlane(ip.s2tn);
  const int nser = __builtin_amdgcn_readfirstlane(ip.s2t_nser);
  const QNode* nodes = d.nodes + n0;
  const double dls = ip.up_s ? md.d[ip.ls - 1] : md.d[ip.ls];
  // lane tid owns the target at chunk position pos (targets in increasing
  // t, sources in increasing u: neighbouring pairs of a round then have
  // similar cuts, so that few lanes idle on the real tail)
  int pos = 0;
  if (tid < nt) {
    pos = tl[tid];
    const int id = d.tgt_perm[t0 + pos];
    double zt = txyz[3 * id + 2];
    tp[tid][0] = txyz[3 * id];
    tp[tid][1] = txyz[3 * id + 1];
    tp[tid][2] = ip.up_t ? zt - md.d[ip.lt] : md.d[ip.lt - 1] - zt;
  }
  __syncthreads();
  cd op[RS], om[RS], oz[RS];  // thread tid < nt: totals of target tid
  for (int rr = 0; rr < RS; rr++) op[rr] = om[rr] = oz[rr] = cd{0, 0};
  {
    const int npair = nt * ns;
    for (int q0 = 0; q0 < npair; q0 += LM_S2T_CHUNK) {
      const int q = q0 + tid;
      const bool pa = q < npair;
      const int i = pa ? q / ns : 0, j = pa ? q - (q / ns) * ns : 0;
      const int sid = sl[j];
      const double* sx = sxyz + 3 * (long long)sid;
      double dx = tp[i][0] - sx[0], dy = tp[i][1] - sx[1];
      double tz = tp[i][2], uz = ip.up_s ? dls - sx[2] : sx[2] - dls;
      double rho = sqrt(dx * dx + dy * dy);
      const double irho = rho > 0 ? 1.0 / rho : 0.0;
      double cph = rho > 0 ? dx * irho : 1.0, sph = rho > 0 ? dy * irho : 0.0;
      // each pair's cut on the real tail; inactive lanes need no node
      double kcut = pa ? a + LM_S2T_DIGITS / (tz + uz) : -1.0;
      cd I1 = cd{0, 0}, I2 = cd{0, 0}, I3 = cd{0, 0}, I4 = cd{0, 0}, I5 = cd{0, 0};
      for (int c0 = 0; c0 < nn; c0 += LM_S2T_CHUNK) {
        const int nc = min(LM_S2T_CHUNK, nn - c0);
        __syncthreads();
        if (tid < nc) {
          const QNode& nd = nodes[c0 + tid];
          nk[tid][0] = nd.kr;
          nk[tid][1] = nd.w * nd.kr;
          nk[tid][2] = nd.kzt;
          nk[tid][3] = nd.kzs;
          for (int f = 0; f < 5; f++) nk[tid][4 + f] = HF ? nd.FH[f] : nd.F[f];
          // 1 / k_rho (real on the tail)
          const double ik2 = 1.0 / (nd.kr.x * nd.kr.x + nd.kr.y * nd.kr.y);
          nk[tid][9] = nd.kr.y == 0.0 ? cd{1.0 / nd.kr.x, 0.0} : cd{nd.kr.x * ik2, -nd.kr.y * ik2};
        }
        __syncthreads();
        for (int m = 0; m < nc; m++) {
          const cd kr = nk[m][0];
          if (kr.y != 0.0) {  // Gamma_1 (complex k_rho): every active pair
            if (!pa) continue;
            // w k_rho exp(i (t k_z + u k_z')); the phase is small (|k_z| (t + u)).
            // Products written out with explicit multiply-adds here and below:
            // every instantiation (right-hand sides per block) rounds alike
            const cd kzt = nk[m][2], kzs = nk[m][3];
            const double ez_re = -fma(tz, kzt.y, uz * kzs.y), ez_im = fma(tz, kzt.x, uz * kzs.x);
            double esn, ecs;
            lm_sincos_red(ez_im, &esn, &ecs);
            const double ea = exp(ez_re);
            const cd base = cmul_exact(nk[m][1], cd{ea * ecs, ea * esn});
            cd jb[3];
            if (SMALLZ) {
              // J0, J1 by the series; J2 = 2 J1 / z - J0 (1/z = (1/k_rho)(1/rho)),
              // or its series z^2/8 (1 - z^2/12) near 0 (explicit multiply-adds)
              const cd z = cd{rho * kr.x, rho * kr.y};
              bessel01_horner(z, nser, jb, jb + 1);
              if (fma(z.x, z.x, z.y * z.y) > 1e-6) {
                const cd t = cmul_exact(jb[1], cd{irho * nk[m][9].x, irho * nk[m][9].y});
                jb[2] = cd{fma(2.0, t.x, -jb[0].x), fma(2.0, t.y, -jb[0].y)};
              } else {
                const cd z2 = cmul_exact(z, z);
                const cd q = cmul_exact(z2, cd{fma(z2.x, -1.0 / 12.0, 1.0), z2.y * (-1.0 / 12.0)});
                jb[2] = cd{0.125 * q.x, 0.125 * q.y};
              }
            } else {
              bessel_jq(2, rho * kr, jb);
            }
            const cd b0 = cmul_exact(base, jb[0]), b1 = cmul_exact(base, jb[1]), b2 = cmul_exact(base, jb[2]);
            I1 = cmac_exact(I1, b0, nk[m][4]);
            I2 = cmac_exact(I2, b1, nk[m][5]);
            I3 = cmac_exact(I3, b2, nk[m][6]);
            I4 = cmac_exact(I4, b1, nk[m][7]);
            I5 = cmac_exact(I5, b0, nk[m][8]);
          } else if (kr.x <= kcut) {
            // real tail: k_z = i |k_z|, Z = exp(-t |k_z| - u |k_z'|)
            double z = exp(-fma(tz, nk[m][2].y, uz * nk[m][3].y));
            double base = nk[m][1].x * z;
            const double x = kr.x * rho, ix = nk[m][9].x * irho;
            double J0, J1;
            bessel01_real(x, ix, &J0, &J1);
            // J2 = 2 J1 / x - J0; its series x^2/8 - x^4/96 near 0
            double J2 = x > 1e-3 ? 2.0 * J1 * ix - J0 : x * x * (0.125 - x * x * (1.0 / 96.0));
            double b0 = base * J0, b1 = base * J1, b2 = base * J2;
            I1 = I1 + b0 * nk[m][4];
            I2 = I2 + b1 * nk[m][5];
            I3 = I3 + b2 * nk[m][6];
            I4 = I4 + b1 * nk[m][7];
            I5 = I5 + b0 * nk[m][8];
          }
        }
        // stop once the next chunk starts on the tail beyond every pair's cut
        bool more = false;
        if (c0 + nc < nn) {
          const cd kn = nodes[c0 + nc].kr;
          more = kn.y != 0.0 || kn.x <= kcut;
        }
        if (!__syncthreads_or(more)) break;
      }
      if (pa) {
        // written out with explicit fma and contraction off: the same
        // rounding whatever the number of right-hand sides a block serves (a
        // column of a batch equals its single-vector evaluation bitwise)
#pragma clang fp contract(off)
        auto cm = [](cd u, cd v) { return cd{fma(u.x, v.x, -(u.y * v.y)), fma(u.x, v.y, u.y * v.x)}; };
        const cd e1 = cd{cph, sph}, e1c = cd{cph, -sph};
        const cd e2 = cm(e1, e1), e2c = cd{e2.x, -e2.y};
        const cd W01 = cd{-I1.y, I1.x};  // i I1
        const cd W05 = cd{-I5.y, I5.x};  // i I5
        const cd t3 = cd{I3.y, -I3.x};   // -i I3
        const cd W2p = cm(e2, t3), W2m = cm(e2c, t3);
        const cd P2 = cm(e1, I2), M2 = cm(e1c, I2), P4 = cm(e1, I4), M4 = cm(e1c, I4);
        const cd W1p2 = cd{-P2.x, -P2.y}, W1m2 = cd{-M2.x, -M2.y};
        const cd W1p4 = cd{-P4.x, -P4.y}, W1m4 = cd{-M4.x, -M4.y};
        for (int rr = 0; rr < RS; rr++) {
          cd rp = cd{0, 0}, rm = cd{0, 0}, rz = cd{0, 0};
          if (rr < nr) {
            const cd* Jp = J + ((long long)(r0 + rr) * n_src + sid) * 3;
            const cd jx = Jp[0], jy = Jp[1], jz = Jp[2];
            const cd up = cd{jx.x - jy.y, jx.y + jy.x}, um = cd{jx.x + jy.y, jx.y - jy.x};
            const cd a1 = cm(W01, up), a2 = cm(W2p, um), a3 = cm(W1p2, jz);
            const cd b1 = cm(W01, um), b2 = cm(W2m, up), b3 = cm(W1m2, jz);
            const cd c1 = cm(W1p4, um), c2 = cm(W1m4, up), c3 = cm(W05, jz);
            rp = cd{(0.5 * a1.x - 0.5 * a2.x) + a3.x, (0.5 * a1.y - 0.5 * a2.y) + a3.y};
            if (HF) {
              rm = cd{(0.5 * b2.x - 0.5 * b1.x) - b3.x, (0.5 * b2.y - 0.5 * b1.y) - b3.y};
              rz = cd{0.5 * c2.x - 0.5 * c1.x, 0.5 * c2.y - 0.5 * c1.y};
            } else {
              rm = cd{(0.5 * b1.x - 0.5 * b2.x) + b3.x, (0.5 * b1.y - 0.5 * b2.y) + b3.y};
              rz = cd{(0.5 * c1.x + 0.5 * c2.x) + c3.x, (0.5 * c1.y + 0.5 * c2.y) + c3.y};
            }
          }
          res[tid][rr][0] = rp;
          res[tid][rr][1] = rm;
          res[tid][rr][2] = rz;
        }
      } else {
        for (int rr = 0; rr < RS; rr++) res[tid][rr][0] = res[tid][rr][1] = res[tid][rr][2] = cd{0, 0};
      }
      __syncthreads();
      // target tid adds its pairs of this round in source order
      if (tid < nt) {
        int qa = max(q0, tid * ns), qb = min(q0 + LM_S2T_CHUNK, (tid + 1) * ns);
        for (int qq = qa; qq < qb; qq++)
          for (int rr = 0; rr < RS; rr++) {
            op[rr] = op[rr] + res[qq - q0][rr][0];
            om[rr] = om[rr] + res[qq - q0][rr][1];
            oz[rr] = oz[rr] + res[qq - q0][rr][2];
          }
      }
      __syncthreads();
    }
  }
  if (tid < nt) {
    // this target's totals go to its slot; k_s2t_gather adds the slots of a
    // point in a fixed order
#pragma clang fp contract(off)
    const double f = 0.079577471545947667884;  // 1 / (4 pi)
#pragma unroll
    for (int rr = 0; rr < RS; rr++) {
      if (rr >= nr) break;
      const double hx = 0.5 * f * (op[rr].x + om[rr].x), hy = 0.5 * f * (op[rr].y + om[rr].y);
      const double dx = 0.5 * f * (op[rr].x - om[rr].x), dy = 0.5 * f * (op[rr].y - om[rr].y);
      cd* Yp = Ys + ((slot0 + pos) * n_rhs + r0 + rr) * 3;
      Yp[0] = cd{hx, hy};
      Yp[1] = cd{dy, -dx};
      Yp[2] = cd{f * oz[rr].x, f * oz[rr].y};
    }
  }
  }
  wq.leave();
}

// A[r][pt][c] += the point's direct-pair slots in their fixed order (the
// order of the reaction components, then of the leaves and chunks), for
// every point that has slots: gpt[i] the point, its slots gslot[gptr[i] ..
// gptr[i+1]-1].  One thread per (point, rhs).
__global__ void k_s2t_gather(const int* gpt, const int* gptr, const int* gslot, int n_pts, int n_rhs, const cd* Ys,
                             long long n_tgt, cd* A) {
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (long long)n_pts * n_rhs) return;
  const int i = (int)(e / n_rhs), r = (int)(e - (long long)i * n_rhs);
  const int id = gpt[i];
  cd* Ap = A + ((long long)r * n_tgt + id) * 3;
  cd a0 = Ap[0], a1 = Ap[1], a2 = Ap[2];
  for (int q = gptr[i]; q < gptr[i + 1]; q++) {
    const cd* Yp = Ys + ((long long)gslot[q] * n_rhs + r) * 3;
    a0 = a0 + Yp[0];
    a1 = a1 + Yp[1];
    a2 = a2 + Yp[2];
  }
  Ap[0] = a0;
  Ap[1] = a1;
  Ap[2] = a2;
}
void launch_s2t_gather(const int* gpt, const int* gptr, const int* gslot, int n_pts, int n_rhs, const cd* Ys,
                       long long n_tgt, cd* A, hipStream_t s) {
  const long long n = (long long)n_pts * n_rhs;
  if (n <= 0) return;
  hipLaunchKernelGGL(k_s2t_gather, dim3((unsigned)((n + NT - 1) / NT)), dim3(NT), 0, s, gpt, gptr, gslot, n_pts,
                     n_rhs, Ys, n_tgt, A);
}
// Source-position gradients through the direct reaction pairs (the swapped
// roles of the gradient path: the "targets" are the points x where the
// gradient is wanted, with weights W, the "sources" carry the currents c of
// the conjugated output gradient).  Per pair the derivatives of the pair's
// field B at x are taken inside the Sommerfeld integrals: with
// D+- = d/dx +- i d/dy on e^{i kappa phi} J_|kappa|(k_rho rho), the Bessel
// ladder D+ (J_n e^{i n phi}) = -k_rho J_{n+1} e^{i (n+1) phi},
// D- (J_n e^{i n phi}) = k_rho J_{n-1} e^{i (n-1) phi} (signed orders), and
// d/dz brings i e k_z of the target layer.  The integrals
//   K_s,n = sum_nodes w k_rho Z F_s k_rho J_n,   L_s,n = sum w k_rho Z F_s (i e k_z) J_n
// give every derivative of the five W(kappa, s); the field derivatives are
// contracted with W, and gX[x] += Re sum_b W_b d_a B_b (summed over the
// right-hand sides), each target adding its pairs in a fixed order.
__device__ inline void bessel3_from012(cd z, cd iz, bool small, const cd* j, cd* j3) {
  // J3 = 4 J2 / z - J1, or its series z^3/48 (1 - z^2/16) near 0
  if (small) {
    cd z2 = z * z;
    *j3 = (z2 * z) * (1.0 / 48.0) * (cd{1.0, 0.0} - z2 * (1.0 / 16.0));
  } else {
    *j3 = 4.0 * (j[2] * iz) - j[1];
  }
}
template <bool SMALLZ>
__global__ __launch_bounds__(LM_S2T_CHUNK, 2) void k_s2t_grad(DevPlan d, MediumDev md, const int* items,
                                                              const int* tlist, const int* slist,
                                                              const double* sxyz, const cd* C, long long n_src,
                                                              const double* txyz, const cd* W, long long n_tgt,
                                                              int n_rhs, double a, double* Gs) {
  __shared__ double tp[LM_S2T_CHUNK][3];
  __shared__ double res[LM_S2T_CHUNK][3];
  __shared__ cd nk[LM_S2T_CHUNK][10];
  __shared__ int tpid[LM_S2T_CHUNK];  // point of each target lane
  const int tid = threadIdx.x;
  // work item as in k_s2t (targets and sources ordered by their distances
  // to the interface planes); each target's gradient goes to its slot of Gs
  const int* it6 = items + 6 * blockIdx.x;
  const int b = __builtin_amdgcn_readfirstlane(it6[0]);
  const int chunk = __builtin_amdgcn_readfirstlane(it6[1]);
  const long long slot0 = __builtin_amdgcn_readfirstlane(it6[2]);
  const int* tl = tlist + __builtin_amdgcn_readfirstlane(it6[3]);
  const int* sl = slist + __builtin_amdgcn_readfirstlane(it6[4]);
  const int ns = __builtin_amdgcn_readfirstlane(it6[5]);
  const TgtBox tb = d.tbox[b];
  const InstParams ip = d.inst[__builtin_amdgcn_readfirstlane(tb.inst)];
  const int t0 = tb.pt0 + chunk * LM_S2T_CHUNK;
  const int nt = min(LM_S2T_CHUNK, tb.pt1 - t0);
  const int n0 = __builtin_amdgcn_readfirstlane(ip.s2t0), nn = __builtin_amdgcn_readfirstlane(ip.s2tn);
  const int nser = __builtin_amdgcn_readfirstlane(ip.s2t_nser);
  const QNode* nodes = d.nodes + n0;
  const double dls = ip.up_s ? md.d[ip.ls - 1] : md.d[ip.ls];
  const double esg = ip.up_t ? 1.0 : -1.0;  // d t / d z at the target
  int pos = 0;
  if (tid < nt) {
    pos = tl[tid];
    const int id = d.tgt_perm[t0 + pos];
    double zt = txyz[3 * id + 2];
    tp[tid][0] = txyz[3 * id];
    tp[tid][1] = txyz[3 * id + 1];
    tp[tid][2] = ip.up_t ? zt - md.d[ip.lt] : md.d[ip.lt - 1] - zt;
    tpid[tid] = id;
  }
  __syncthreads();
  double gx = 0, gy = 0, gz = 0;  // thread tid < nt: totals of target tid
  {
    const int npair = nt * ns;
    for (int q0 = 0; q0 < npair; q0 += LM_S2T_CHUNK) {
      const int q = q0 + tid;
      const bool pa = q < npair;
      const int i = pa ? q / ns : 0, j = pa ? q - (q / ns) * ns : 0;
      const int sid = sl[j];
      const double* sx = sxyz + 3 * (long long)sid;
      double dx = tp[i][0] - sx[0], dy = tp[i][1] - sx[1];
      double tz = tp[i][2], uz = ip.up_s ? dls - sx[2] : sx[2] - dls;
      double rho = sqrt(dx * dx + dy * dy);
      const double irho = rho > 0 ? 1.0 / rho : 0.0;
      double cph = rho > 0 ? dx * irho : 1.0, sph = rho > 0 ? dy * irho : 0.0;
      double kcut = pa ? a + LM_S2T_DIGITS / (tz + uz) : -1.0;
      cd K11 = cd{0, 0}, K51 = cd{0, 0}, K20 = cd{0, 0}, K22 = cd{0, 0}, K40 = cd{0, 0}, K42 = cd{0, 0};
      cd K31 = cd{0, 0}, K33 = cd{0, 0};
      cd L10 = cd{0, 0}, L21 = cd{0, 0}, L32 = cd{0, 0}, L41 = cd{0, 0}, L50 = cd{0, 0};
      for (int c0 = 0; c0 < nn; c0 += LM_S2T_CHUNK) {
        const int nc = min(LM_S2T_CHUNK, nn - c0);
        __syncthreads();
        if (tid < nc) {
          const QNode& nd = nodes[c0 + tid];
          nk[tid][0] = nd.kr;
          nk[tid][1] = nd.w * nd.kr;
          nk[tid][2] = nd.kzt;
          nk[tid][3] = nd.kzs;
          for (int f = 0; f < 5; f++) nk[tid][4 + f] = nd.F[f];
          nk[tid][9] = cd{nd.kr.y == 0.0 ? 1.0 / nd.kr.x : 0.0, 0.0};
        }
        __syncthreads();
        for (int m = 0; m < nc; m++) {
          const cd kr = nk[m][0];
          cd jb[4], base;
          if (kr.y != 0.0) {
            if (!pa) continue;
            const cd ez = cd{0, 1} * (tz * nk[m][2] + uz * nk[m][3]);
            double esn, ecs;
            lm_sincos_red(ez.y, &esn, &ecs);
            const double ea = exp(ez.x);
            base = nk[m][1] * cd{ea * ecs, ea * esn};
            const cd z = rho * kr;
            if (SMALLZ)
              bessel012_horner(z, nser, jb, jb + 1, jb + 2);
            else
              bessel_jq(2, z, jb);
            const bool small = rho * cabsd(kr) < 1e-2;
            bessel3_from012(z, small ? cd{0, 0} : cd{1.0, 0.0} / z, small, jb, jb + 3);
          } else if (kr.x <= kcut) {
            double zf = exp(-(tz * nk[m][2].y + uz * nk[m][3].y));
            base = cd{nk[m][1].x * zf, 0.0};
            const double x = kr.x * rho, ix = nk[m][9].x * irho;
            double J0, J1;
            bessel01_real(x, ix, &J0, &J1);
            double J2 = x > 1e-3 ? 2.0 * J1 * ix - J0 : x * x * (0.125 - x * x * (1.0 / 96.0));
            double J3 = x > 1e-2 ? 4.0 * J2 * ix - J1 : x * x * x * (1.0 / 48.0) * (1.0 - x * x * (1.0 / 16.0));
            jb[0] = cd{J0, 0};
            jb[1] = cd{J1, 0};
            jb[2] = cd{J2, 0};
            jb[3] = cd{J3, 0};
          } else {
            continue;
          }
          const cd bk = base * kr;                                 // K weight
          const cd bl = base * (cd{0.0, esg} * nk[m][2]);          // L weight: i e k_z
          K11 = K11 + (bk * jb[1]) * nk[m][4];
          K51 = K51 + (bk * jb[1]) * nk[m][8];
          K20 = K20 + (bk * jb[0]) * nk[m][5];
          K22 = K22 + (bk * jb[2]) * nk[m][5];
          K40 = K40 + (bk * jb[0]) * nk[m][7];
          K42 = K42 + (bk * jb[2]) * nk[m][7];
          K31 = K31 + (bk * jb[1]) * nk[m][6];
          K33 = K33 + (bk * jb[3]) * nk[m][6];
          L10 = L10 + (bl * jb[0]) * nk[m][4];
          L21 = L21 + (bl * jb[1]) * nk[m][5];
          L32 = L32 + (bl * jb[2]) * nk[m][6];
          L41 = L41 + (bl * jb[1]) * nk[m][7];
          L50 = L50 + (bl * jb[0]) * nk[m][8];
        }
        bool more = false;
        if (c0 + nc < nn) {
          const cd kn = nodes[c0 + nc].kr;
          more = kn.y != 0.0 || kn.x <= kcut;
        }
        if (!__syncthreads_or(more)) break;
      }
      double r0v = 0, r1v = 0, r2v = 0;
      if (pa) {
        const cd I{0.0, 1.0};
        const cd e1 = cd{cph, sph}, e1c = cd{cph, -sph};
        const cd e2 = e1 * e1, e2c = cconj(e2), e3 = e2 * e1, e3c = cconj(e3);
        // derivatives of W(kappa, s) = e^{i kappa phi} i^{1+|kappa|} I_s,|kappa|: [D+, D-, d/dz]
        const cd W1[3] = {-(I * e1) * K11, -(I * e1c) * K11, I * L10};
        const cd W5[3] = {-(I * e1) * K51, -(I * e1c) * K51, I * L50};
        const cd W2p[3] = {e2 * K22, -K20, -(e1 * L21)};
        const cd W2m[3] = {-K20, e2c * K22, -(e1c * L21)};
        const cd W4p[3] = {e2 * K42, -K40, -(e1 * L41)};
        const cd W4m[3] = {-K40, e2c * K42, -(e1c * L41)};
        const cd W3p[3] = {(I * e3) * K33, -(I * e1) * K31, -(I * e2) * L32};
        const cd W3m[3] = {-(I * e1c) * K31, (I * e3c) * K33, -(I * e2c) * L32};
        const double f = 0.079577471545947667884;  // 1 / (4 pi)
        for (int r = 0; r < n_rhs; r++) {
          const cd* cp = C + ((long long)r * n_src + sid) * 3;
          const cd cx = cp[0], cy = cp[1], czv = cp[2];
          const cd cpl = cx + I * cy, cmi = cx - I * cy;
          const cd* wp = W + ((long long)r * n_tgt + tpid[i]) * 3;
          const cd wpl = wp[0] + I * wp[1], wmi = wp[0] - I * wp[1], wz = wp[2];
          cd Q[3];
          for (int x = 0; x < 3; x++) {
            const cd dop = 0.5 * (W1[x] * cpl) - 0.5 * (W3p[x] * cmi) + W2p[x] * czv;
            const cd dom = 0.5 * (W1[x] * cmi) - 0.5 * (W3m[x] * cpl) + W2m[x] * czv;
            const cd doz = 0.5 * (W4p[x] * cmi) + 0.5 * (W4m[x] * cpl) + W5[x] * czv;
            Q[x] = (0.5 * f) * (wpl * dom + wmi * dop) + f * (wz * doz);
          }
          // d/dx = (D+ + D-)/2, d/dy = (D+ - D-)/(2i)
          r0v += 0.5 * (Q[0].x + Q[1].x);
          r1v += 0.5 * (Q[0].y - Q[1].y);
          r2v += Q[2].x;
        }
      }
      res[tid][0] = r0v;
      res[tid][1] = r1v;
      res[tid][2] = r2v;
      __syncthreads();
      if (tid < nt) {
        int qa = max(q0, tid * ns), qb = min(q0 + LM_S2T_CHUNK, (tid + 1) * ns);
        for (int qq = qa; qq < qb; qq++) {
          gx += res[qq - q0][0];
          gy += res[qq - q0][1];
          gz += res[qq - q0][2];
        }
      }
      __syncthreads();
    }
  }
  if (tid < nt) {
    double* g = Gs + (slot0 + pos) * 3;
    g[0] = gx;
    g[1] = gy;
    g[2] = gz;
  }
}
void launch_s2t_grad(const DevPlan& d, MediumDev md, const int* items, const int* tlist, const int* slist, int n,
                     const double* sxyz, const cd* C, long long n_src, const double* txyz, const cd* W,
                     long long n_tgt, int n_rhs, double a, bool smallz, double* Gs, hipStream_t s) {
  if (n <= 0) return;
  if (smallz)
    hipLaunchKernelGGL(k_s2t_grad<true>, dim3(n), dim3(LM_S2T_CHUNK), 0, s, d, md, items, tlist, slist, sxyz, C,
                       n_src, txyz, W, n_tgt, n_rhs, a, Gs);
  else
    hipLaunchKernelGGL(k_s2t_grad<false>, dim3(n), dim3(LM_S2T_CHUNK), 0, s, d, md, items, tlist, slist, sxyz, C,
                       n_src, txyz, W, n_tgt, n_rhs, a, Gs);
}
// gradient slots (three reals each) added into gX, per point in slot order
__global__ void k_s2t_gather_grad(const int* gpt, const int* gptr, const int* gslot, int n_pts, const double* Gs,
                                  double* gX) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_pts) return;
  double* g = gX + 3 * (long long)gpt[i];
  double g0 = g[0], g1 = g[1], g2 = g[2];
  for (int q = gptr[i]; q < gptr[i + 1]; q++) {
    const double* Gp = Gs + 3 * (long long)gslot[q];
    g0 += Gp[0];
    g1 += Gp[1];
    g2 += Gp[2];
  }
  g[0] = g0;
  g[1] = g1;
  g[2] = g2;
}
void launch_s2t_gather_grad(const int* gpt, const int* gptr, const int* gslot, int n_pts, const double* Gs,
                            double* gX, hipStream_t s) {
  if (n_pts <= 0) return;
  hipLaunchKernelGGL(k_s2t_gather_grad, dim3((n_pts + NT - 1) / NT), dim3(NT), 0, s, gpt, gptr, gslot, n_pts, Gs, gX);
}

// items: n work items (target leaf, chunk, first output slot, offset of its
// target order in tlist, offset of its source list in slist, source count)
// of any reaction components, each block writing its targets' totals to its
// own slots of Ys [slot][rhs][3]; smallz: |k_rho| rho <= 7.5 on Gamma_1 for all
// of their pairs (the series length comes from each block's instance)
void launch_s2t(const DevPlan& d, MediumDev md, const int* items, const int* tlist, const int* slist, int n,
                const double* sxyz, const cd* J, long long n_src, const double* txyz, long long n_tgt, int n_rhs,
                double a, bool smallz, cd* Ys, hipStream_t s, bool hfield) {
  if (n <= 0) return;
#define LM_S2T_GO(SZ, RS, H)                                                                                 \
  do {                                                                                                       \
    const int g = persistent_grid((const void*)k_s2t<SZ, RS, H>, LM_S2T_CHUNK, 0,                            \
                                  (long long)n * ((n_rhs + RS - 1) / RS));                                   \
    hipLaunchKernelGGL((k_s2t<SZ, RS, H>), dim3(g), dim3(LM_S2T_CHUNK), 0, s, d, md, items, n, tlist, slist, \
                       sxyz, J, n_src, txyz, n_tgt, n_rhs, a, Ys);                                           \
  } while (0)
  if (hfield) {
    if (n_rhs == 1) {
      if (smallz)
        LM_S2T_GO(true, 1, true);
      else
        LM_S2T_GO(false, 1, true);
    } else {
      if (smallz)
        LM_S2T_GO(true, 4, true);
      else
        LM_S2T_GO(false, 4, true);
    }
  } else if (n_rhs == 1) {
    if (smallz)
      LM_S2T_GO(true, 1, false);
    else
      LM_S2T_GO(false, 1, false);
  } else {
    if (smallz)
      LM_S2T_GO(true, 4, false);
    else
      LM_S2T_GO(false, 4, false);
  }
#undef LM_S2T_GO
}

// ------------------------------------------------------------------ translation tables
// (R|R) and (S|R) by the addition theorem of wave functions written with
// Gaunt coefficients G = int Y^mu_nu conj(Y^m_n) conj(Y^{mu-m}_q):
//   f_nu^mu(x + b) = sum_nm [4 pi sum_q i^{n+q-nu} f_q(k|b|) Y^{mu-m}_q(b) G] j_n Y^m_n(x)
// with f = j (regular) or h (outgoing, |x| < |b|).
__device__ inline double gaunt_at(const double* G, int gp, int nu, int mu, int n, int m, int q) {
  long long Pg = (long long)(gp + 1) * (gp + 1);
  return G[(((long long)nm_idx(nu, mu) * Pg) + nm_idx(n, m)) * (2 * gp + 1) + q];
}
__global__ __launch_bounds__(NT) void k_trans(DevPlan d, int gp) {
  __shared__ cd fq[2 * LM_PMAX + 2];
  __shared__ cd Yq[(2 * LM_PMAX + 1) * (2 * LM_PMAX + 1)];
  __shared__ double leg[(2 * LM_PMAX + 1) * (2 * LM_PMAX + 2) / 2];
  __shared__ double jq[2 * LM_PMAX + 2], yq[2 * LM_PMAX + 2];
  TransJob job = d.trans[blockIdx.x];
  int p = job.p, P = (p + 1) * (p + 1), Q = 2 * p;
  int tid = threadIdx.x;
  double bx = job.b[0], by = job.b[1], bz = job.b[2];
  double bn = sqrt(bx * bx + by * by + bz * bz), bxy = sqrt(bx * bx + by * by);
  double ct = bn > 0 ? bz / bn : 1.0, st = bn > 0 ? bxy / bn : 0.0;
  double phi = bxy > 0 ? atan2(by, bx) : 0.0;
  if (tid == 0) {
    legendre_r(Q, ct, st, leg);
    sph_jn(Q, job.k * bn, jq);
    if (job.kind == 0) sph_yn(Q, job.k * bn, yq);
  }
  __syncthreads();
  for (int e = tid; e <= Q; e += NT) fq[e] = job.kind == 0 ? cd{jq[e], yq[e]} : cd{jq[e], 0.0};
  for (int e = tid; e < (Q + 1) * (Q + 1); e += NT) {
    int q = n_of(e), s = e - q * q - q, as = s < 0 ? -s : s;
    double v = leg[tri_idx(q, as)];
    if (s < 0 && (as & 1)) v = -v;
    Yq[e] = cd{v * cos(s * phi), v * sin(s * phi)};
  }
  __syncthreads();
  cd* M = d.mats + job.mat;
  const double fourpi = 12.566370614359172954;
  for (long long e = tid; e < (long long)P * P; e += NT) {
    int a = (int)(e / P), bcol = (int)(e - (long long)a * P);
    cd v = cd{0, 0};
    if (job.kind == 0) {
      // row-major [out nm = a][in nu mu = bcol]
      int n = n_of(a), m = a - n * n - n, nu = n_of(bcol), mu = bcol - nu * nu - nu;
      int s = mu - m;
      for (int q = abs(n - nu); q <= n + nu; q += 2) {
        if (abs(s) > q) continue;
        v = v + (fourpi * gaunt_at(d.gaunt, gp, nu, mu, n, m, q)) * (ipow(n + q - nu) * fq[q] * Yq[nm_idx(q, s)]);
      }
      v = cd{0.0, job.k} * v;  // i k prefactor of the free-space multipole expansion
    } else if (job.kind == 1) {
      // [in nu mu = a][out nm = bcol]: conj of (R|R)_{nm -> nu mu}(b)
      int nu = n_of(a), mu = a - nu * nu - nu, n = n_of(bcol), m = bcol - n * n - n;
      int s = m - mu;
      for (int q = abs(n - nu); q <= n + nu; q += 2) {
        if (abs(s) > q) continue;
        v = v + (fourpi * gaunt_at(d.gaunt, gp, n, m, nu, mu, q)) * (ipow(nu + q - n) * fq[q] * Yq[nm_idx(q, s)]);
      }
      v = cconj(v);
    } else {
      // [in nu mu = a][out nm = bcol]: (R|R)_{nu mu -> nm}(b)
      int nu = n_of(a), mu = a - nu * nu - nu, n = n_of(bcol), m = bcol - n * n - n;
      int s = mu - m;
      for (int q = abs(n - nu); q <= n + nu; q += 2) {
        if (abs(s) > q) continue;
        v = v + (fourpi * gaunt_at(d.gaunt, gp, nu, mu, n, m, q)) * (ipow(n + q - nu) * fq[q] * Yq[nm_idx(q, s)]);
      }
    }
    M[e] = v;
  }
}
void launch_trans(const DevPlan& d, int n_jobs, int gp, hipStream_t s) {
  if (n_jobs <= 0) return;
  hipLaunchKernelGGL(k_trans, dim3(n_jobs), dim3(NT), 0, s, d, gp);
}

// ------------------------------------------------------------------ reaction densities
// Generalized reflection coefficients (the classical O(L) recursion for the
// layered 1-D interface problems of Sec. 3.1): amplitude, in the target
// layer, of the up-going (up_t) or down-going wave excited by a unit source
// wave leaving the source layer upward (up_s) or downward, with local
// reference planes (every exponential factor has modulus <= 1).
__device__ cd react_coef(const MediumDev& md, cd kr, int lt, int ls, int up_t, int up_s, int pol) {
  int n = md.n, L = n - 1;
  cd kz[LM_MAXL], E[LM_MAXL], Rd[LM_MAXL], Ru[LM_MAXL];
  double beta[LM_MAXL];
  for (int m = 0; m < n; m++) {
    kz[m] = kz_of(md.k[m], kr);
    // interface conditions of Sec. 3.1: [[u'/mu]] = 0 (TE), [[u'/eps]] = 0 (TM), eps ~ k^2 / mu
    beta[m] = pol ? md.k[m] * md.k[m] / md.mu[m] : md.mu[m];
    E[m] = (m >= 1 && m <= L - 1) ? cexpd(cd{0, 1} * kz[m] * (md.d[m - 1] - md.d[m])) : cd{0, 0};
    Rd[m] = Ru[m] = cd{0, 0};
  }
  auto fres = [&](int a, int b) {
    cd x = (1.0 / beta[a]) * kz[a], y = (1.0 / beta[b]) * kz[b];
    return (x - y) / (x + y);
  };
  for (int m = L - 1; m >= 0; m--) {
    cd r = fres(m, m + 1);
    if (m + 1 <= L - 1) {
      cd e2 = E[m + 1] * E[m + 1];
      Rd[m] = (r + Rd[m + 1] * e2) / (cd{1, 0} + r * Rd[m + 1] * e2);
    } else
      Rd[m] = r;
  }
  for (int m = 1; m <= L; m++) {
    cd r = fres(m, m - 1);
    if (m - 1 >= 1) {
      cd e2 = E[m - 1] * E[m - 1];
      Ru[m] = (r + Ru[m - 1] * e2) / (cd{1, 0} + r * Ru[m - 1] * e2);
    } else
      Ru[m] = r;
  }
  int s = ls;
  cd c = cd{0, 1} / (2.0 * kz[s]);
  cd Es = E[s];
  cd den = cd{1, 0} - Ru[s] * Rd[s] * Es * Es;
  cd Aa, Bb, ctop = cd{0, 0}, cbot = cd{0, 0};
  if (up_s) {
    Bb = Ru[s] * c / den;
    Aa = Rd[s] * Es * Bb;
    ctop = c;
  } else {
    Aa = Rd[s] * c / den;
    Bb = Ru[s] * Es * Aa;
    cbot = c;
  }
  cd a, b;
  if (lt == s) {
    a = Aa;
    b = Bb;
  } else if (lt > s) {
    cd Dn = (cbot + Bb * Es) * (cd{1, 0} + Rd[s]) /
            (cd{1, 0} + ((s + 1 <= L - 1) ? Rd[s + 1] * E[s + 1] * E[s + 1] : cd{0, 0}));
    for (int m = s + 1; m < lt; m++)
      Dn = Dn * E[m] * (cd{1, 0} + Rd[m]) / (cd{1, 0} + ((m + 1 <= L - 1) ? Rd[m + 1] * E[m + 1] * E[m + 1] : cd{0, 0}));
    b = Dn;
    a = (lt <= L - 1) ? Rd[lt] * Dn * E[lt] : cd{0, 0};
  } else {
    cd Up = (ctop + Aa * Es) * (cd{1, 0} + Ru[s]) /
            (cd{1, 0} + ((s - 1 >= 1) ? Ru[s - 1] * E[s - 1] * E[s - 1] : cd{0, 0}));
    for (int m = s - 1; m > lt; m--)
      Up = Up * E[m] * (cd{1, 0} + Ru[m]) / (cd{1, 0} + ((m - 1 >= 1) ? Ru[m - 1] * E[m - 1] * E[m - 1] : cd{0, 0}));
    a = Up;
    b = (lt >= 1) ? Ru[lt] * Up * E[lt] : cd{0, 0};
  }
  return up_t ? a : b;
}

// Spectral densities of a reaction component at one quadrature node: the
// coefficients of the eight-term angular decomposition of the spectral
// dyadic (paper Sec. 3.1; sigma_3 with the sign that follows from Theta),
// written as F = -(2i/k^2) S with
//   S1 = k^2 c_TE - e h kz kz' c_TM,  S3 = k^2 c_TE + e h kz kz' c_TM,
//   S2 = -e kz kr c_TM,  S4 = h kz' kr c_TM,  S5 = kr^2 c_TM,
// e = +1 (-1) for a wave arriving up (down), h = -1 (+1) for leaving up (down).
__global__ void k_nodes(DevPlan d, MediumDev md, int n_nodes, const int* node_inst, const cd* krs, const cd* ws) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_nodes) return;
  InstParams ip = d.inst[node_inst[i]];
  cd kr = krs[i];
  QNode q;
  q.kr = kr;
  q.w = ws[i];
  q.kzt = kz_of(ip.kt, kr);
  q.kzs = kz_of(ip.ks, kr);
  cd cte = react_coef(md, kr, ip.lt, ip.ls, ip.up_t, ip.up_s, 0);
  // the TM terms carry mu of the target layer over mu of the source layer
  // (the TM coefficient's mu_l and its 1-D source's 1/mu_l', Sec. 3.1)
  cd ctm = (md.mu[ip.lt] / md.mu[ip.ls]) * react_coef(md, kr, ip.lt, ip.ls, ip.up_t, ip.up_s, 1);
  double e = ip.up_t ? 1.0 : -1.0, h = ip.up_s ? -1.0 : 1.0;
  double k2 = ip.kt * ip.kt;
  cd kk = q.kzt * q.kzs;
  cd S[5];
  S[0] = k2 * cte - (e * h) * (kk * ctm);
  S[1] = (-e) * (q.kzt * kr * ctm);
  S[2] = k2 * cte + (e * h) * (kk * ctm);
  S[3] = h * (q.kzs * kr * ctm);
  S[4] = kr * kr * ctm;
  cd pre = cd{0.0, -2.0 / k2};
  for (int j = 0; j < 5; j++) q.F[j] = pre * S[j];
  // curl of the field (mu_t G_H, the J6..J9 form of Sec. 3.1) in the same
  // slots: d/dz brings i e kz_t, d/dz' i h kz_s; the xy block's kappa = 0
  // and kappa = 2 parts (J9 and half of J8) go to slots 1 and 3, the z
  // column (J7) to slot 2, the z row (J6) to slot 4, nothing to slot 5; the
  // near-field kernel combines them with the signs of the curl
  cd etc = (e * cte) * q.kzt, hsc = (h * ctm) * q.kzs;
  cd SH[5];
  SH[0] = hsc - etc;
  SH[1] = kr * ctm;
  SH[2] = -(etc + hsc);
  SH[3] = kr * cte;
  SH[4] = cd{0.0, 0.0};
  for (int j = 0; j < 5; j++) q.FH[j] = cd{0.0, -2.0} * SH[j];
  q.tau_t[0] = cd{1, 0};
  q.tau_t[1] = cd{ip.kt, 0} / q.kzt;
  q.tau_t[2] = (1.0 / ip.kt) * kr;
  q.tau_t[3] = kr / q.kzt;
  q.tau_s[0] = cd{1, 0};
  q.tau_s[1] = cd{ip.ks, 0} / q.kzs;
  q.tau_s[2] = (1.0 / ip.ks) * kr;
  q.tau_s[3] = kr / q.kzs;
  double kb = ip.kt <= ip.ks ? ip.kt : ip.ks;
  q.x0 = cd{1, 0} - (2.0 / (kb * kb)) * (kr * kr);
  d.nodes[i] = q;
}
void launch_nodes(const DevPlan& d, MediumDev med, int n_nodes, const int* node_inst, const cd* kr, const cd* w,
                  hipStream_t s) {
  if (n_nodes <= 0) return;
  hipLaunchKernelGGL(k_nodes, dim3((n_nodes + 127) / 128), dim3(128), 0, s, d, med, n_nodes, node_inst, kr, w);
}

// per (case, node): g = w kr Z(centres) and J_q(kr rho), q <= 2p+2
__global__ void k_tab_bessel(DevPlan d, MediumDev md, int case0, int ncase, int maxnode, int p, cd* scr) {
  long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  int NQ = 2 * p + 3;
  if (i >= (long long)ncase * maxnode) return;
  int ci = (int)(i / maxnode), nd = (int)(i - (long long)ci * maxnode);
  TabCase tc = d.cases[case0 + ci];
  cd* out = scr + i * (NQ + 1);
  if (nd >= tc.nnode) return;
  QNode q = d.nodes[tc.node0 + nd];
  InstParams ip = d.inst[tc.inst];
  double tz = ip.up_t ? tc.zt_orig - md.d[ip.lt] : md.d[ip.lt - 1] - tc.zt_orig;
  double uz = ip.up_s ? md.d[ip.ls - 1] - tc.zs_orig : tc.zs_orig - md.d[ip.ls];
  cd ex = cd{0, 1} * (tz * q.kzt + uz * q.kzs);
  out[0] = q.w * q.kr * cexpd(ex);
  bessel_jq(NQ - 1, tc.rho * q.kr, out + 1);
}

// Chebyshev-weighted Sommerfeld integrals of one case (Sec. 3.4):
//   I[sig][tt][ts][l][q] = sum_nodes w kr Z F_sig tau_tt(b) tau_ts(b') T_l(cos 2 b0) J_q(kr rho)
#define TAB_NC 8
#define TAB_OUT 16  // outputs per thread (a block: NT * TAB_OUT consecutive entries of one case)
__global__ __launch_bounds__(NT) void k_tab_integrals(DevPlan d, int case0, int p, int maxnode, const cd* scr) {
  extern __shared__ cd shm[];
  int NQ = 2 * p + 3, NL = p + 2, NLQ = NL * NQ;
  int E = 80 * NLQ;
  cd* H = shm;                      // [TAB_NC][80]
  cd* U = H + TAB_NC * 80;          // [TAB_NC][NLQ]
  cd* Tl = U + TAB_NC * NLQ;        // [TAB_NC][NL]
  int ci = blockIdx.x;
  TabCase tc = d.cases[case0 + ci];
  int tid = threadIdx.x;
  int e0 = blockIdx.y * (NT * TAB_OUT);
  cd acc[TAB_OUT];
  for (int j = 0; j < TAB_OUT; j++) acc[j] = cd{0, 0};
  const cd* sc = scr + (long long)ci * maxnode * (NQ + 1);
  for (int n0 = 0; n0 < tc.nnode; n0 += TAB_NC) {
    int nn = min(TAB_NC, tc.nnode - n0);
    __syncthreads();
    if (tid < nn) cheb_t(NL - 1, d.nodes[tc.node0 + n0 + tid].x0, Tl + tid * NL);
    for (int e = tid; e < TAB_NC * 80; e += NT) {
      int t = e / 80, a = e - t * 80;
      cd v = cd{0, 0};
      if (t < nn) {
        const QNode& q = d.nodes[tc.node0 + n0 + t];
        int sg = a / 16, tt = (a / 4) & 3, ts = a & 3;
        v = sc[(long long)(n0 + t) * (NQ + 1)] * q.F[sg] * q.tau_t[tt] * q.tau_s[ts];
      }
      H[e] = v;
    }
    __syncthreads();
    for (int e = tid; e < TAB_NC * NLQ; e += NT) {
      int t = e / NLQ, b = e - t * NLQ, l = b / NQ, qq = b - l * NQ;
      U[e] = (t < nn) ? Tl[t * NL + l] * sc[(long long)(n0 + t) * (NQ + 1) + 1 + qq] : cd{0, 0};
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < TAB_OUT; j++) {
      int e = e0 + j * NT + tid;
      if (e >= E) break;
      int a = e / NLQ, b = e - a * NLQ;
      cd s = acc[j];
      for (int t = 0; t < nn; t++) s = s + H[t * 80 + a] * U[t * NLQ + b];
      acc[j] = s;
    }
  }
#pragma unroll
  for (int j = 0; j < TAB_OUT; j++) {
    int e = e0 + j * NT + tid;
    if (e < E) d.ibuf[tc.ibuf + e] = acc[j];
  }
}

void launch_tab_integrals(const DevPlan& d, MediumDev med, int case0, int ncase, int p, cd* scr, long long maxnode,
                          hipStream_t s) {
  if (ncase <= 0) return;
  long long nth = (long long)ncase * maxnode;
  hipLaunchKernelGGL(k_tab_bessel, dim3((unsigned)((nth + 127) / 128)), dim3(128), 0, s, d, med, case0, ncase,
                     (int)maxnode, p, scr);
  int NQ = 2 * p + 3, NL = p + 2;
  int E = 80 * NL * NQ;
  size_t shm = (size_t)(TAB_NC * 80 + TAB_NC * NL * NQ + TAB_NC * NL) * sizeof(cd);
  set_dyn_lds((const void*)k_tab_integrals, shm);
  hipLaunchKernelGGL(k_tab_integrals, dim3(ncase, (E + NT * TAB_OUT - 1) / (NT * TAB_OUT)), dim3(NT), shm, s, d, case0, p,
                     (int)maxnode, scr);
}

// Assembly of the reaction M2L matrices from the Chebyshev integrals
// (Sec. 3.4): the product of the two associated Legendre functions is
// expanded as s/2 tau tau sum_i sum_j B_i B_j sum_s C_js (T_{i+s} + T_{|i-s|})
// in the variable of the smaller wavenumber, so every entry
//   Ihat = s_{m mu}/2 sum_i sum_j B^i_{n|m|} B^j_{nu|mu|} A_ij,
//   A_ij = sum_s C_js (I_{i+s} + I_{|i-s|})   (roles of i, j swapped if k > k')
// and V = 4 pi i^{1+n+|q|} (-i)^nu s^{n+m+nu+mu} Ihat with q = kappa - m + mu.
// The matrices for the three spin outputs are stored as P x 3P blocks.
// Writes, per case, the + and z output rows of the spin-basis tensor (the -
// rows are their mirror images): out[ci * stride + (slot * P + a) * 3P + blk * P
// + b], slot 0 for +, 1 for z, with the column blocks of each output type in the order of its
// input channels (+: u+, u-, z; z: u-, u+, z).  One block per (case,
// density, pair of tau types): the entries of one pair of types are
// disjoint from those of every other pair.
__global__ __launch_bounds__(NT) void k_tab_assemble(DevPlan d, int case0, int p, int KB, int BS, cd* out,
                                                     long long stride) {
  extern __shared__ cd Aij[];  // [(KB+1)^2][NQ]
  int ci = blockIdx.x, sg = blockIdx.y;
  TabCase tc = d.cases[case0 + ci];
  InstParams ip = d.inst[tc.inst];
  int P = ip.P, NQ = 2 * p + 3, NL = p + 2, NLQ = NL * NQ;
  int W = KB + 2;  // stride of C
  const double* C = d.Ccoef + d.Ccoef0[tc.inst];
  bool tbase = ip.kt <= ip.ks;
  int tid = threadIdx.x;
  int K1 = KB + 1;
  // kappa list and target slots for this density
  int nk = 0, kap[2], slot_t[2][2], slot_b[2][2];
  double coef[2][2];
  int nslot[2] = {0, 0};
  if (sg == 0) { nk = 1; kap[0] = 0; nslot[0] = 2; slot_t[0][0] = 0; slot_b[0][0] = 0; coef[0][0] = 0.5; slot_t[0][1] = 1; slot_b[0][1] = 0; coef[0][1] = 0.5; }
  if (sg == 2) { nk = 2; kap[0] = 2; kap[1] = -2; nslot[0] = nslot[1] = 1; slot_t[0][0] = 0; slot_b[0][0] = 1; coef[0][0] = -0.5; slot_t[1][0] = 1; slot_b[1][0] = 1; coef[1][0] = -0.5; }
  if (sg == 1) { nk = 2; kap[0] = 1; kap[1] = -1; nslot[0] = nslot[1] = 1; slot_t[0][0] = 0; slot_b[0][0] = 2; coef[0][0] = 1.0; slot_t[1][0] = 1; slot_b[1][0] = 2; coef[1][0] = 1.0; }
  if (sg == 3) { nk = 2; kap[0] = 1; kap[1] = -1; nslot[0] = nslot[1] = 1; slot_t[0][0] = 2; slot_b[0][0] = 0; coef[0][0] = 0.5; slot_t[1][0] = 2; slot_b[1][0] = 1; coef[1][0] = 0.5; }
  if (sg == 4) { nk = 1; kap[0] = 0; nslot[0] = 1; slot_t[0][0] = 2; slot_b[0][0] = 2; coef[0][0] = 1.0; }
  const cd* Ib = d.ibuf + tc.ibuf;
  cd* Mbase = out + (long long)ci * stride;
  const double fourpi = 12.566370614359172954;
  const int tt = blockIdx.z >> 2, ts = blockIdx.z & 3;
  // the rows (n, m) of tau type tt and the columns (nu, mu) of type ts (in
  // any order: every entry is computed and written on its own)
  __shared__ int rows[(LM_PMAX + 1) * (LM_PMAX + 1)], cols[(LM_PMAX + 1) * (LM_PMAX + 1)];
  __shared__ int nrow, ncol;
  if (tid == 0) nrow = ncol = 0;
  __syncthreads();
  for (int a = tid; a < P; a += NT) {
    const int n = n_of(a), am = abs(a - n * n - n);
    const int t = (n % 2 == 0) ? ((am % 2 == 0) ? 0 : 3) : ((am % 2 == 0) ? 1 : 2);
    if (t == tt) rows[atomicAdd(&nrow, 1)] = a;
    if (t == ts) cols[atomicAdd(&ncol, 1)] = a;
  }
  const cd* I = Ib + ((long long)(sg * 16 + tt * 4 + ts)) * NLQ;
  for (int e = tid; e < K1 * K1 * NQ; e += NT) {
    int ij = e / NQ, q = e - ij * NQ, i = ij / K1, j = ij - i * K1;
    // ib: index on the base (smaller-k) side, io: index expanded by C
    int ib = tbase ? i : j, io = tbase ? j : i;
    cd v = cd{0, 0};
    for (int s = 0; s <= io; s++) {
      double c = C[io * W + s];
      if (c == 0.0) continue;
      int l1 = ib + s, l2 = ib > s ? ib - s : s - ib;
      cd t1 = l1 < NL ? I[l1 * NQ + q] : cd{0, 0};
      cd t2 = l2 < NL ? I[l2 * NQ + q] : cd{0, 0};
      v = v + c * (t1 + t2);
    }
    Aij[e] = v;
  }
  __syncthreads();
  // tau types (Appendix B): t1 = tt, t2 = ts for every entry below
  const int nc = ncol;
  for (int e = tid; e < nrow * nc; e += NT) {
    const int a = rows[e / nc], bb = cols[e - (e / nc) * nc];
    int n = n_of(a), m = a - n * n - n, nu = n_of(bb), mu = bb - nu * nu - nu;
    int am = m < 0 ? -m : m, amu = mu < 0 ? -mu : mu;
    int Kn = (n % 2 == 0) ? n / 2 : ((am % 2 == 0) ? (n + 1) / 2 : (n - 1) / 2);
    int Kv = (nu % 2 == 0) ? nu / 2 : ((amu % 2 == 0) ? (nu + 1) / 2 : (nu - 1) / 2);
    double smu = ((m < 0 && (am & 1)) ? -1.0 : 1.0) * ((mu < 0 && (amu & 1)) ? -1.0 : 1.0);
    const double* Bn = d.Bcoef + (long long)tri_idx(n, am) * BS;
    const double* Bv = d.Bcoef + (long long)tri_idx(nu, amu) * BS;
    double sgn_s = ((n + m + nu + mu) & 1) ? (double)ip.sgn : 1.0;
    for (int kk = 0; kk < nk; kk++) {
      int q = kap[kk] - m + mu, aq = q < 0 ? -q : q;
      cd ih = cd{0, 0};
      for (int i = 0; i <= Kn; i++) {
        cd row = cd{0, 0};
        for (int j = 0; j <= Kv; j++) row = row + Bv[j] * Aij[(i * K1 + j) * NQ + aq];
        ih = ih + Bn[i] * row;
      }
      ih = (0.5 * smu) * ih;
      cd V = (fourpi * sgn_s) * (ipow(1 + n + aq) * ipow(-nu) * ih);  // i^{1+n+|q|} (-i)^nu
      for (int sl = 0; sl < nslot[kk]; sl++) {
        int t = slot_t[kk][sl], blk = slot_b[kk][sl];
        if (t == 1) continue;  // the - rows: mirror images of the + rows
        Mbase[(long long)(t >> 1) * 3 * P * P + (long long)a * 3 * P + (long long)blk * P + bb] = coef[kk][sl] * V;
      }
    }
  }
}
void launch_tab_assemble(const DevPlan& d, int case0, int ncase, int p, int KB, int BS, cd* out, long long stride,
                         hipStream_t s) {
  if (ncase <= 0) return;
  int NQ = 2 * p + 3;
  size_t shm = (size_t)(KB + 1) * (KB + 1) * NQ * sizeof(cd);
  set_dyn_lds((const void*)k_tab_assemble, shm);
  hipLaunchKernelGGL(k_tab_assemble, dim3(ncase, 5, 16), dim3(NT), shm, s, d, case0, p, KB, BS, out, stride);
}

// Even (par 0) and odd (par 1) blocks of each case's reaction M2L tensor
// from the + and z output rows written by k_tab_assemble (src[ci]): with
// e_m = (-1)^m, sign s = +1 (even) or -1 (odd), and the input blocks
// (u+, u-) in the order of the row's output type,
//   column (+, nu mu):  (A[row][u+][nu mu] + s e_mu A[row][u-][nu, -mu]) / 2
//   column (z, nu mu):  (A[row][z][nu mu] + s e_mu A[row][z][nu, -mu]) / 2,
//                       A[row][z][nu 0] for mu = 0 (even only),
// over the rows (+, nm) (every nm) and (z, nm) (m >= 0 even, m >= 1 odd),
// stored row-major [lm_sym_dim(p, par)]^2, the even block first.
__global__ __launch_bounds__(NT) void k_tab_sym(DevPlan d, int case0, const cd* src, long long stride) {
  const int ci = blockIdx.x, par = blockIdx.z;
  const TabCase tc = d.cases[case0 + ci];
  const int p = d.inst[tc.inst].p, P = (p + 1) * (p + 1), R = lm_sym_dim(p, par);
  const cd* A = src + (long long)ci * stride;
  cd* M = d.mats + tc.mat + (par ? (long long)lm_sym_dim(p, 0) * lm_sym_dim(p, 0) : 0);
  const double sg = par ? -1.0 : 1.0;
  const long long n_el = (long long)R * R;
  for (long long e = (long long)blockIdx.y * NT + threadIdx.x; e < n_el; e += (long long)gridDim.y * NT) {
    const int r = (int)(e / R), c = (int)(e - (long long)r * R);
    const bool zrow = r >= P;
    const int a = zrow ? sym_znm(r - P, par) : r;
    const cd* Ar = A + (zrow ? 3LL * P * P : 0) + (long long)a * 3 * P;
    cd v;
    if (c < P) {
      const int nu = n_of(c), mu = c - nu * nu - nu;
      const int bp = zrow ? 1 : 0, bm = zrow ? 0 : 1;  // blocks of u+ and u- in this row's output type
      const double f = sg * ((mu & 1) ? -1.0 : 1.0);
      v = 0.5 * (Ar[(long long)bp * P + c] + f * Ar[(long long)bm * P + c - 2 * mu]);
    } else {
      const int b = sym_znm(c - P, par), nu = n_of(b), mu = b - nu * nu - nu;
      const double f = sg * ((mu & 1) ? -1.0 : 1.0);
      v = mu == 0 ? Ar[2LL * P + b] : 0.5 * (Ar[2LL * P + b] + f * Ar[2LL * P + b - 2 * mu]);
    }
    M[e] = v;
  }
}
void launch_tab_sym(const DevPlan& d, int case0, int ncase, const cd* src, long long stride, hipStream_t s) {
  if (ncase <= 0) return;
  hipLaunchKernelGGL(k_tab_sym, dim3(ncase, 16, 2), dim3(NT), 0, s, d, case0, src, stride);
}
