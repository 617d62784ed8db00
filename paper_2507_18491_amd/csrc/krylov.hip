// krylov.hip -- vector kernels of the GMRES solve over the layered sum.
//
// Every vector is complex128 [n_rhs][n3] (n3 = 3 n values per column) and is
// named by an index into a device table of base pointers (the Krylov basis,
// the work vector, the iterate and the right-hand side).  All of these passes
// are bound by HBM bandwidth: each reads its vectors once, in coalesced
// 16-byte loads, and the inner products reduce in a fixed order (a strided
// per-thread sum, an LDS tree per block, then the blocks in index order), so
// a solve is bitwise repeatable.
#include <hip/hip_runtime.h>

#include "kernels.h"

#define KV_NT 256   // threads per block
#define KV_G 8      // inner products per pass over the right-hand vector
#define KV_MAXV (LM_SOLVE_MAX_RESTART + 4)

__device__ inline cd cmla_conj(cd acc, cd v, cd w) {  // acc + conj(v) w
  return cd{acc.x + v.x * w.x + v.y * w.y, acc.y + v.x * w.y - v.y * w.x};
}

// part[((k0 + q) R + r) NB + blk] = partial sum of conj(V_{first+k0+q}) w over
// the block's share of column r (q < KV_G), grid (NB, R, groups of KV_G).
__global__ __launch_bounds__(KV_NT) void k_kv_dots(cd* const* vt, int first, int count, int w, long long n3,
                                                    int R, int NB, cd* part) {
  const int blk = blockIdx.x, r = blockIdx.y, k0 = blockIdx.z * KV_G;
  const int nk = min(KV_G, count - k0);
  const long long off = (long long)r * n3;
  const cd* wp = vt[w] + off;
  const cd* vp[KV_G];
#pragma unroll
  for (int q = 0; q < KV_G; q++) vp[q] = q < nk ? vt[first + k0 + q] + off : wp;
  cd acc[KV_G];
#pragma unroll
  for (int q = 0; q < KV_G; q++) acc[q] = cd{0.0, 0.0};
  for (long long i = (long long)blk * KV_NT + threadIdx.x; i < n3; i += (long long)NB * KV_NT) {
    const cd wi = wp[i];
#pragma unroll
    for (int q = 0; q < KV_G; q++)
      if (q < nk) acc[q] = cmla_conj(acc[q], vp[q][i], wi);
  }
  __shared__ cd sm[KV_G][KV_NT];
  const int t = threadIdx.x;
#pragma unroll
  for (int q = 0; q < KV_G; q++) sm[q][t] = acc[q];
  __syncthreads();
  for (int s = KV_NT / 2; s > 0; s >>= 1) {
    if (t < s)
#pragma unroll
      for (int q = 0; q < KV_G; q++) sm[q][t] = sm[q][t] + sm[q][t + s];
    __syncthreads();
  }
  if (t < nk) part[((long long)(k0 + t) * R + r) * NB + blk] = sm[t][0];
}

// out[t] = sum of part[t NB + b] over b, one 64-lane block per t: lane l adds
// b = l, l + 64, ... in order, then a fixed LDS tree (deterministic)
__global__ __launch_bounds__(64) void k_kv_sum(const cd* part, int NB, cd* out) {
  const int t = blockIdx.x, l = threadIdx.x;
  cd s{0.0, 0.0};
  for (int b = l; b < NB; b += 64) s = s + part[(long long)t * NB + b];
  __shared__ cd sm[64];
  sm[l] = s;
  __syncthreads();
  for (int h = 32; h > 0; h >>= 1) {
    if (l < h) sm[l] = sm[l] + sm[l + h];
    __syncthreads();
  }
  if (l == 0) out[t] = sm[0];
}

// dst[r][i] += sum_k V_{first+k}[r][i] c[k R + r], grid (blocks, R)
__global__ __launch_bounds__(KV_NT) void k_kv_combine(cd* const* vt, int first, int count, const cd* c,
                                                       int dst, long long n3, int R) {
  const int r = blockIdx.y;
  __shared__ cd cs[KV_MAXV];
  __shared__ const cd* vps[KV_MAXV];
  const long long off = (long long)r * n3;
  for (int k = threadIdx.x; k < count; k += KV_NT) {
    cs[k] = c[(long long)k * R + r];
    vps[k] = vt[first + k] + off;
  }
  __syncthreads();
  cd* dp = vt[dst] + off;
  for (long long i = (long long)blockIdx.x * KV_NT + threadIdx.x; i < n3; i += (long long)gridDim.x * KV_NT) {
    cd a = dp[i];
#pragma unroll 4
    for (int k = 0; k < count; k++) a = a + vps[k][i] * cs[k];
    dp[i] = a;
  }
}

// dst[r][i] = c[r] src[r][i]
__global__ __launch_bounds__(KV_NT) void k_kv_scale(cd* const* vt, int src, const cd* c, int dst, long long n3) {
  const int r = blockIdx.y;
  const cd cr = c[r];
  const cd* sp = vt[src] + (long long)r * n3;
  cd* dp = vt[dst] + (long long)r * n3;
  for (long long i = (long long)blockIdx.x * KV_NT + threadIdx.x; i < n3; i += (long long)gridDim.x * KV_NT)
    dp[i] = sp[i] * cr;
}

// w = b - w
__global__ __launch_bounds__(KV_NT) void k_kv_rsub(cd* const* vt, int b, int w, long long n3) {
  const int r = blockIdx.y;
  const cd* bp = vt[b] + (long long)r * n3;
  cd* wp = vt[w] + (long long)r * n3;
  for (long long i = (long long)blockIdx.x * KV_NT + threadIdx.x; i < n3; i += (long long)gridDim.x * KV_NT)
    wp[i] = bp[i] - wp[i];
}

// dst = D src - dst  (dst holds G src; diag: one value per point, or null)
__global__ __launch_bounds__(KV_NT) void k_kv_diag(cd* const* vt, int src, const cd* diag, int dst,
                                                    long long n3) {
  const int r = blockIdx.y;
  const cd* sp = vt[src] + (long long)r * n3;
  cd* dp = vt[dst] + (long long)r * n3;
  for (long long i = (long long)blockIdx.x * KV_NT + threadIdx.x; i < n3; i += (long long)gridDim.x * KV_NT) {
    const cd g = dp[i];
    dp[i] = diag ? diag[i / 3] * sp[i] - g : -g;
  }
}

static unsigned kv_blocks(long long n3) {
  long long nb = (n3 + KV_NT - 1) / KV_NT;
  return (unsigned)std::max(1LL, std::min(nb, 16384LL));
}

int kv_dots_nb(long long n3, int n_rhs, int count) {
  const long long groups = (count + KV_G - 1) / KV_G;
  long long nb = std::max(1LL, 4096 / std::max(1LL, (long long)n_rhs * groups));
  nb = std::min(nb, std::max(1LL, (n3 + KV_NT - 1) / KV_NT));
  return (int)std::min(nb, 1024LL);
}

void launch_kv_dots(cd* const* vt, int first, int count, int w, long long n3, int n_rhs, int nb, cd* part,
                    cd* out, hipStream_t s) {
  dim3 g((unsigned)nb, (unsigned)n_rhs, (unsigned)((count + KV_G - 1) / KV_G));
  hipLaunchKernelGGL(k_kv_dots, g, dim3(KV_NT), 0, s, vt, first, count, w, n3, n_rhs, nb, part);
  const int cnt = count * n_rhs;
  hipLaunchKernelGGL(k_kv_sum, dim3((unsigned)cnt), dim3(64), 0, s, part, nb, out);
}

void launch_kv_combine(cd* const* vt, int first, int count, const cd* c, int dst, long long n3, int n_rhs,
                       hipStream_t s) {
  hipLaunchKernelGGL(k_kv_combine, dim3(kv_blocks(n3), (unsigned)n_rhs), dim3(KV_NT), 0, s, vt, first, count, c,
                     dst, n3, n_rhs);
}

void launch_kv_scale(cd* const* vt, int src, const cd* c, int dst, long long n3, int n_rhs, hipStream_t s) {
  hipLaunchKernelGGL(k_kv_scale, dim3(kv_blocks(n3), (unsigned)n_rhs), dim3(KV_NT), 0, s, vt, src, c, dst, n3);
}

void launch_kv_rsub(cd* const* vt, int b, int w, long long n3, int n_rhs, hipStream_t s) {
  hipLaunchKernelGGL(k_kv_rsub, dim3(kv_blocks(n3), (unsigned)n_rhs), dim3(KV_NT), 0, s, vt, b, w, n3);
}

void launch_kv_diag(cd* const* vt, int src, const cd* diag, int dst, long long n3, int n_rhs, hipStream_t s) {
  hipLaunchKernelGGL(k_kv_diag, dim3(kv_blocks(n3), (unsigned)n_rhs), dim3(KV_NT), 0, s, vt, src, diag, dst, n3);
}
