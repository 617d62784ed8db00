// lmfmm_internal.h -- data structures shared by the host planner and the
// HIP kernels of the layered-media dyadic FMM.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "special.h"

#define LM_MAXL 16
#define LM_PMAX 24
#define LM_P2P_CHUNK 256   // targets per near-field work item (= threads per block)
#define LM_P2M_CHUNK 512   // source points per P2M work item (larger leaves: partials, summed)
#define LM_L2P_CHUNK(kind) ((kind) == 0 ? 256 : 64)   // points per L2P work item (free / reaction)
#define LM_S2T_CHUNK 64    // targets per reaction near-field work item (= threads per block)
#define LM_S2T_DIGITS 28.0 // the S2T tail stops where e^{-k (t + u)} < e^{-28}
#define LM_S2T_SEG 32      // near boxes per source segment of one S2T work item

// Octree records sorted outside the host planner (lm_build sorts them on
// the device).  Tree t holds the points of its segments in segment order:
// a segment lists the ids of source (tgt = 0) or target (tgt = 1) points,
// with tag `tag`, whose positions in the tree's frame are (x, y, za z + zb).
// A record's key is the Morton code of its cell in the depth-LM_TREE_DK
// lattice of cells of size S0 / 2^LM_TREE_DK from (x0, y0, z0) (the cell
// index floor((x - x0) 2^LM_TREE_DK / S0), clamped to the lattice, per axis;
// bits interleaved x, y, z from the lowest).  The sorted output holds every
// tree's records in tree order, each tree's by key with equal keys in input
// order: the key and id | tag << 31.  A sorter may also return the boxes:
// for every box, in record order and, per record, level order, the entry
// (level << 40) | r, r the index (in the sorted output) of the box's first
// record.
#define LM_TREE_DK 20
struct TreeSeg {
  const int* ids;  // host array of point ids
  int n;
  int tgt;         // 0: source points, 1: target points
  int tag;         // 0 or 1
  double za, zb;   // z in the tree's frame: za z + zb
};
struct TreeJob {
  double x0, y0, z0, S0;
  int seg0, nseg;  // segments of the tree
  // refinement rule of the boxes (for a sorter that also forms them): every
  // non-empty box above level `depth` is split, with gap_only only those
  // whose gap index j is 0 (the z index from the gap side: iz, or
  // 2^l - 1 - iz with zflip)
  int depth, gap_only, zflip;
};

// Reaction M2L in the mirror-adapted basis: the reaction M2L tensor
// commutes with the mirror that swaps the +/- channels and takes m to -m
// (with the sign (-1)^m), so it acts on the even and the odd part of a
// vector separately.  Dimension of the even (par 0) or odd (par 1) part at
// order q: the (q+1)^2 entries of the + channel, then the z-channel entries
// with m >= 0 (even) or m >= 1 (odd), both n-major.
__host__ __device__ inline int lm_sym_dim(int q, int par) {
  return (q + 1) * (q + 1) + (par == 0 ? (q + 1) * (q + 2) / 2 : q * (q + 1) / 2);
}

// One FMM instance: the free-space part of one layer, or one reaction
// component (target layer lt, source layer ls, arrival direction at the
// target, departure direction at the source).
struct InstParams {
  int kind;          // 0 free space, 1 reaction component
  int lt, ls;        // target layer, source layer
  int up_t, up_s;    // reaction: 1 if the wave arrives at the target going up / leaves the source going up
  int sgn;           // reaction sign s of the component
  int p, P;          // expansion order, (p+1)^2
  double kt, ks;     // target-side and source-side wavenumbers
  double at, bt;     // target effective location  zhat = at*z + bt
  double as, bs;     // source polarization image  zbrv = as*z + bs
  double Dgap;       // distance between the two anchor planes (reaction)
  int s2t0, s2tn;    // reaction: quadrature nodes of the direct (S2T) near field
  double s2t_rho;    // reaction: largest horizontal distance of an S2T pair (-1: none)
  int s2t_nser;      // reaction: terms of the S2T complex Bessel series (Gamma_1)
  int s2t_smallz;    // reaction: 1 if |k_rho| rho <= 7.5 on Gamma_1 for every S2T pair
};

// source-side box record (device)
struct SrcBox {
  double c[3];       // centre in image coordinates
  int pt0, pt1;      // range in the concatenated source permutation
  int inst;          // instance
  int level;
  int child0, nchild;  // children (source box ids) for M2M
  int octant;        // octant of this box inside its parent (0..7), -1 for roots
  int parent;
  long long me_off;  // offset (in complex numbers) of this box's multipole vectors
};

// target-side box record (device)
struct TgtBox {
  double c[3];
  int pt0, pt1;
  int inst;
  int level;
  int parent;
  int octant;
  int leaf;
  long long le_off;  // offset of this box's local vectors
  int p2p0, p2p1;    // free space: range in the near-box list (P2P)
};

// M2L class: a set of target boxes sharing one list of potential source
// offsets; each offset owns (per output type) a P x K matrix.
struct M2LClass {
  int inst;
  int n_off;          // number of offsets
  int off0;           // first offset record
  int n_tgt;          // number of target boxes
  int tgt0;           // first entry in the class target list
  int nblk;           // 1 (free) or 3 (reaction)
  int P;              // output/input vector length
};

struct M2LOffset {
  long long mat[3];   // per output type: offset (in complex) of the P x (nblk*P) matrix
  double phi;         // azimuth of the box-centre offset (reaction phases)
  int pord;           // order used for this offset (<= p): leading (pord+1)^2 rows/columns
  int pad_;
};

// a block of M2L work: up to a fixed number of targets of one class, with
// their (target, source) pairs sorted by offset
struct M2LBlock {
  int cls;
  int nt;             // targets in the block
  int bt0;            // first block-target record
  int q0, nq;         // pair range (global pair indices)
  int offr0;          // start of the per-offset pair ranges (n_off + 1 entries)
};

// one work tile of the M2L GEMM: one matrix (free space: one offset;
// reaction: the offsets of one table case, which differ only in azimuth),
// one output part, up to 64 rows and 64 (pair, rhs) columns; everything the
// kernel needs to start the tile in one record (no chain of dependent loads)
struct M2LTile {
  long long mat;      // offset of the tile's matrix in the tables
  long long ybase;    // scratch base of the tile's M2L block
  int qo, q0b;        // first pair of the tile's offsets; first pair of the block
  int P, p;           // (p+1)^2 and p of the class
  int R, Pb, Kf;      // rows (= columns) used, (pord+1)^2, row pitch of the stored matrix
  int ot;             // free space: output type 0..2; reaction: 0 even, 1 odd block
  int sym;            // 1: reaction (mirror-adapted blocks)
  int row0;           // first output row
  int col0, ncol;     // column range within the offset's (pair, rhs) list
};

// node of a Sommerfeld quadrature set (one per instance and level)
struct QNode {
  cd kr, w;           // node and weight (includes d kr / dt)
  cd kzt, kzs;        // vertical wavenumbers of target and source layer
  cd F[5];            // densities F_sigma = -(2i/k^2) S_sigma (no centre exponential)
  cd FH[5];           // the same slots for the curl of the field (magnetic field times mu_t)
  cd tau_t[4];        // 1, sec b, sin b, tan b for the target side
  cd tau_s[4];        // same for the source side
  cd x0;              // cos 2 b0 (base side = smaller wavenumber)
};

// one reaction M2L table case
struct TabCase {
  int inst;
  int node0, nnode;   // quadrature node range
  double rho;         // horizontal centre distance
  double zt_orig;     // target centre mapped back to physical z
  double zs_orig;     // source centre mapped back to physical z
  long long mat;      // offset of the three P x 3P matrices (A+, A-, Az)
  long long ibuf;     // offset of the Chebyshev integral buffer
};

// free-space / translation matrix job
struct TransJob {
  double b[3];        // translation vector
  double k;
  int p;
  int kind;           // 0: S|R (M2L, times ik), 1: M2M conj(R|R) transposed, 2: L2L R|R
  long long mat;      // output offset
};

std::string lm_fmt(const char* fmt, ...);
