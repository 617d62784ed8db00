// plan.h -- host-side planner of the layered-media dyadic FMM: medium,
// reaction components, trees, interaction lists, M2L classes and table
// cases, coefficient tables.
#pragma once
#include <functional>
#include <map>
#include <string>
#include <vector>

#include "lmfmm_internal.h"

struct Medium {
  int n = 0;                 // number of layers
  double d[LM_MAXL] = {0};   // interfaces d[0] > d[1] > ... (n-1 values)
  double k[LM_MAXL] = {0};   // wavenumbers (n values)
  double mu[LM_MAXL] = {0};  // relative permeabilities (n values)
  bool mu_one = true;        // every mu is 1
  double kmax = 0;
  int layer_of(double z) const {
    int l = 0;
    while (l < n - 1 && z < d[l]) l++;
    return l;
  }
};

struct PlanParams {
  int p = 12;
  int p_free = 0;        // 0: same as p
  int free_depth = 0;    // 0: chosen by a cost model
  int max_depth = 14;    // cap of the reaction refinement
  int gamma1_panels = 4; // Gauss-Legendre panels on the Gamma_1 contour
  double contour_a = 0;  // 0: 1.5 * max k
  double tail_digits = 60;
  int components = 3;    // bit 0: free space, bit 1: reaction
  int m2l_adapt = 1;     // per-offset M2L order from the separation ratio
  double m2l_margin = 3.0;  // decades below the worst pair's truncation bound
  int react_s2t = 1;         // 0: refine reaction trees until no adjacent leaves remain;
                             // 1: stop one level early next to the gap where direct (S2T)
                             // pairs are estimated cheaper; 2: always stop one level early;
                             // 3: every reaction pair direct
  double tol = 0;            // requested accuracy: plans whose quadrature rules are coarser fail
};

// prefix of the planner's messages for a requested accuracy out of reach
#define LM_PLAN_ACCURACY_PREFIX "accuracy: "

struct Plan {
  Medium med;
  PlanParams prm;
  int p = 0, pf = 0;
  int64_t n_src = 0, n_tgt = 0;
  std::vector<InstParams> inst;
  std::vector<int> src_perm, tgt_perm;
  std::vector<SrcBox> sbox;
  std::vector<TgtBox> tbox;
  std::vector<long long> sbox_m2m;   // matrix offset (child -> parent) per source box, -1 for roots
  std::vector<long long> tbox_l2l;   // matrix offset (parent -> child) per target box, -1 for roots
  std::vector<std::vector<int>> m2m_parents;  // per level (parent level), parent box ids with children
  std::vector<std::vector<int>> l2l_children; // per level (child level), child box ids
  std::vector<int> p2m_leaves;                // source boxes doing P2M
  std::vector<std::vector<int>> l2p_leaves;   // per instance, target leaf boxes
  std::vector<std::vector<int>> p2p_tboxes;   // per free instance, near-field work items (target leaf, chunk) pairs
  std::vector<int> p2p_list;                  // near source boxes
  // M2L
  std::vector<M2LClass> cls;
  std::vector<M2LOffset> offs;
  std::vector<int> cls_tgt;                   // target box ids
  std::vector<int> cls_srcof;                 // [tgt][off] source box id or -1
  std::vector<long long> cls_srcof0;          // per class start in cls_srcof
  std::vector<M2LBlock> blocks;               // M2L work blocks
  std::vector<int> bt_tbox;                   // per block-target: target box
  std::vector<int> bt_ptr;                    // per block-target: first entry in bt_pairs (+ end)
  std::vector<int> bt_pairs;                  // pair indices, per target sorted by offset
  std::vector<int> pair_src;                  // per pair: source box
  std::vector<int> offr;                      // per block: n_off+1 pair-range starts
  std::vector<int> bt_blk;                    // per block-target: its block
  std::vector<int> pair_P;                    // per pair: (pord+1)^2 of its offset
  std::vector<double> pair_phi;               // per pair: azimuth of its offset (reaction phases)
  std::vector<int> s2t_items;                 // reaction near field: (target leaf, chunk) pairs
  // tables
  std::vector<TransJob> trans;
  std::vector<TabCase> cases;
  std::vector<cd> node_kr, node_w;            // quadrature nodes (kr, weight)
  std::vector<int> node_inst;                 // instance of each node
  std::vector<double> Bcoef;                  // [n][m][k] Chebyshev coefficients of P^m_n / tau
  std::vector<double> Ccoef;                  // per instance [j][s]
  std::vector<long long> Ccoef0;              // per instance offset
  std::vector<double> gaunt;                  // Gaunt table for the translations
  int gaunt_p = -1;
  long long me_size = 0, le_size = 0, mat_size = 0, ibuf_size = 0;
  int kmaxcheb = 0;                           // max Chebyshev index K
  // statistics
  long long n_m2l_pairs = 0, n_p2p_pairs = 0, n_m2l_pairs_free = 0, n_m2l_pairs_react = 0, n_s2t_pairs = 0;
  int n_free_inst = 0, n_react_inst = 0;
  std::vector<int> free_depth_used;
};

// builds the whole plan; returns "" on success or an error message
std::string lm_make_plan(Plan& pl, const Medium& med, const PlanParams& prm, int64_t n_src,
                         const double* src, int64_t n_tgt, const double* tgt);

// Host threads of the planner and of the build's list construction: the
// LMFMM_HOST_THREADS environment variable (1..256) when set, else the
// hardware's count up to 16.  Plans and lists do not depend on it.
unsigned lm_host_thread_count();

// several independent geometries in one plan: geometry g owns sources
// src_off[g] .. src_off[g+1]-1 and targets tgt_off[g] .. tgt_off[g+1]-1 (global
// indices into src / tgt); each gets its own lattice and FMM instances, and
// only same-geometry pairs interact.  With `sorter`, the records of every
// octree are keyed and sorted by it, all trees in one call (lm_build does it
// on the device), instead of on the host; the plan is the same.
using TreeSorter = std::function<std::string(const std::vector<TreeJob>& jobs, const std::vector<TreeSeg>& segs,
                                             std::vector<uint64_t>& keys, std::vector<uint32_t>& pay,
                                             std::vector<uint64_t>& boxes)>;
std::string lm_make_plan_multi(Plan& pl, const Medium& med, const PlanParams& prm, int n_geom,
                               const int64_t* src_off, const double* src, const int64_t* tgt_off,
                               const double* tgt, const TreeSorter* sorter = nullptr);

// small helpers exported for host-only tests
void lm_cheb_affine(int jmax, double a, double b, std::vector<double>& C);
void lm_legendre_cheb(int p, std::vector<double>& B);
int lm_cheb_K(int n, int m);
int lm_tau_type(int n, int m);
void lm_gaunt_table(int p, std::vector<double>& G);
long long lm_gaunt_index(int p, int nu, int mu, int n, int m, int q);
int lm_enumerate_components(const Medium& med, std::vector<InstParams>& out);
