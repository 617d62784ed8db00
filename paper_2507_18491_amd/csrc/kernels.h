// kernels.h -- host-side launchers of the HIP kernels.
#pragma once
#include "../../include/lmfmm.h"
#include "lmfmm_internal.h"

struct MediumDev {
  int n;
  double d[LM_MAXL];
  double k[LM_MAXL];
  double mu[LM_MAXL];  // relative permeabilities
};

// device-side view of a built plan
struct DevPlan {
  InstParams* inst;
  SrcBox* sbox;
  TgtBox* tbox;
  long long* sbox_m2m;
  long long* tbox_l2l;
  int* src_perm;
  int* tgt_perm;
  int* p2p_list;
  M2LClass* cls;
  M2LTile* tiles;
  M2LBlock* blocks;
  int* bt_tbox;
  int* bt_ptr;
  int* bt_pairs;
  long long* pair_me;   // per pair: multipole vector offset of its source box
  int* bt_blk;          // block of each block-target
  int* pair_P;          // per pair: number of rows/columns used ((pord+1)^2)
  double* pair_phi;     // per pair: azimuth of its offset (reaction output phases)
  long long* blk_ybase; // per block: first scratch element (depends on the rhs count)
  cd* mats;        // all translation / M2L matrices
  double* gaunt;
  int gaunt_p;
  double* Bcoef;
  double* Ccoef;
  long long* Ccoef0;
  TabCase* cases;
  QNode* nodes;
  cd* ibuf;        // Chebyshev-Sommerfeld integrals
  TransJob* trans;
  int* wq;         // work-queue counters of the persistent launches (LM_WQ_*), two each
};
// counter pairs in DevPlan::wq
#define LM_WQ_P2P 0
#define LM_WQ_P2PS 2
#define LM_WQ_S2T 4
#define LM_WQ_COUNT 8

void launch_fill(cd* p, long long n, hipStream_t s);
// Keys and sorts the records of every octree on the device, and forms their
// boxes (the sorter of lm_make_plan_multi): d_src / d_tgt are the point positions on the device;
// returns "" or a message; *ms (if given) the time of the kernels.
std::string lm_device_tree_sort(const std::vector<TreeJob>& jobs, const std::vector<TreeSeg>& segs,
                                const double* d_src, const double* d_tgt, std::vector<uint64_t>& keys,
                                std::vector<uint32_t>& pay, std::vector<uint64_t>& boxes, float* ms,
                                hipStream_t s);
// uploads the Legendre recurrence coefficients to the current device (once)
int lm_upload_leg_tables();
void launch_trans(const DevPlan& d, int n_jobs, int pmax_gaunt, hipStream_t s);
void launch_nodes(const DevPlan& d, MediumDev med, int n_nodes, const int* node_inst, const cd* kr,
                  const cd* w, hipStream_t s);
void launch_tab_integrals(const DevPlan& d, MediumDev med, int case0, int ncase, int p, cd* scratch,
                          long long scratch_stride, hipStream_t s);
void launch_tab_assemble(const DevPlan& d, int case0, int ncase, int p, int KB, int BS, cd* out, long long stride,
                         hipStream_t s);
void launch_tab_sym(const DevPlan& d, int case0, int ncase, const cd* src, long long stride, hipStream_t s);
void launch_p2m(const DevPlan& d, const int* items, int n, const double* xyz, const cd* J, long long n_src,
                int n_rhs, cd* ME, cd* part, int pl, hipStream_t s);
void launch_p2m_sum(const DevPlan& d, const int* items, int n, int n_rhs, const cd* part, int Pg, cd* ME,
                    hipStream_t s);
void launch_m2m(const DevPlan& d, const int* parents, int n, int n_rhs, cd* ME, int pmax, hipStream_t s);
// tile-shape variants of the M2L GEMM kernel (LM_M2L_VARIANTS of the C ABI)
void launch_m2l(const DevPlan& d, const M2LTile* tiles, int n_tiles, int n_rhs, const cd* ME, cd* Y, int pmax,
                int variant, hipStream_t s);
void launch_m2l_reduce(const DevPlan& d, int bt0, int nbt, int n_rhs, const cd* Y, cd* LE, int pmax,
                       hipStream_t s);
void launch_l2l(const DevPlan& d, const int* children, int n, int n_rhs, cd* LE, int pmax, hipStream_t s);
void launch_l2p(const DevPlan& d, const int* leaves, int n, int kind, const double* xyz, long long n_tgt,
                int n_rhs, const cd* LE, cd* A, int pi, hipStream_t s);
void launch_p2p_sym(const DevPlan& d, const int* items, int n, const int* part, const double* xyz, const cd* J,
                    long long n_pts, int n_rhs, cd* A, cd* Ys, bool red, hipStream_t s);
void launch_p2p(const DevPlan& d, const int* tboxes, int n, const double* sxyz, const cd* J, long long n_src,
                const double* txyz, long long n_tgt, int n_rhs, cd* A, bool red, hipStream_t s);
void launch_conj(cd* out, const cd* in, long long n, hipStream_t s);
// out[r][i][c] = conj(in[r][i][c]) mu(layer of point i)^pw, pw = +1 or -1 (n points, n_rhs vectors)
void launch_conj_mu(cd* out, const cd* in, long long n, int n_rhs, const double* xyz, MediumDev md, int pw,
                    hipStream_t s);
// v[r][i][c] *= mu(layer of point i)^pw
void launch_scale_mu(cd* v, long long n, int n_rhs, const double* xyz, MediumDev md, int pw, hipStream_t s);
// magnetic field (curl of the electric field): far part from the local
// expansions, free-space near part grad g x q; both add into Hc [rhs][point][3]
void launch_l2p_curl(const DevPlan& d, const int* leaves, int n, int kind, const double* xyz, long long n_pts,
                     int n_rhs, const cd* LE, cd* Hc, int pi, hipStream_t s);
void launch_p2p_curl(const DevPlan& d, const int* tboxes, int n, const double* sxyz, const cd* J, long long n_src,
                     const double* txyz, long long n_tgt, int n_rhs, cd* Hc, bool red, hipStream_t s);
// g[i][c] *= mu(layer of point i)^pw
void launch_scale_mu_d(double* g, long long n, const double* xyz, MediumDev md, int pw, hipStream_t s);
void launch_s2t(const DevPlan& d, MediumDev md, const int* items, const int* tlist, const int* slist, int n,
                const double* sxyz, const cd* J, long long n_src, const double* txyz, long long n_tgt, int n_rhs,
                double a, bool smallz, cd* Ys, hipStream_t s, bool hfield = false);
void launch_s2t_gather(const int* gpt, const int* gptr, const int* gslot, int n_pts, int n_rhs, const cd* Ys,
                       long long n_tgt, cd* A, hipStream_t s);
// source-position gradients through the direct reaction pairs (gradient path roles)
void launch_s2t_grad(const DevPlan& d, MediumDev md, const int* items, const int* tlist, const int* slist, int n,
                     const double* sxyz, const cd* C, long long n_src, const double* txyz, const cd* W,
                     long long n_tgt, int n_rhs, double a, bool smallz, double* Gs, hipStream_t s);
void launch_s2t_gather_grad(const int* gpt, const int* gptr, const int* gslot, int n_pts, const double* Gs,
                            double* gX, hipStream_t s);
void launch_fill_d(double* p, long long n, hipStream_t s);
void launch_selftest_math(const double* x, long long n, double* out, hipStream_t s);
void launch_l2p_grad(const DevPlan& d, const int* leaves, int n, int kind, const double* xyz, long long n_pts,
                     int n_rhs, const cd* LE, const cd* W, double* gX, int pi, hipStream_t s);
void launch_p2p_grad(const DevPlan& d, const int* tboxes, int n, const double* sxyz, const cd* Jsrc,
                     long long n_src, const double* txyz, const cd* W, long long n_tgt, int n_rhs, double* gX,
                     bool red, hipStream_t s);

// vector kernels of the GMRES solve (krylov.hip); vt: device table of vector base pointers
int kv_dots_nb(long long n3, int n_rhs, int count);
void launch_kv_dots(cd* const* vt, int first, int count, int w, long long n3, int n_rhs, int nb, cd* part,
                    cd* out, hipStream_t s);
void launch_kv_combine(cd* const* vt, int first, int count, const cd* c, int dst, long long n3, int n_rhs,
                       hipStream_t s);
void launch_kv_scale(cd* const* vt, int src, const cd* c, int dst, long long n3, int n_rhs, hipStream_t s);
void launch_kv_rsub(cd* const* vt, int b, int w, long long n3, int n_rhs, hipStream_t s);
void launch_kv_diag(cd* const* vt, int src, const cd* diag, int dst, long long n3, int n_rhs, hipStream_t s);
