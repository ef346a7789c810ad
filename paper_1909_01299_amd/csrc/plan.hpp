// Host plan of the separable Helmholtz solver: grid, blocks, FP64 tables,
// workspace layout, stage descriptors and the enqueue logic of one solve.
#pragma once

#include <hip/hip_runtime.h>

#include <complex>
#include <string>
#include <vector>

#include "../../include/helmsep.h"
#include "common.hpp"
#include "eig.hpp"
#include "kernels.hpp"

namespace hs {

struct Axis {
  int n = 0;
  bool sine = false;
  int dstV = 0;                        // > 0: sine transform by FFT with V = (n + 1) / 16
  bool real_tables = false;            // uniform axis: W and W^{-1} are real sine matrices
  AxisEig e;
  int64_t fwd = 0, inv = 0, lam = 0;   // table offsets (complex elements)
  int64_t ffwd = 0, finv = 0;          // the same tables as MFMA fragments of their real embedding
  int64_t rfwd = -1, rinv = -1;        // uniform axes (real sine tables): fragments of the tables themselves
  // complex64 path: the matrix-core tables (real or embedded, as above) as
  // split-fp16 fragments (16-byte units in the fp16 image; -1: none) and the
  // inverses of their scales
  int64_t hfwd = -1, hinv = -1;
  float hsfwd = 1.f, hsinv = 1.f;
};

// Matrix-core table of a dense descriptor: the real table where the axis has
// one, else the real embedding of the complex table (offsets + base).
template <typename D>
inline void set_frag(D& d, const Axis& a, bool fwd, int64_t base = 0, int64_t hbase = 0) {
  const bool real = a.rfwd >= 0;
  d.real_tab = real ? 1 : 0;
  d.ftab = base + (real ? (fwd ? a.rfwd : a.rinv) : (fwd ? a.ffwd : a.finv));
  const int64_t h = fwd ? a.hfwd : a.hinv;
  d.htab = h >= 0 ? hbase + h : -1;
  d.hsinv = fwd ? a.hsfwd : a.hsinv;
}

struct Block {
  int bi = 0, bj = 0;            // block column / row
  int x0 = 0, nbx = 0, y0 = 0, nby = 0;
  int ax = -1, ay = -1;          // axis table indices
  int sep_lo_x = -1, sep_hi_x = -1, sep_lo_y = -1, sep_hi_y = -1;
  int rs = 0;                    // row stride of its spectral arrays (spectral_row(nbx))
  int64_t pplane = 0;            // z-plane stride of its spectral arrays (spectral_plane(nby*rs))
  int64_t spec = 0;              // workspace offset of the block spectral array
  int64_t vt = 0;                // workspace offset of its spectral block solution v~ (steps 2-3)
  int64_t cpart = 0;             // slab partial sums of its face contraction (split planes only)
};

// One transform stage: dense-table descriptors plus sine-FFT descriptors per V.
constexpr int kNumV = 6;   // V = 1, 2, 4, 8, 16, 32
template <typename DenseDesc>
struct StageList {
  std::vector<DenseDesc> dense;
  std::vector<DstDesc> dst[kNumV];
  const DenseDesc* p_dense = nullptr;
  const DstDesc* p_dst[kNumV] = {};
  int max_lines[kNumV] = {};
};

struct StageProf {
  std::string name;
  double ms = 0;
  int64_t launches = 0;
  double bytes = 0, flops = 0;   // per launch, algorithmic
};

struct Plan {
  // ---------------- grid
  int NX = 0, NY = 0, NZ = 0, nlayers = 0;
  std::vector<cd> hx, hy;
  std::vector<double> hz;
  std::vector<int32_t> layer;
  std::vector<cd> k2;
  std::vector<double> sig_node, sig_step;   // sigma(z) at the z nodes and steps (ones when not given)
  std::vector<int32_t> sepx, sepy;
  int prec = 0;          // 0 = complex128, 1 = complex64 + FP64 refinement
  int refine_steps = 0;
  double tol = 0;        // > 0: every solve checks the residual of its result
  int max_rhs = 1;
  int flags = 0;
  int device = 0;
  double plan_seconds = 0;

  // ---------------- tables
  std::vector<Axis> axes;
  int gax = -1, gay = -1;        // global axes (decomposed grids)
  std::vector<Block> blocks;
  int nbx_blocks = 1, nby_blocks = 1;
  bool decomposed = false;
  bool dense_glob = false;        // the global right-hand side is expanded densely (else low-rank terms in the z solve)
  bool glob_forced = false;       // dense expansion required: more than kMaxTerms separators on an axis, or flag bit 3
  // separators of one axis in the largest interface-contraction descriptor;
  // every descriptor of that launch is split for this count
  int sig_terms() const {
    return int(std::min<size_t>(std::max(sepx.size(), sepy.size()), size_t(kMaxContractTerms)));
  }
  std::vector<cd> htab;          // host FP64 table image
  std::vector<_Float16> h16;     // complex64 path: split-fp16 fragment image (8 halves per unit)
  int64_t zlo = 0, zdiag = 0, zup = 0, zsig = 0;
  int64_t cx_lo = 0, cx_hi = 0, cy_lo = 0, cy_hi = 0;
  int64_t ex_cx = 0, ex_cy = 0;  // dense_glob: W_x^{-1}[a][s_i] as [i][a], W_y^{-1}[b][t_j] as [j][b]
  std::vector<int64_t> lift_cf;  // per block 4 coefficient offsets
  void* dtab64 = nullptr;
  void* dtab32 = nullptr;
  void* dtab16 = nullptr;
  size_t tab_elems = 0;
  int32_t* dint = nullptr;       // sep_x | sep_y | xblk | xloc | yblk | yloc | layer_of_z
  int64_t i_sepx = 0, i_sepy = 0, i_xblk = 0, i_xloc = 0, i_yblk = 0, i_yloc = 0, i_layer = 0;
  double2* dsten = nullptr;      // FP64 stencil arrays
  StencilGeom sten{};
  double min_pivot = 0;
  int tune_chunks = 0;           // z-line chunks per mode (0 = default for NZ)
  int tune_lt = 0;               // sine-transform lines per workgroup (0 = default)
  int tune_full = 0;             // 1: z solves with chunks of a fixed row count where nz fills them
  int tune_side = 1;             // complex64: FP64 z solves on a second stream (1) or before the FP32 launch (0)
  double fp64_below = -1e300;    // complex64 path: z solves of modes with Re(lam_x + lam_y) <= this in FP64
  SideStream side;               // complex64 path: stream of the FP64 z solves
  int64_t n_fp64_modes = 0;

  // ---------------- workspace (layout for max_rhs)
  size_t ws_elems = 0;           // compute-precision complex elements
  size_t ws_bytes = 0;
  size_t off_d64 = 0;            // byte offset of the FP64 region
  size_t off_res = 0;            // byte offset of the complex64 residual (mixed)
  size_t off_gpart = 0;          // byte offset of the gradient's slice sums
  size_t off_npart = 0;          // byte offset of the residual kernel's workgroup sums
  size_t off_norms = 0;          // byte offset of the residual norms [eval][r][3]
  int64_t n_rwg = 0;             // residual workgroups per right-hand side
  // convergence record of the last solve (host side: what the workspace holds)
  int last_nrhs = 0, last_evals = 0;
  bool last_final = false;       // the last evaluation is of the returned u
  void* ws = nullptr;
  int NF = 0;
  int64_t w_face = 0, w_vface = 0, w_gface = 0, w_Gface = 0;
  int64_t w_rx = 0, w_ry = 0, w_Rx = 0, w_Ry = 0, w_Qx = 0, w_Qy = 0, w_wx = 0, w_wy = 0;
  int64_t w_gspec = 0;           // global spectral solution w~ of the interface solve
  int grs = 0;                   // its row stride
  int64_t gpplane = 0;           // its z-plane stride
  int64_t w_cpart = 0;           // slab partial sums of the interface contraction (split plane only)
  ExpandDesc ex{};               // dense_glob: dense spectral right-hand side of the global solve
  // nested partitions: the interface problem of Alg. step 5 solved by the
  // cyclic reduction of a coarser plan (its separators a subset of these)
  Plan* coarse = nullptr;
  int64_t w_F = 0;               // coarse: the interface residual scattered onto the grid [R][nz][ny][nx]
  size_t off_W = 0;              // coarse: byte offset of its solution (complex128, same layout)

  // ---------------- descriptors (device copies in one buffer)
  void* ddesc = nullptr;
  size_t ddesc_bytes = 0;
  StageList<XformDesc> s_fwdx, s_invx;
  StageList<XformYDesc> s_fwdy, s_invy;
  std::vector<XformDesc> d_vface, d_gface, d_glob_in, d_glob_out;
  int64_t twid = 0;                  // twiddle table offset
  std::vector<SweepDesc> d_sweep, d_sweepB, d_sweepC, d_sweepG;
  std::vector<ContractDesc> d_face, d_sig;
  ContractLaunch cl_face, cl_sig;
  std::vector<LiftBlock> d_lift;
  // device pointers of each list
  const XformDesc *p_vface = nullptr, *p_gface = nullptr, *p_glob_in = nullptr, *p_glob_out = nullptr;
  const SweepDesc *p_sweep = nullptr, *p_sweepB = nullptr, *p_sweepC = nullptr, *p_sweepG = nullptr;
  // complex64: near-resonance selections of the four sweep lists (d_sweep,
  // d_sweepB, d_sweepC, d_sweepG) for chunk counts 8, 16, 32 (device copies
  // in the descriptor buffer; rebuilt with the FP64 threshold)
  SweepSelHost sel_host[4][3];
  SweepSel sel_dev[4][3];
  const ContractDesc *p_face = nullptr, *p_sig = nullptr;
  const LiftBlock* p_lift = nullptr;
  SigmaGeom sg{};
  int64_t max_modes_blk = 0;
  int max_block_n = 0;

  // ---------------- per-stage event timing
  bool prof_on = false;
  std::string prof_only;   // non-empty: only this stage records events
  std::vector<StageProf> prof;
  std::vector<hipEvent_t> ev_pool;
  std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> ev_pending;
  size_t ev_next = 0;
  int cur_stage = -1;
  hipStream_t cur_stream = nullptr;
  hs_status profile_enable(bool on, std::string& err);
  hs_status profile_read(hs_stage_time* out, int max_out, int* n_out, std::string& err);
  void stage_begin(const char* name, double bytes, double flops, hipStream_t st);
  void stage_end();

  ~Plan();
  hs_status build(const hs_grid* g, const hs_blocks* b, const hs_options* o, std::string& err);
  hs_status set_k2(const double* k2v, std::string& err);
  hs_status bind(void* p, size_t bytes, std::string& err);

  hs_status solve(const void* f, void* u, int nrhs, hipStream_t st, std::string& err);
  hs_status solve_adjoint(const void* g, void* a, int nrhs, hipStream_t st, std::string& err);
  hs_status grad_k2(const void* u, const void* a, void* grad, int nrhs, hipStream_t st, std::string& err);
  // the same with the partial sums in the library's static device scratch
  hs_status grad_k2_noalloc(const void* u, const void* a, void* grad, int nrhs, hipStream_t st, std::string& err);
  hs_status residual(const void* f, const void* u, void* r, int apply_only, int nrhs, hipStream_t st,
                     std::string& err);
  hs_status tune(int nrhs, const char* cache_path, hipStream_t st, std::string& err);
  // form of the global interface solve's right-hand side (decomposed grids):
  // dense expansion or low-rank terms; waits for the device, rebuilds descriptors
  hs_status set_global_dense(bool dense, std::string& err);
  // attach (or detach with nullptr) the coarser plan of a nested partition;
  // re-lays out the workspace and unbinds it
  hs_status set_coarse(Plan* c, std::string& err);
  // relative residuals of the last solve, [eval][r] (synchronous copy)
  hs_status residuals(std::vector<double>& rel, int& evals, int& nrhs, std::string& err) const;

  // one pass of the block (or decomposed) solver in compute precision
  void solve_pass(const void* f, int in64, void* u, int acc, int nrhs, hipStream_t st);

 private:
  hs_status build_tables(std::string& err);
  void build_z_tables();
  void build_stencil_host(std::vector<double2>& out);
  void layout_workspace();
  void build_descriptors();
  hs_status upload(std::string& err);
  hs_status upload_descs(std::string& err);
  // modes a sweep launch over the list provisions (largest sweep_modes_bound)
  static int64_t sweep_modes(const std::vector<SweepDesc>& v);
  void set_fp64_threshold();
  hs_status scan_pivots(std::string& err);
  const void* tab() const { return prec == 0 ? dtab64 : dtab32; }
  void run_x(const StageList<XformDesc>& sl, int in64, int out64, int acc, const void* src, void* dst, int nrhs,
             hipStream_t st);
  void run_y(const StageList<XformYDesc>& sl, int nrhs, hipStream_t st);
};

}  // namespace hs
