// Launch interface between the host plan and the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <complex>
#include <functional>
#include <string>
#include <vector>

#include "common.hpp"

namespace hs {

// Geometry of the separator lines and block faces used by the interface
// kernels.  Offsets (complex elements) index the workspace; `coef` points at
// the table buffer of the compute precision and cx_lo... index it.
struct SigmaGeom {
  int32_t NX, NY, nz, nsx;
  int32_t nsy, NF, rmax, nbx_blocks;
  int64_t f_r;                    // elements per right-hand side of f / u
  int64_t face, face_f;           // face arrays [blk][r][4][nz][NF], face_f = nz * NF
  int64_t gface;                  // lifted face data, same layout
  int64_t rx, ry;                 // residual on separator lines [r][s][nz][NY] / [r][t][nz][NX]
  int64_t wx, wy;                 // w on separator lines, same layout
  const int32_t* sep_x;
  const int32_t* sep_y;
  const int32_t* xblk;            // global x -> block column or -1 on a separator
  const int32_t* xloc;            // global x -> local index in its block
  const int32_t* yblk;
  const int32_t* yloc;
  const void* coef;
  int64_t cx_lo, cx_hi, cy_lo, cy_hi;   // coefficient offsets per separator
  int64_t zsig;                         // offset of sigma at the z nodes (scales the x / y couplings)
};

struct LiftBlock {
  int32_t x0, y0, nbx, nby;
  int32_t sep_lo_x, sep_hi_x, sep_lo_y, sep_hi_y;   // separator index or -1 (wall)
  int64_t cfx[2], cfy[2];                            // coefficient offsets (in `coef`)
};

struct StencilGeom {
  int32_t nx, ny, nz, pad_;
  const double2 *xd, *xl, *xu;
  const double2 *yd, *yl, *yu;
  const double2 *zd, *zl, *zu;
  const double2 *mx, *my, *mz;
  const double2* sg;   // sigma at the z nodes (real parts): scales the x and y terms of a plane
};

// Dense transforms (xform_mfma.hip): matrix cores for long lines in numbers
// that fill the chip, complex FMA tiles otherwise; the choice and the grid
// come from the host copy of the descriptor list.
struct LinesLaunch {
  int tiles = 0;
  bool mfma = false;
  bool real = false;   // matrix cores with a real table (descriptors with real_tab)
  int tm = 1;          // complex FMA tiles: 16 tm x 16 tm outputs per workgroup
};
bool xform_lines_use_mfma(const XformDesc& d);
LinesLaunch xform_lines_launch(const XformDesc* host_descs, int ndesc, bool mfma, bool real);
void xform_lines(int prec, int in64, int out64, int acc, const XformDesc* d, int ndesc, const LinesLaunch& L,
                 const void* tab, const void* src, void* dst, int nrhs, hipStream_t st);
// y planes on matrix cores: 32 <= n <= 256 (complex128) or 512 (complex64)
bool xform_y_use_mfma(int prec, int n);
int xform_y_mfma_tiles(const XformYDesc& d);
void xform_y_mfma(int prec, const XformYDesc* d, int ndesc, int max_n, int max_tiles, const void* tab, void* ws,
                  int nrhs, hipStream_t st, bool real);
// Lists of dense descriptors are partitioned once (matrix-core descriptors
// first, order otherwise kept; the count is returned) and launched in two
// parts, so a block takes the same kernel in any list it belongs to.
int partition_lines(std::vector<XformDesc>& v);
int partition_y(int prec, std::vector<XformYDesc>& v);
// htab: split-fp16 fragment tables (complex64 path; descriptors with htab >= 0)
void run_lines_list(int prec, int in64, int out64, int acc, const XformDesc* dev, const std::vector<XformDesc>& host,
                    const void* tab, const void* htab, const void* src, void* dst, int nrhs, hipStream_t st);
void run_y_list(int prec, const XformYDesc* dev, const std::vector<XformYDesc>& host, const void* tab,
                const void* htab, void* ws, int nrhs, hipStream_t st);
// Fragment image of an n_out x n_in complex table (row-major): real values,
// mfma_table_reals(n_out, n_in) of them.
int64_t mfma_table_reals(int n_out, int n_in);
void mfma_table_build(const std::complex<double>* T, int n_out, int n_in, double* out);
// Fragment image of a real table (the real parts of T): mfma_rtable_reals of them.
int64_t mfma_rtable_reals(int n_out, int n_in);
void mfma_rtable_build(const std::complex<double>* T, int n_out, int n_in, double* out);

// Complex64 dense transforms on fp16 matrix cores with a two-term split
// (xform_h3.hip): tables of at most 256 complex (512 real) points per axis.
bool h3_fits(int n, bool real);
int64_t h3_table_frags(int n_out, int n_in, bool real);   // 16-byte units
// writes h3_table_frags * 8 halves; returns 1 / the table's power-of-two scale
float h3_table_build(const std::complex<double>* T, int n_out, int n_in, bool real, _Float16* out);
// panel width class of a descriptor (4: rows of at most 256 halves, else 2);
// lists are grouped by it so each launch takes the widest panel it can
int h3_width(const XformDesc& d);
int h3_width(const XformYDesc& d);
void xform_lines_h3(int in64, int out64, int acc, const XformDesc* dev, const XformDesc* host, int ndesc,
                    const void* htab, const void* src, void* dst, int nrhs, hipStream_t st);
void xform_y_h3(const XformYDesc* dev, const XformYDesc* host, int ndesc, const void* htab, void* ws, int nrhs,
                hipStream_t st);

constexpr size_t kMaxLdsBytes = 163840;   // LDS of one workgroup on gfx950
// Sine transform of lines of n = 16 V - 1 points (V in {1, 2, 4, 8, 16, 32}).
constexpr int kTwiddleN = 1024;
// lt: lines per workgroup (4, 8 or 16; 0 or an unusable value = default)
void dst_lines(int prec, int in64, int out64, int acc, int V, const DstDesc* d, int ndesc, int max_lines,
               const void* tw, const void* src, void* dst, int nrhs, hipStream_t st, int lt = 0);
int dst_lines_per_wg(int prec, int V);
bool dst_lt_ok(int prec, int V, int lt);

void xform_y(int prec, const XformYDesc* d, int ndesc, int max_n, int max_tiles16, int max_tiles8,
             const void* tab, void* ws, int nrhs, hipStream_t st);
int xform_y_ppw(int prec, int max_n, int ct);
int xform_y_tiles(const XformYDesc& d, int ct, int ppw);

// z solves: LDS of one workgroup (z tables + chunk-end exchange), and the
// batched launch over descriptors (max_modes = largest sweep_modes_bound(na, nb)).
size_t sweep_lds_bytes(int arith_bytes, int nz, int chunks, int max_xterms);
// z-plane stride of a spectral array of n = na*nb modes: planes of 1024
// modes or more are padded to an odd multiple of 16 elements, so that the z
// solves' tiles of 16 consecutive modes start on whole 128-byte lines in both
// precisions and consecutive planes do not map to one memory channel; smaller
// planes stay dense (their padding would cost more than it saves).
// row stride of a spectral array of rows of na modes: a multiple of 16
// elements where that adds at most one element in eight, else na.
inline int spectral_row(int na) {
  const int r = (na + 15) / 16 * 16;
  return (r - na) * 8 <= na ? r : na;
}
inline int64_t spectral_plane(int64_t n) {
  if (n < 1024) return n;
  int64_t q = (n + 15) / 16;
  if ((q & 1) == 0) ++q;
  return 16 * q;
}
constexpr int kMaxNz = 512;    // 32 chunks of 16 rows; keeps the LDS within 64 KiB
// chunks: z-line chunks per mode (8, 16 or 32, each at most 16 rows; 256 / chunks
// modes per workgroup); 0 or an unusable value = default for max_nz
// max_xterms: largest number of x-type low-rank terms over the descriptors;
// side: a second stream (default priority) and two events; when given, the
// FP64 launch runs on it beside the FP32 one (disjoint modes), joined before
// sweep returns, so its few long workgroups overlap the bulk launch.
struct SideStream {
  hipStream_t st = nullptr;
  hipEvent_t fork = nullptr, join = nullptr;
};
// Near-resonance selection of a complex64 sweep launch for one chunk count:
// the (descriptor, workgroup) pairs whose workgroup holds a mode with
// Re(lam_x + lam_y) <= its descriptor's fp64_below (run by the FP64 launch),
// and the same as one bit per workgroup (skipped by the FP32 launch), `words`
// 32-bit words per descriptor.  Device pointers; n = 0: no FP64 launch.
struct SweepSel {
  const int2* list = nullptr;
  const uint32_t* bits = nullptr;
  int n = 0, words = 0;
};
struct SweepSelHost {
  std::vector<int2> list;
  std::vector<uint32_t> bits;
  int words = 0;
};
// chunk count a sweep launch uses for a requested one (0 or unusable: default)
int sweep_effective_chunks(int chunks, int max_nz);
// workgroups along x of a sweep launch
int sweep_grid_x(int64_t max_modes, int chunks);
// host: selection of descriptors d[0..ndesc) for the launch shape of
// (max_modes, chunks); lam_re(off) is the real part of the FP64 table at off
void sweep_select(const SweepDesc* d, int ndesc, int64_t max_modes, int chunks,
                  const std::function<double(int64_t)>& lam_re, SweepSelHost& out);
// sel: complex64 only, three selections (chunk counts 8, 16, 32) or NULL (no
// mode in FP64)
// full_nz: the common nz of every descriptor (0 when they differ); when it
// fills the chunks' register rows exactly, the kernel takes fixed-length rows
void sweep(int prec, const SweepDesc* d, int ndesc, int64_t max_modes, int max_nz, int max_xterms, const void* tab,
           const void* tab64, void* ws, int nrhs, hipStream_t st, int chunks, const SweepSel* sel,
           const SideStream* side = nullptr, int full_nz = 0);
// creates / destroys a SideStream on the current device (false on failure)
bool side_stream_create(SideStream& s);
void side_stream_destroy(SideStream& s);
int sweep_default_chunks(int nz);
// modes a launch provisions for one descriptor of nb rows of row stride rs (>= na)
inline int64_t sweep_modes_bound(int rs, int nb) { return (int64_t)nb * ((rs + 31) / 32 * 32); }
bool sweep_chunks_ok(int chunks, int nz);
// true when nz fills `chunks` chunks of a fixed register row count exactly
bool sweep_rows_fixed(int chunks, int nz);

// Fused two-axis contractions of spectral arrays (each array read once).
// contract_split chooses the column and row slabs of a descriptor (ncs, cols,
// nslab, rows) from its plane size and its term count (at least `terms`:
// every descriptor of one launch must be split with the launch's largest
// count); contract_launch gathers the launch shape of a descriptor list.
struct ContractLaunch {
  int ndesc = 0, max_slab = 1, max_cs = 1, smax = 1, max_nz = 0;
  int max_terms = 0;       // most x or y terms of one descriptor
  int64_t fin_units = 0;   // largest count of slab sums of a split descriptor (0: none split)
  size_t lds = 0;          // dynamic LDS bytes
};
void contract_split(ContractDesc& d, int terms = 0);
ContractLaunch contract_launch(const ContractDesc* d, int ndesc, int prec);
void contract(int prec, const ContractDesc* d, const ContractLaunch& L, const void* tab, void* ws, int nrhs,
              hipStream_t st);

void expand(int prec, const ExpandDesc& e, const void* tab, void* ws, int nrhs, hipStream_t st);
void sigma_resid(int prec, int in64, const SigmaGeom& g, const void* f, void* ws, int nrhs, hipStream_t st);
void lift(int prec, const SigmaGeom& g, const LiftBlock* lb, int nblocks, void* ws, int nrhs,
          hipStream_t st);
void sigma_scatter(int prec, int acc, const SigmaGeom& g, const void* ws, void* u, int nrhs, hipStream_t st);
// nested partitions: zero F (f_off elements into ws, nrhs grid arrays) and
// scatter the separator residual onto it; read W (complex128) back onto the
// separator lines wx / wy
void ml_scatter(int prec, const SigmaGeom& g, void* ws, int64_t f_off, int nrhs, hipStream_t st);
void ml_gather(int prec, const SigmaGeom& g, const void* W, void* ws, int nrhs, hipStream_t st);

// One plan's residual in a batched launch: its stencil, the element offsets of
// its f, u (complex128) and r (complex64) from the launch's base pointers, its
// right-hand sides; gx, gy, wg0 are filled by residual_list_items.
struct ResidualItem {
  StencilGeom g;
  int64_t f, u, r;
  int32_t nrhs, gx, gy, pad_;
  int64_t wg0;
};
// sets gx, gy, wg0 of every item; returns the total number of workgroups
int64_t residual_list_items(std::vector<ResidualItem>& items);
void residual_list(const ResidualItem* dev, int n, int64_t total_wg, const void* f0, const void* u0, void* r0,
                   hipStream_t st);
// part (may be NULL): 3 * residual_workgroups(g) * nrhs doubles of workgroup
// sums; norms (with part): 3 * nrhs doubles, per right-hand side |r|^2,
// |f|^2, |u|^2 summed in a fixed order; write_out = 0 stores no r.
int64_t residual_workgroups(const StencilGeom& g);
void residual(const StencilGeom& g, const void* f, const void* u, void* out, int out64, int apply_only,
              int nrhs, hipStream_t st, double* part = nullptr, double* norms = nullptr, int write_out = 1);
void conj_mass(const StencilGeom& g, const void* in, void* out, int inverse, int nrhs, hipStream_t st);
// Layer gradient grad[r][l] = sum over layer l of a * conj(u): slice partials
// of every z plane into `part` (grad_partials(plane, nz, nrhs) complex128
// values, all overwritten), then per-layer sums in a fixed order.
int grad_slices(int64_t plane, int nz, int nrhs);
// The allocation-free gradient keeps its partials in a static device array of
// kGradScratchElems complex128 values; grad_scratch_init (current device =
// `device`, once per device, at plan creation) looks up its device address,
// grad_scratch_ptr returns it (NULL before init).
constexpr int64_t kGradScratchElems = 65536;
constexpr int kMaxDevices = 64;
bool grad_scratch_init(int device, std::string& err);
void* grad_scratch_ptr(int device);
int64_t grad_partials(int64_t plane, int nz, int nrhs);
void grad_layers(int64_t plane, int nz, int nlayers, const int* layer_of_z, const void* a, const void* u,
                 void* part, void* grad, int nrhs, hipStream_t st);

}  // namespace hs
