// Batched solve of many independent single-block plans (uneven sizes, several
// right-hand sides each) as one captured HIP graph: every stage is one batched
// launch over all (plan, right-hand side) pairs.
#pragma once

#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "plan.hpp"

namespace hs {

struct Batch {
  std::vector<const Plan*> plans;
  std::vector<int> nrhs;
  int prec = 0;
  int refine_steps = 0;
  int device = 0;
  // combined tables
  std::vector<int64_t> tab_off;   // per plan, element offset of its tables
  void* dtab64 = nullptr;
  void* dtab32 = nullptr;
  void* dtab16 = nullptr;         // complex64 path: split-fp16 fragment images
  std::vector<int64_t> h16_off;   // per plan, 16-byte-unit offset of its fp16 image
  size_t tab_elems = 0;
  // workspace layout: per (plan, rhs) spectral array; complex64 residual per plan
  std::vector<int64_t> spec_off;  // per plan, first rhs (elements of the compute precision)
  std::vector<size_t> res_off;    // per plan, byte offset of its residual
  size_t ws_elems = 0, ws_bytes = 0;
  void* ws = nullptr;
  int max_nz = 0;
  int common_nz = 0;   // the plans' nz when they all share one, else 0
  int64_t max_modes = 0;
  // descriptors rebuilt when the caller's pointers change
  std::vector<const void*> last_f;
  std::vector<void*> last_u;
  std::vector<int64_t> foff, uoff;   // byte offsets of each plan's f / u from the first plan's
  StageList<XformDesc> s_fwdx, s_fwdx_res, s_invx;
  StageList<XformYDesc> s_fwdy, s_invy;
  std::vector<SweepDesc> d_sweep;
  const SweepDesc* p_sweep = nullptr;
  // complex64 path: every plan's FP64 residual in one flat launch
  std::vector<ResidualItem> d_resid;
  const ResidualItem* p_resid = nullptr;
  int64_t resid_wg = 0;
  // launch shapes of the batch (those of plans[0] until hs_batch_tune)
  int tune_chunks = 0, tune_lt = 0, tune_full = 0;
  bool recapture = false;         // launch shapes changed: capture the graph again
  // complex64: near-resonance selection of d_sweep for chunk counts 8, 16, 32
  SweepSelHost sel_host[3];
  SweepSel sel_dev[3];
  void* ddesc = nullptr;
  size_t ddesc_bytes = 0;
  // graph
  hipStream_t cap_stream = nullptr;
  SideStream side;                // complex64 path: stream of the FP64 z solves
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;

  ~Batch();
  hs_status build(const std::vector<const Plan*>& ps, const std::vector<int>& rs, std::string& err);
  hs_status bind(void* p, size_t bytes, std::string& err);
  hs_status solve(const void* const* f, void* const* u, hipStream_t st, std::string& err);
  // time the usable launch shapes on the whole captured graph with the
  // caller's arrays (u is overwritten) and keep the fastest
  hs_status tune(const void* const* f, void* const* u, const char* cache_path, hipStream_t st, std::string& err);

 private:
  hs_status rebuild(const void* const* f, void* const* u, std::string& err);
  void enqueue(const void* f0, void* u0, hipStream_t st);
  void run_x(const StageList<XformDesc>& sl, int in64, int out64, int acc, const void* src, void* dst,
             hipStream_t st);
  void run_y(const StageList<XformYDesc>& sl, hipStream_t st);
  const void* tab() const { return prec == 0 ? dtab64 : dtab32; }
};

}  // namespace hs
