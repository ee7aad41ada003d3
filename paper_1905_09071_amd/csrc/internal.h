// Library-internal helpers shared by the plan API and the serving engine.
#pragma once
#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "../../include/agg.h"
#include "kernels.h"
#include "planner.h"

namespace agg {

agg_status set_error(agg_status code, const std::string& msg);
agg_status hip_fail(hipError_t e, const char* what);

// Device allocations owned by one plan or one engine request.
struct DeviceArena {
  std::vector<void*> ptrs;
  size_t total = 0;
  agg_status alloc(size_t bytes, void** p);
  void release();
};

// Device copies of everything a kernel set needs that is shared by all the
// states using it: distinct columns, term tables, twiddles.
struct SharedTables {
  const PlanTables* tab = nullptr;
  double* cols = nullptr;
  const int* tabs = nullptr;       // int blob (see SlotDesc)
  const double* coef = nullptr;    // coefficient blob
  int Tp = 0, Tq = 0, ntab = 0, o_pids = 0, o_qoff = 0, o_qids = 0, o_qkm = 0, o_pfrom = 0;
  int nch = 0, o_chc = 0, o_chcols = 0, o_cht = 0;
  int tt = 0, o_tt = 0;
  void *twP1 = nullptr, *twP2 = nullptr, *twLlo = nullptr, *twLhi = nullptr;
};

// Host image of the shared tables, laid out for a single upload.
struct SharedImage {
  std::vector<unsigned char> bytes;
  size_t o_cols = 0, o_tabs = 0, o_coef = 0, o_tw1 = 0, o_tw2 = 0, o_twlo = 0, o_twhi = 0;
  int Tp = 0, Tq = 0, ntab = 0, o_pids = 0, o_qoff = 0, o_qids = 0, o_qkm = 0, o_pfrom = 0;
  int nch = 0, o_chc = 0, o_chcols = 0, o_cht = 0;
  int tt = 0, o_tt = 0;
};
SharedImage make_shared_image(const PlanTables& T);
void bind_shared(const SharedImage& im, void* dev, SharedTables* st);

agg_status upload(void* dst, const void* src, size_t bytes, hipStream_t s);
agg_status build_slots(const PlanTables& T, const SharedTables& st, DeviceArena& arena, int batch,
                       SlotDesc* sd, SlotStride* stride);
agg_status build_shared(const PlanTables& T, hipStream_t s, DeviceArena& arena, SharedTables* st);
// Dynamic LDS a row-pass workgroup may take, and the check that a kernel set's
// row pass fits (AGG_EUNSUPPORTED otherwise).
constexpr size_t kRowLdsLimit = 160 * 1024 - 4096;
agg_status row_lds_check(const PlanTables& T, int ntab, int ncoef);
// spread: narrow the column group g below the plan's when the launch has fewer
// column groups than CUs, and split the groups' distinct columns over several
// workgroups when that is still too few; every launch that shares a slot's
// partial dot products or Heun vectors must be built with the same choice and
// slot count (a split stage-2 launch reads the state its stage-1 launch kept).
LaunchArgs base_args(const PlanTables& T, const SharedTables& st, const SlotDesc* d_slots, int nslots,
                     bool spread = false);

// api.cpp: the plain evaluation with caller-provided per-state workspace
size_t rhs_workspace_bytes(const agg_plan* p);
agg_status rhs_in_workspace(agg_plan* p, const double* n, double* dndt, int batch, void* ws);
int plan_device(const agg_plan* p);
int plan_batch(const agg_plan* p);
bool plan_is_plain(const agg_plan* p);

// kernels.hip
hipError_t launch_col(int prec, const LaunchArgs& a, hipStream_t s);
hipError_t launch_row(int prec, const LaunchArgs& a, hipStream_t s);
hipError_t launch_moments(const double* n, int64_t total, int64_t N, double* part, int nblocks,
                          hipStream_t s);
hipError_t launch_heun(int stage, double* n, const double* k1, const double* k2, double* ntil, double dt,
                       int64_t total, hipStream_t s);
hipError_t launch_zero(double* x, int64_t total, hipStream_t s);
hipError_t launch_tick(int64_t* t, hipStream_t s);
size_t row_smem_bytes(int prec, int umax, int M2, int tab_max, int coef_max);
size_t row_chunk_smem_bytes(int prec, int cmax, int umax, int M2, int tab_max, int coef_max);
int col_batch(int prec, int M1, int u, int nworkgroups);

}  // namespace agg
