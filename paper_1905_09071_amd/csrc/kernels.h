// Shared host/device definitions of the RHS pipeline.
//
// The right-hand side is computed with real transforms of length L carried by
// complex transforms of length M = L/2 (even/odd packing), each split as
// M = M1*M2 (four-step).  Index conventions:
//   time side:  j = j2 + M2*j1   (z[j] = x[2j] + i x[2j+1], x indexed by size)
//   frequency:  k = k1 + M1*k2
// Buffers per state (slot):
//   Z1[c][k1][j2]  forward column transforms of the u weighted columns, already
//                  multiplied by w_M^(j2*k1)
//   V [k1][j2]     inverse row transforms of the combined spectrum, multiplied by
//                  w_M^(-j2*k1)
// The column kernel turns V into the gain term, adds the loss term, applies the
// requested state update and (optionally) starts the next evaluation by forming
// and transforming the weighted columns of the new state.  The row kernel does
// everything between the two column passes.
#pragma once
#include <cstdint>

namespace agg {

// What the column kernel does for a slot.
enum ColMode : int {
  CM_NONE = 0,      // nothing
  CM_FWD = 1,       // forward only, from the state
  CM_RHS = 2,       // inverse + epilogue: out = f(state)
  CM_H1 = 3,        // inverse + epilogue: k1 = f(n), n~ = n + dt k1, forward of n~
  CM_H2 = 4,        // inverse + epilogue: n <- n + dt/2 (k1 + f(n~))
  CM_H2_FWD = 5,    // as CM_H2, then forward of the new n
  CM_RHS_ACC = 6,   // inverse + epilogue: out += f(state)  (term-by-term evaluation)
};

__host__ __device__ inline bool mode_has_inverse(int m) { return m >= CM_RHS; }
__host__ __device__ inline bool mode_writes_rhs(int m) { return m == CM_RHS || m == CM_RHS_ACC; }
__host__ __device__ inline bool mode_has_forward(int m) { return m == CM_FWD || m == CM_H1 || m == CM_H2_FWD; }

struct SlotDesc {
  double* n_state;        // state (used when the launch passes no external state)
  double* k1;             // Heun stage-1 slope, N
  double* ntil;           // Heun stage-1 state n~, N
  double* nprev;          // the state at Heun stage 1 (column order): read by stage 2 of
                          //   launches whose column groups are split (LaunchArgs::usplit)
  const double* cols;     // u distinct factor columns, N each (binary64)
  void* Z1;               // u*M stored complex values
  void* V;                // M stored complex values
  double* dots;           // u*ngroups partial dot products (column kernel -> row kernel)
  double* G;              // u loss-term weights of the current evaluation
  // term tables, one int blob: p_off[Tp+1] | p_ids | q_off[Tq+1] | q_ids | q_kmode[Tq] | p_from[Tp]
  // | ch_coff[nch+1] | ch_cols | ch_toff[nch+1]
  // (p_from[t] > p_off[t]: gain term t extends term t-1, whose ids are its prefix)
  // (offsets below), and one binary64 blob: p_coef[Tp] (mult/d!) | q_coef[Tq] (mult/(d-1)!).
  // With row-pass chunks (nch > 0) the gain terms are listed chunk by chunk,
  // chunk h owning terms [ch_toff[h], ch_toff[h+1]) and columns
  // ch_cols[ch_coff[h] .. ch_coff[h+1]), and p_ids hold positions in that list.
  const int* tab;
  const double* coef;
  int ntab, o_pids, o_qoff, o_qids, o_qkm, o_pfrom;
  int nch, o_chc, o_chcols, o_cht;
  int N, u, Tp, Tq;
  int mode;               // per-slot column mode (when the launch mode is < 0)
  int row_on;             // per-slot row pass switch (when the launch mode is < 0)
  double dt;              // per-slot step (when the launch mode is < 0); the step
                          //   of a solve's full steps (launches with a tick counter)
  double* out;            // per-slot RHS output (CM_RHS without external output)
  // solves driven by a device tick counter (LaunchArgs::tick): the slot's stage
  // is tick - start_tick (0: forward pass of n(0); 2s+1, 2s+2: the two Heun
  // stages of step s < nsteps; anything else: nothing), the last step takes
  // dt_last
  int64_t start_tick;
  int64_t nsteps;
  double dt_last;
  // kernels in tensor-train form: number of chain terms (0: CP terms) and the
  // offset of the core records in the int blob (7 ints per core: term, lambda,
  // d, r_in, r_out, offset of its chunk-local ids, offset of its global ids;
  // with nch chunks whose ch_toff ranges are core ranges); the coefficient blob
  // holds 1/d! and 1/(d-1)! per chain term
  int tt;
  int o_tt;
};

// Byte strides between consecutive slots' buffers when every slot of a launch
// shares one kernel set and its buffers are carved from batched allocations.
struct SlotStride {
  int64_t k1, ntil, Z1, V, dots, G, nprev;
};

struct LaunchArgs {
  const SlotDesc* slots;  // per-slot descriptors in device memory, or nullptr:
  SlotDesc base;          //   then slot s is base with its buffers moved by s*stride
  SlotStride stride;
  int nslots;
  int mode;               // >= 0: same mode for all slots; < 0: per slot
  double dt;
  double* ext_state;      // batch-contiguous state (nullptr: slot n_state)
  double* ext_out;        // batch-contiguous RHS output (CM_RHS)
  const void* twP1;       // w_{M1}^e, e < M1
  const void* twP2;       // w_{M2}^e, e < M2
  const void* twLlo;      // w_L^a,       a < 2^b
  const void* twLhi;      // w_L^(a 2^b), a < L/2^b
  int M1, M2, g, b;
  int lgg;                // log2(g)
  int64_t L;
  int umax;               // largest u among the slots (row kernel LDS sizing)
  int cmax;               // > 0: slots combine chunk by chunk, at most cmax columns each
  int ub;                 // forward columns transformed together in the column pass
  int tab_max;            // largest term-table int blob among the slots
  int coef_max;           // largest coefficient blob (Tp + Tq) among the slots
  int lean;               // column pass variant for launches that fill the GPU
  int usplit;             // column pass: workgroups sharing one column group's distinct
                          //   columns (1: one workgroup per group)
  double tilt;            // binary32 spectra: inputs weighted by exp(tilt s), gain by exp(-tilt s) (0: off)
  // serving launches (captured once, replayed every tick): logical slot s of
  // the launch is table entry active[1 + s] while s < active[0] (its workgroups
  // exit otherwise), and each slot's stage follows from *tick (mode < 0)
  const int* active;
  const int64_t* tick;
};

constexpr int kColBatch = 4;             // upper bound of LaunchArgs::ub
constexpr int kColThreads = 512;         // threads of a column-pass workgroup
constexpr int kChunkThreads = 512;       // threads of a chunked row-pass workgroup (one per CU: its LDS)
constexpr int kColPrefetch = 4;          // factor columns held in registers by the column pass
constexpr int kColLdsBudget = 120 * 1024; // LDS the column pass may use
constexpr int kLeanWorkgroups = 512;     // column-pass workgroups from which a launch counts as saturating
constexpr int kLeanMaxM1 = 512;          // largest column length with a lean column-pass variant
constexpr int kRowRegCols = 4;          // row pass: distinct columns up to which unpacked spectra stay in registers
constexpr int kSpreadWorkgroups = 256;   // column-pass workgroups a small launch is spread over (one per CU)
constexpr int kSplitMinColumns = 4;      // fewest distinct columns a share of a split column group takes
constexpr int kTTMaxRank = 8;            // largest tensor-train rank (the chain's per-bin vectors live in registers)

}  // namespace agg
