// Host planner: turns (D, N, CP factors, precision) into the integer tables and
// binary64 twiddles that the device kernels consume.  Pure host code.
#pragma once
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/agg.h"
#include "kernels.h"

namespace agg {

struct PlanTables {
  int D = 0, De = 2;
  int64_t N = 0;
  int prec = AGG_FP64;
  int64_t L = 0, M = 0;
  int M1 = 0, M2 = 0, g = 0;
  int b = 0;                               // split of the length-L twiddle lookup
  int u = 0;                               // distinct factor columns
  std::vector<int> colmap;                 // id per (d, m, r) in scan order
  std::vector<std::vector<double>> ucols;  // u columns of N doubles
  // gain terms: column ids (sorted), multiplicity, sum of the merged ranks'
  // weights (= multiplicity without weights); coefficient = weight sum / d!
  std::vector<std::vector<int>> p_ids;
  std::vector<int> p_mult;
  std::vector<double> p_wsum;
  // loss terms: k-mode id, other ids (sorted), multiplicity, weight sum;
  // coefficient = weight sum / (d-1)!
  std::vector<int> q_d, q_kmode, q_mult;
  std::vector<double> q_wsum;
  std::vector<std::vector<int>> q_ids;
  // row-pass chunks when the combine cannot hold every column at once (cmax > 0):
  // each chunk's distinct column ids (ascending) and gain-term indices
  int cmax = 0;
  std::vector<std::vector<int>> ch_cols, ch_terms;
  // kernels in tensor-train form (plan_build_tt; Sec. 2): order d's gain and
  // loss sums are products of the d cores' matrices per frequency bin and of
  // their dot-product matrices.  Cores are numbered in the order (term by
  // ascending d, lambda = 1..d); core k belongs to term tc_term[k] as core
  // tc_lambda[k], has tc_rin[k] x tc_rout[k] columns whose ids (row-major, -1
  // for an all-zero column) start at tc_ids[tc_off[k]].  TT plans always run
  // the chunked row pass: ch_cols as above, ch_terms holding core indices.
  bool tt = false;
  std::vector<int> tt_d;
  std::vector<int> tc_term, tc_lambda, tc_rin, tc_rout, tc_off, tc_ids;
  std::vector<int64_t> flat;
};

// Validates the arguments and builds the tables.  Returns AGG_OK or an error
// code with a message in *err.
// dedup = false gives every (d, m, r) column its own id (the unshared reference
// evaluation); the rules are otherwise unchanged.
// mixed = true: the transform length may be 3 2^a or 5 2^a (rules in
// planner.cpp's split_mixed), with the odd factor in the column length.
agg_status plan_build(int D, int64_t N, const agg_term* terms, int nterms, int prec,
                      PlanTables* out, std::string* err, bool dedup = true, bool mixed = false);

// The same for kernels given in tensor-train form: one agg_tt_term per order.
// Adds to the rules of plan_build: column ids by first appearance scanning
// terms by ascending d, cores lambda = 1..d, then a < r_{lambda-1}, b <
// r_lambda (the core column H^(lambda)_{a,:,b}), all-zero columns getting -1;
// row-pass chunks group whole cores in scan order, a chunk taking the next
// core while the union of distinct ids stays within the chunk capacity.
// The transform length and its split follow plan_build, with the same
// mixed-radix option.  Unsupported: ranks above kTTMaxRank, rows longer than
// 512 values (the chain's per-bin vectors are held in registers), a core with
// more distinct columns than a chunk holds.
agg_status plan_build_tt(int D, int64_t N, const agg_tt_term* terms, int nterms, int prec, PlanTables* out,
                         std::string* err, bool mixed = false);

// exp(-2 pi i e / P) for e = 0..P-1, interleaved (re, im), binary64; and one entry.
void twiddle_table(int64_t P, double* out);
void twiddle_at(int64_t P, int64_t e, double* re, double* im);

// Time grid of a solve: number of steps and the size of the last one.
void time_grid(double dt, double t_end, int64_t* nsteps, double* last_dt);

// Length of a vector stored in the column pass's column order: size s = 2 j + e
// with j = j2 + M2 j1 sits at 2 (j2 J + j1) + e, J = N/(2 M2) + 1 rows.
inline int64_t colorder_len(int64_t N, int M2) { return 2 * (int64_t)M2 * (N / (2 * (int64_t)M2) + 1); }
inline int64_t colorder_index(int64_t s, int64_t N, int M2) {
  const int64_t J = N / (2 * (int64_t)M2) + 1, j = s >> 1;
  return 2 * ((j % M2) * J + j / M2) + (s & 1);
}

// Bytes of one stored complex value of the spectral path for a precision.
inline int complex_bytes(int prec) { return prec == AGG_FP32 ? 8 : 16; }

}  // namespace agg
