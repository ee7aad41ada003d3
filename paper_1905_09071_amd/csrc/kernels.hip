// Device kernels of the RHS pipeline (definitions in kernels.h).
//
// Per evaluation of f = sum_d (P^(d) + Q^(d)) (Sec. 1) the library runs
//   column pass (forward) -> row pass -> column pass (inverse + epilogue)
// and, inside a time loop, the inverse column pass of one evaluation and the
// forward column pass of the next are the same launch.
//
// Gain term (Sec. 1 CP remark): with x_c[i] = U_c(i) n_i for the u distinct
// factor columns, every rank-one term of p^(d) is a d-fold linear convolution,
// so on the spectra X_c = DFT_L(x_c)
//     P = IDFT_L( sum_t coef_t prod_{c in t} X_c ),   coef_t = mult_t / d!
// and one inverse transform serves every d because the length L keeps outputs
// 2..N free of wrap-around.  Loss term: s_c = U_c . n (binary64), then
// G_c = sum over loss terms t with k-mode c of coef_t prod_{others} s, and
// q_k = -n_k sum_c U_c(k) G_c.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "fft_lds.h"
#include "fft_wave.h"
#include "kernels.h"

namespace agg {

// Largest radix of the in-LDS transform stages: radix 4 for float-float (its
// long arithmetic chains favour more, shorter butterflies), radix 8 otherwise
// (fewer LDS passes).  Measured on the D=4, N=65536 workload.
template <class T> struct StageRadixBase { static constexpr int value = 8; };
template <> struct StageRadixBase<ff> { static constexpr int value = 4; };
// Every variant of a pass (workgroup-wide LDS stages or one transform per
// wavefront, lean or full) runs the same stage sequence for a given length, so
// a state's result does not depend on which variant a launch picked (a slot
// served in a mix computes exactly what it computes alone).  A wavefront holds
// 256 values as 4 per lane, so its stages are at most radix 4 at that length.
template <class T, int P> struct StageRadix {
  static constexpr int value = (P == 256 && StageRadixBase<T>::value > 4) ? 4 : StageRadixBase<T>::value;
};

// Loads and stores of device memory through global-address-space pointers.
// Pointers taken from descriptors and launch structs would otherwise compile
// to flat (generic) accesses, which also count against the LDS wait counter:
// every LDS barrier would then wait for all prefetched global loads.
// Class types (complex values, descriptors) move as the widest whole words:
// 16 bytes when the size allows (every buffer and element offset of a 16-byte
// type is 16-byte aligned), else 8.  Two 8-byte stores per 16-byte element
// were measured to double the HBM write bytes of a fully coalesced store.
typedef unsigned int gword __attribute__((ext_vector_type(2)));
typedef unsigned int gword4 __attribute__((ext_vector_type(4)));
template <class T> struct GWord {
  using type = typename std::conditional<sizeof(T) % 16 == 0, gword4, gword>::type;
  static constexpr int count = sizeof(T) / sizeof(type);
};
template <class T> __device__ __forceinline__ T ldg(const T* p) {
  if constexpr (__is_class(T)) {
    static_assert(sizeof(T) % 8 == 0 && alignof(T) >= 4, "whole 8-byte words");
    using W = typename GWord<T>::type;
    W w[GWord<T>::count];
    const __attribute__((address_space(1))) W* q = (const __attribute__((address_space(1))) W*)p;
#pragma unroll
    for (int i = 0; i < GWord<T>::count; ++i) w[i] = q[i];
    T v;
    __builtin_memcpy(&v, w, sizeof(T));
    return v;
  } else {
    return *(const __attribute__((address_space(1))) T*)p;
  }
}
template <class T> __device__ __forceinline__ void stg(T* p, T v) {
  if constexpr (__is_class(T)) {
    static_assert(sizeof(T) % 8 == 0, "whole 8-byte words");
    using W = typename GWord<T>::type;
    W w[GWord<T>::count];
    __builtin_memcpy(w, &v, sizeof(T));
    __attribute__((address_space(1))) W* q = (__attribute__((address_space(1))) W*)p;
#pragma unroll
    for (int i = 0; i < GWord<T>::count; ++i) q[i] = w[i];
  } else {
    *(__attribute__((address_space(1))) T*)p = v;
  }
}

template <class T>
__device__ __forceinline__ cplx<T> twL(const LaunchArgs& a, int64_t e) {
  const cplx<T>* lo = (const cplx<T>*)a.twLlo;
  const cplx<T>* hi = (const cplx<T>*)a.twLhi;
  int64_t mask = (int64_t(1) << a.b) - 1;
  return cmul(ldg(hi + (e >> a.b)), ldg(lo + (e & mask)));
}

// One data-parallel-primitive move of a binary64 value (both 32-bit halves);
// lanes without a source (or outside ROW_MASK) receive 0.
template <int CTRL, int ROW_MASK = 0xf>
__device__ __forceinline__ double dpp_move(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, ROW_MASK, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, ROW_MASK, 0xf, false);
  return __hiloint2double(hi, lo);
}

// Sum over the 64 lanes of a wavefront in a fixed order (reproducible), with
// register-to-register lane moves: pairs, quads, rows of 16 (row_shr 4 and 8
// leave the row sum in lane 15), then rows 1 and 3 take lane 15 of the row
// below and rows 2-3 lane 31, leaving the total in lane 63, which is read back
// into every lane.  The whole wavefront must be active.
__device__ __forceinline__ double wave_sum(double v) {
  v += dpp_move<0xb1>(v);          // quad_perm [1,0,3,2]
  v += dpp_move<0x4e>(v);          // quad_perm [2,3,0,1]
  v += dpp_move<0x114>(v);         // row_shr:4
  v += dpp_move<0x118>(v);         // row_shr:8
  v += dpp_move<0x142, 0xa>(v);    // row_bcast:15 into rows 1 and 3
  v += dpp_move<0x143, 0xc>(v);    // row_bcast:31 into rows 2 and 3
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), 63);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), 63);
  return __hiloint2double(hi, lo);
}

// The same value in every lane, held in scalar registers: a pointer that is
// uniform over the workgroup (a slot's table) read through the constant address
// space compiles to scalar loads, which need no LDS or vector-memory round trip.
template <class T> __device__ __forceinline__ const __attribute__((address_space(4))) T* uniform_ptr(const T* p) {
  const unsigned long long v = (unsigned long long)p;
  const unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)v);
  const unsigned hi = __builtin_amdgcn_readfirstlane((unsigned)(v >> 32));
  return (const __attribute__((address_space(4))) T*)(((unsigned long long)hi << 32) | lo);
}
__device__ __forceinline__ int uniform_int(int x) { return __builtin_amdgcn_readfirstlane(x); }

// The value held by the neighbouring lane (lane ^ 1), word by word, through a
// DPP quad permute (a register move, no LDS round trip).
template <class T> __device__ __forceinline__ cplx<T> lane_swap1(cplx<T> v) {
  static_assert(sizeof(cplx<T>) % 4 == 0, "whole 32-bit words");
  constexpr int W = sizeof(cplx<T>) / 4;
  int w[W];
  __builtin_memcpy(w, &v, sizeof(v));
#pragma unroll
  for (int i = 0; i < W; ++i) w[i] = __builtin_amdgcn_mov_dpp(w[i], 0xb1, 0xf, 0xf, false);   // quad_perm [1,0,3,2]
  cplx<T> r;
  __builtin_memcpy(&r, w, sizeof(r));
  return r;
}

// The value held by lane `src` of this wavefront, word by word (ds_bpermute: a
// lane-crossing move, no LDS allocation).  The source lane must be active.
template <class T> __device__ __forceinline__ cplx<T> lane_read(cplx<T> v, int src) {
  static_assert(sizeof(cplx<T>) % 4 == 0, "whole 32-bit words");
  constexpr int W = sizeof(cplx<T>) / 4;
  int w[W];
  __builtin_memcpy(w, &v, sizeof(v));
#pragma unroll
  for (int i = 0; i < W; ++i) w[i] = __builtin_amdgcn_ds_bpermute(src << 2, w[i]);
  cplx<T> r;
  __builtin_memcpy(&r, w, sizeof(r));
  return r;
}

// Descriptor of one slot: from device memory, or built from the launch's base
// descriptor and strides (no dependent load before the first data request).
__device__ __forceinline__ SlotDesc slot_desc(const LaunchArgs& a, int slot) {
  if (a.slots) return ldg(a.slots + slot);
  SlotDesc sd = a.base;
  sd.k1 = (double*)((char*)sd.k1 + slot * a.stride.k1);
  sd.ntil = (double*)((char*)sd.ntil + slot * a.stride.ntil);
  sd.Z1 = (void*)((char*)sd.Z1 + slot * a.stride.Z1);
  sd.V = (void*)((char*)sd.V + slot * a.stride.V);
  sd.dots = (double*)((char*)sd.dots + slot * a.stride.dots);
  sd.G = (double*)((char*)sd.G + slot * a.stride.G);
  sd.nprev = (double*)((char*)sd.nprev + slot * a.stride.nprev);
  return sd;
}

// Table entry of logical slot s of a launch (-1: beyond the launch's active list).
__device__ __forceinline__ int launch_slot(const LaunchArgs& a, int s) {
  if (!a.active) return s;
  const auto act = uniform_ptr(a.active);
  return s < act[0] ? act[1 + s] : -1;
}

// What a slot does in this launch: the column mode, whether the row pass runs,
// and the step.  Launch-wide mode (>= 0), per-slot fields (< 0), or the stage
// of a solve counted by the device tick counter.
__device__ __forceinline__ void slot_stage(const LaunchArgs& a, const SlotDesc& sd, int& mode, int& row_on,
                                           double& dt) {
  if (a.mode >= 0) {
    mode = a.mode; row_on = 1; dt = a.dt;
  } else if (a.tick) {
    const int64_t st = *uniform_ptr(a.tick) - sd.start_tick, ns = sd.nsteps;
    if (st < 0 || st > 2 * ns) {
      mode = CM_NONE; row_on = 0; dt = 0.0;
    } else if (st == 0) {
      mode = CM_FWD; row_on = 0; dt = 0.0;
    } else {
      const int64_t step = (st - 1) / 2;
      const bool last = step == ns - 1;
      row_on = 1;
      dt = last ? sd.dt_last : sd.dt;
      mode = (st & 1) ? CM_H1 : (last ? CM_H2 : CM_H2_FWD);
    }
  } else {
    mode = sd.mode; row_on = sd.row_on; dt = sd.dt;
  }
}

// Block index -> work index such that consecutive work indices run on the same
// XCD (workgroups are dealt round-robin over the 8 XCDs), so neighbouring
// column groups share one L2 and its cache lines are written whole.
__device__ __forceinline__ int xcd_contiguous(int b, int nb) {
  return (nb & 7) == 0 ? (b & 7) * (nb >> 3) + (b >> 3) : b;
}

template <class T, int NUM, int NT>
__device__ __forceinline__ void load_table(cplx<T>* dst, const void* src) {
  const cplx<T>* s = (const cplx<T>*)src;
#pragma unroll
  for (int i = threadIdx.x; i < NUM; i += NT) dst[i] = ldg(s + i);
}

// ---------------------------------------------------------------------------
// Column pass.  Work item = (slot, group of g adjacent columns j2, share).
// With usplit > 1 shares (launches with fewer groups than CUs) each share
// transforms its own range of the distinct factor columns; every share
// computes the group's inverse and epilogue, which its weighting needs, and
// share 0 alone stores them.  A state that Heun stage 2 overwrites in place
// would then be read by shares that start after share 0 has written it, so
// split launches keep stage 1's state in nprev and stage 2 reads it from there.
// LDS: the M1 twiddles, then up to ub*g columns of M1 values.
// Every global value the pass needs (the combined spectrum's columns, the
// state and Heun vectors, the first kColPrefetch factor columns and the
// four-step twiddles) is requested in one round at the start, so a launch
// costs about three memory round trips: descriptor, data, stores.
// ---------------------------------------------------------------------------
// Second transform buffer (one barrier per Stockham stage instead of two): a
// gain for the long float-float stages of small launches; binary64 and binary32
// lose more to the extra registers than the barrier costs (measured).
template <class T, int M1, bool LEAN>
constexpr bool kColPingPong = !LEAN && M1 < 2048 && std::is_same<T, ff>::value;
// Forward transforms that skip a broadcast-only first stage (see the column
// pass): enabled where the variant measured faster with it.
template <class T, bool LEAN>
constexpr bool kColPrune = std::is_same<T, ff>::value ? !LEAN : (std::is_same<T, double>::value && LEAN);

// LEAN (used when a launch already fills the GPU): no factor columns or Heun
// vectors held in registers, and a register budget that lets two workgroups
// share a CU, so one workgroup's memory wait overlaps another's arithmetic.
// TILT (binary32 only): exponential tilting of the transforms' inputs, x[s]
// exp(tilt s), and of the gain, exp(-tilt s) (a d-fold convolution of tilted
// inputs is the tilted convolution), so that values decaying like exp(-tilt s)
// keep their relative accuracy in binary32 spectra; the dot products use the
// untilted values.
template <class T, int M1, bool LEAN, bool TILT = false>
__global__ __launch_bounds__(kColThreads, LEAN ? 4 : 1) void col_kernel(LaunchArgs a) {
  constexpr int NT = kColThreads;
  constexpr int GMAX = (1024 / M1) > 0 ? 1024 / M1 : 1;
  constexpr int STR = lds_len(M1);
  constexpr int CAP = GMAX * M1;
  constexpr int IPT = (CAP + NT - 1) / NT;
  constexpr int NWAVE = NT / 64;
  constexpr int UP = LEAN ? 0 : (IPT <= 2 ? kColPrefetch : 2);   // register budget at the largest M1
  constexpr int UPA = UP > 0 ? UP : 1;
  extern __shared__ __align__(16) unsigned char smem[];
  cplx<T>* tw = (cplx<T>*)smem;
  cplx<T>* buf = tw + M1;
  cplx<T>* alt = buf + (size_t)a.ub * GMAX * STR;
  __shared__ double red[NWAVE][kColBatch];
  // launches that fill the GPU, columns of 256 and 512 values: each forward
  // transform is held by one wavefront in registers (fft_wave.h), the
  // wavefronts taking the columns of a group in turn; smaller launches keep the
  // workgroup-wide stages, whose several wavefronts per transform give shorter
  // chains
  constexpr bool CWAVE = LEAN && (M1 == 256 || M1 == 512);
  const int wave_u = uniform_int(threadIdx.x >> 6);

  const int M2 = a.M2, g = a.g, lgg = a.lgg;
  const int ngroups = M2 >> lgg;
  const int nshare = a.usplit > 1 ? a.usplit : 1;
  // the shares of a group are adjacent work items (one XCD, whose L2 serves
  // their common loads)
  const int w = xcd_contiguous(blockIdx.x, a.nslots * ngroups * nshare);
  const int wg = w / nshare;
  const int share = w - wg * nshare;
  const int lslot = wg / ngroups;
  const int grp = wg - lslot * ngroups;
  const int slot = launch_slot(a, lslot);
  if (slot < 0) return;
  const SlotDesc sd = slot_desc(a, slot);
  int mode, row_on_unused;
  double dt;
  slot_stage(a, sd, mode, row_on_unused, dt);
  if (mode == CM_NONE) return;
  if (share > 0 && !mode_has_forward(mode)) return;   // nothing of its own to transform
  const bool split = nshare > 1;
  const bool store = share == 0;                     // the epilogue's stores
  const int64_t N = sd.N;
  const int64_t M = (int64_t)M1 * M2;
  const int j2_0 = grp * g;
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int nitems = g * M1;
  const int u = sd.u;
  // this share's distinct columns [c_lo, c_hi)
  const int c_lo = (int)(((int64_t)share * u) / nshare), c_hi = (int)(((int64_t)(share + 1) * u) / nshare);
  const bool inv = mode_has_inverse(mode), fwd = mode_has_forward(mode);
  const bool stage2 = (mode == CM_H2 || mode == CM_H2_FWD);
  double* state = a.ext_state ? a.ext_state + (size_t)slot * N : sd.n_state;

  // ---- one round of global requests, issued in the order they are needed
  // (completions are counted in issue order) ----
  constexpr int TPT = (M1 + NT - 1) / NT;
  cplx<T> vreg[IPT], twreg[TPT];
  const cplx<T>* V = (const cplx<T>*)sd.V;
#pragma unroll
  for (int it = 0; it < IPT; ++it) {
    int idx = tid + it * NT;
    int k1 = idx >> lgg, jl = idx & (g - 1);
    vreg[it] = (inv && idx < nitems) ? ldg(V + ((int64_t)k1 * M2 + j2_0 + jl)) : czero<T>();
  }
#pragma unroll
  for (int i = 0; i < TPT; ++i) {
    int e = tid + i * NT;
    twreg[i] = e < M1 ? ldg((const cplx<T>*)a.twP1 + e) : czero<T>();
  }
  double Gv[UPA];
#pragma unroll
  for (int q = 0; q < UPA; ++q) Gv[q] = (inv && q < u) ? ldg(sd.G + q) : 0.0;
  // sizes 2j, 2j+1 of each item; the vectors only this pass touches (k1, n~ and
  // the factor columns) are stored in column order, item (j2, j1, e) at
  // 2 (j2 J + j1) + e with J = N/(2 M2) + 1 rows, so a workgroup's accesses are
  // contiguous; the caller's state keeps the size order
  const int64_t Jr = N / (2 * (int64_t)M2) + 1;
  const int64_t CSZ = 2 * (int64_t)M2 * Jr;
  int64_t pos[IPT], cix[IPT];
  double pe[IPT][2], pn[IPT][2], pk[IPT][2], uc[UPA][IPT][2];
#pragma unroll
  for (int it = 0; it < IPT; ++it) {
    int idx = tid + it * NT;
    int j1 = idx >> lgg, jl = idx & (g - 1);
    pos[it] = idx < nitems ? 2 * (j2_0 + jl + (int64_t)M2 * j1) : N + 1;
    cix[it] = idx < nitems ? 2 * ((int64_t)(j2_0 + jl) * Jr + j1) : 0;
#pragma unroll
    for (int e = 0; e < 2; ++e) {
      int64_t s = pos[it] + e, ci = cix[it] + e;
      bool ok = s >= 1 && s <= N;
      pe[it][e] = ok ? (stage2 ? ldg(sd.ntil + ci) : ldg(state + (s - 1))) : 0.0;
      pn[it][e] = (!LEAN && ok && stage2) ? (split ? ldg(sd.nprev + ci) : ldg(state + (s - 1))) : 0.0;
      pk[it][e] = (!LEAN && ok && stage2) ? ldg(sd.k1 + ci) : 0.0;
#pragma unroll
      for (int q = 0; q < UP; ++q) uc[q][it][e] = (ok && q < u) ? ldg(sd.cols + ((size_t)q * CSZ + ci)) : 0.0;
    }
  }
  // four-step twiddles w_M^(j2 k1) (two table halves; multiplied when used)
  cplx<T> wsh[IPT], wsl[IPT];
#pragma unroll
  for (int it = 0; it < IPT; ++it) {
    int idx = tid + it * NT;
    int k1 = idx >> lgg, jl = idx & (g - 1);
    int64_t e = (2 * (int64_t)(j2_0 + jl) * k1) % a.L;
    bool ok = fwd && idx < nitems;
    wsh[it] = ok ? ldg((const cplx<T>*)a.twLhi + (e >> a.b)) : czero<T>();
    wsl[it] = ok ? ldg((const cplx<T>*)a.twLlo + (e & ((int64_t(1) << a.b) - 1))) : czero<T>();
  }
  // the spectrum block and the twiddle table go to LDS (waits only for them)
#pragma unroll
  for (int it = 0; it < IPT; ++it) {
    int idx = tid + it * NT;
    int k1 = idx >> lgg, jl = idx & (g - 1);
    if (inv && idx < nitems) buf[jl * STR + lds_pad(k1)] = vreg[it];
  }
#pragma unroll
  for (int i = 0; i < TPT; ++i) {
    int e = tid + i * NT;
    if (e < M1) tw[e] = twreg[i];
  }

  double s0[IPT], s1[IPT];   // state the forward pass weights, at sizes 2j, 2j+1
  if (inv) {
    lds_barrier();
    cplx<T>* ib = buf;   // inverse transforms' result
    // (the g inverse transforms keep the workgroup-wide stages in every
    // variant: one wavefront per transform would leave most of them idle)
    if constexpr (!kColPingPong<T, M1, LEAN>) {
      fft_batch<T, M1, +1, GMAX, STR, NT, StageRadix<T, M1>::value>(buf, g, tw);
    } else {
      ib = fft_batch_pp<T, M1, +1, GMAX, STR, NT, StageRadix<T, M1>::value>(buf, alt, g, tw);
    }

    // loss weight g_k = sum_c U_c(k) G_c
    double gk[IPT][2];
#pragma unroll
    for (int it = 0; it < IPT; ++it) gk[it][0] = gk[it][1] = 0.0;
#pragma unroll
    for (int q = 0; q < UP; ++q) {
      if (q < u) {
        const double Gc = Gv[q];
#pragma unroll
        for (int it = 0; it < IPT; ++it) {
          gk[it][0] += uc[q][it][0] * Gc;
          gk[it][1] += uc[q][it][1] * Gc;
        }
      }
    }
    // (columns with a zero weight add exact zeros to the finite sums: skipped;
    // a tensor-train kernel weights only its last cores' columns)
    const auto Gu = uniform_ptr((const double*)sd.G);
    for (int c = UP; c < u; ++c) {
      const double Gc = Gu[c];
      if (Gc == 0.0) continue;
      const double* col = sd.cols + (size_t)c * CSZ;
#pragma unroll
      for (int it = 0; it < IPT; ++it)
#pragma unroll
        for (int e = 0; e < 2; ++e) {
          int64_t s = pos[it] + e;
          if (s >= 1 && s <= N) gk[it][e] += ldg(col + (cix[it] + e)) * Gc;
        }
    }

    const double invL = 1.0 / (double)a.L;
    double* out = a.ext_out ? a.ext_out + (size_t)slot * N : sd.out;
#pragma unroll
    for (int it = 0; it < IPT; ++it) {
      int idx = tid + it * NT;
      s0[it] = 0.0;
      s1[it] = 0.0;
      if (idx < nitems) {
        int j1 = idx >> lgg, jl = idx & (g - 1);
        cplx<T> wv = ib[jl * STR + lds_pad(j1)];
        double y[2] = {Real<T>::to_d(wv.re), Real<T>::to_d(wv.im)};
#pragma unroll
        for (int e = 0; e < 2; ++e) {
          int64_t s = pos[it] + e;
          double val = 0.0;
          if (s >= 1 && s <= N) {
            double p = s >= 2 ? y[e] * invL : 0.0;
            if constexpr (TILT) p *= exp(-a.tilt * (double)s);
            double f = p - pe[it][e] * gk[it][e];
            if (mode == CM_RHS) {
              stg(out + (s - 1), f);
            } else if (mode == CM_RHS_ACC) {
              stg(out + (s - 1), ldg(out + (s - 1)) + f);
            } else if (mode == CM_H1) {
              val = pe[it][e] + dt * f;
              if (store) {
                stg(sd.k1 + (cix[it] + e), f);
                stg(sd.ntil + (cix[it] + e), val);
                if (split) stg(sd.nprev + (cix[it] + e), pe[it][e]);
              }
            } else {
              const double nb =
                  LEAN ? (split ? ldg(sd.nprev + (cix[it] + e)) : ldg(state + (s - 1))) : pn[it][e];
              const double kb = LEAN ? ldg(sd.k1 + (cix[it] + e)) : pk[it][e];
              val = nb + 0.5 * dt * (kb + f);
              if (store) stg(state + (s - 1), val);
            }
          }
          if (e == 0) s0[it] = val; else s1[it] = val;
        }
      }
    }
    if (!fwd) return;
    lds_barrier();
  } else {
#pragma unroll
    for (int it = 0; it < IPT; ++it) {
      s0[it] = pe[it][0];
      s1[it] = pe[it][1];
    }
  }

  cplx<T> wst[IPT];
#pragma unroll
  for (int it = 0; it < IPT; ++it) wst[it] = cmul(wsh[it], wsl[it]);
  cplx<T>* Z1 = (cplx<T>*)sd.Z1;
  // Sizes 2(j2 + M2 j1) + e exceed N for j1 > jmax.  When every nonzero input
  // of the group's columns lies in the first block of the first radix-R1 stage
  // (j1 < M1/R1), that stage only copies each input to its R1 outputs: the
  // weighting writes them directly and the transform starts at its second stage.
  constexpr int R1 = stage_radix(M1, 1, StageRadix<T, M1>::value);   // radix of the first stage
  const int64_t rest = N - 2 * (int64_t)j2_0;
  const bool prune = kColPrune<T, LEAN> && !CWAVE && (M1 & (M1 - 1)) == 0 &&
                     (rest < 0 ? -1 : rest / (2 * (int64_t)M2)) < M1 / R1;
  auto put = [&](int slot, int j1, cplx<T> v) {
    if (prune) {
      if (j1 < M1 / R1) {
#pragma unroll
        for (int r = 0; r < R1; ++r) buf[slot * STR + lds_pad(R1 * j1 + r)] = v;
      }
    } else {
      buf[slot * STR + lds_pad(j1)] = v;
    }
  };
  auto tilted = [&](double x, int it, int e) -> double {
    if constexpr (TILT) {
      const int64_t s = pos[it] + e;
      if (s >= 1 && s <= N) return x * exp(a.tilt * (double)s);
    }
    return x;
  };
  for (int cb = c_lo; cb < c_hi; cb += a.ub) {
    const int nc = c_hi - cb < a.ub ? c_hi - cb : a.ub;
    // weighted columns x_c = U_c * state for c in [cb, cb+nc)
#pragma unroll
    for (int q = 0; q < UP; ++q) {
      if (q >= cb && q < cb + nc) {
        double dsum = 0.0;
#pragma unroll
        for (int it = 0; it < IPT; ++it) {
          int idx = tid + it * NT;
          if (idx < nitems) {
            int j1 = idx >> lgg, jl = idx & (g - 1);
            double x0 = uc[q][it][0] * s0[it];
            double x1 = uc[q][it][1] * s1[it];
            put((q - cb) * g + jl, j1, cplx<T>{Real<T>::from_d(tilted(x0, it, 0)), Real<T>::from_d(tilted(x1, it, 1))});
            dsum += x0 + x1;
          }
        }
        dsum = wave_sum(dsum);
        if (lane == 0) red[wave][q - cb] = dsum;
      }
    }
    for (int c = cb > UP ? cb : UP; c < cb + nc; ++c) {
      const double* col = sd.cols + (size_t)c * CSZ;
      double dsum = 0.0;
#pragma unroll
      for (int it = 0; it < IPT; ++it) {
        int idx = tid + it * NT;
        if (idx < nitems) {
          int j1 = idx >> lgg, jl = idx & (g - 1);
          int64_t s = pos[it];
          double x0 = (s >= 1 && s <= N) ? ldg(col + cix[it]) * s0[it] : 0.0;
          double x1 = (s + 1 <= N) ? ldg(col + (cix[it] + 1)) * s1[it] : 0.0;
          put((c - cb) * g + jl, j1, cplx<T>{Real<T>::from_d(tilted(x0, it, 0)), Real<T>::from_d(tilted(x1, it, 1))});
          dsum += x0 + x1;
        }
      }
      dsum = wave_sum(dsum);
      if (lane == 0) red[wave][c - cb] = dsum;
    }
    lds_barrier();
    // transforms per register pass: fewer above 1024 values and at the
    // mixed-radix lengths, to stay within 256 VGPRs (four groups per pass
    // spilled to scratch memory there: at 1280 values the spill traffic more
    // than doubled the pass's HBM writes)
    // lean launches transform one column per pass (ub = 1): one group of columns per register pass
    constexpr int FNB = LEAN ? GMAX : GMAX * ((M1 > 1024 || M1 % 3 == 0 || M1 % 5 == 0) ? 2 : kColBatch);
    constexpr int RF = StageRadix<T, M1>::value;
    cplx<T>* fb = buf;   // forward transforms' result
    if constexpr (CWAVE) {
      for (int q = wave_u; q < nc * g; q += NWAVE) fft_wave_lds<T, M1, -1, StageRadix<T, M1>::value>(buf + (size_t)q * STR, tw);
      lds_barrier();
    } else if constexpr (!kColPingPong<T, M1, LEAN>) {
      if (prune) fft_batch<T, M1, -1, FNB, STR, NT, RF, R1>(buf, nc * g, tw);
      else fft_batch<T, M1, -1, FNB, STR, NT, RF>(buf, nc * g, tw);
    } else {
      fb = prune ? fft_batch_pp<T, M1, -1, FNB, STR, NT, RF, R1>(buf, alt, nc * g, tw)
                 : fft_batch_pp<T, M1, -1, FNB, STR, NT, RF>(buf, alt, nc * g, tw);
    }
    for (int q = 0; q < nc; ++q) {
#pragma unroll
      for (int it = 0; it < IPT; ++it) {
        int idx = tid + it * NT;
        if (idx < nitems) {
          int k1 = idx >> lgg, jl = idx & (g - 1);
          stg(Z1 + ((size_t)(cb + q) * M + (int64_t)k1 * M2 + j2_0 + jl),
              cnorm(cmul(fb[(q * g + jl) * STR + lds_pad(k1)], wst[it])));
        }
      }
    }
    if (tid < nc) {
      double t = 0.0;
#pragma unroll
      for (int wv = 0; wv < NWAVE; ++wv) t += red[wv][tid];
      stg(sd.dots + ((size_t)(cb + tid) * ngroups + grp), t);
    }
    lds_barrier();
  }
}

// ---------------------------------------------------------------------------
// Row pass.  Work item = (slot, k1 in [0, M1/2]) covering rows k1 and M1-k1.
// LDS: M2 twiddles (global for M2 = 2048, where the rows need the room), the
// gain-term tables, u*nrows rows, u Nyquist values.
// ---------------------------------------------------------------------------
// Threads per row-pass workgroup: below saturation (about one workgroup per
// CU) twice the threads halve every per-thread chain of the transforms.
template <int M2, bool LEAN> struct RowThreads {
  static constexpr int value = (!LEAN && M2 >= 128) ? 2 * kThreads : kThreads;
};

template <class T, int M2, bool LEAN>
__global__ __launch_bounds__((RowThreads<M2, LEAN>::value), LEAN ? 4 : 1) void row_kernel(LaunchArgs a) {
  constexpr int NT = RowThreads<M2, LEAN>::value;
  constexpr bool TW_LDS = M2 <= 512;
  // transforms per register pass: 2048 values for 256 threads, twice that for
  // 512 threads at the longest rows (so every thread holds a butterfly)
  constexpr int NB = (M2 >= 1024 && NT > kThreads) ? 4096 / M2 : ((2048 / M2) > 0 ? 2048 / M2 : 1);
  constexpr int STR = lds_len(M2);
  constexpr int NWAVE = NT / 64;
  constexpr int UPT = (M2 + NT - 1) / NT;       // combine units per thread
  constexpr int HPT = (2 * M2 + NT - 1) / NT;   // combine half-units per thread (two lanes per unit)
  constexpr int CPT = UPT > HPT ? UPT : HPT;
  // rows of 256 and 512 values: each transform is held by one wavefront in
  // registers (fft_wave.h), loaded from and stored to device memory directly;
  // other lengths run the workgroup-wide LDS stages
  constexpr bool WAVE = M2 == 256 || (M2 == 512 && !(LEAN && std::is_same<T, ff>::value));   // (that one spilled)
  constexpr int E = WAVE ? M2 / 64 : 1;         // values per lane of a wavefront transform
  constexpr int VPT = WAVE ? E : (2 * M2 + NT - 1) / NT;   // output values per thread
  // lanes sharing a bin pair's gain terms (rows of at most 64 values, where both
  // variants run 256 threads, so every variant shares a pair the same way)
  constexpr int TS = M2 <= 64 ? (256 / M2 >= 8 ? 8 : 256 / M2) : 1;
  static_assert(TS == 1 || NT / TS >= (M2 > 32 ? M2 : 32), "a lane group per bin pair");
  extern __shared__ __align__(16) unsigned char smem[];

  const int M1 = a.M1;
  const int nwork = M1 / 2 + 1;
  const int lslot = blockIdx.x / nwork;
  const int k1 = blockIdx.x - lslot * nwork;
  const int slot = launch_slot(a, lslot);
  if (slot < 0) return;
  const SlotDesc sd = slot_desc(a, slot);
  int mode_unused, row_on;
  double dt_unused;
  slot_stage(a, sd, mode_unused, row_on, dt_unused);
  if (!row_on) return;
  const int u = sd.u;
  const int64_t M = (int64_t)M1 * M2;
  const int tid = threadIdx.x;
  // the wavefront index is uniform over the wavefront: held in a scalar
  // register, loops over a wavefront's jobs are uniform branches
  const int lane = tid & 63, wave = uniform_int(tid >> 6);

  // LDS layout
  cplx<T>* twl = (cplx<T>*)smem;                         // M2 when TW_LDS
  const cplx<T>* tw = TW_LDS ? twl : (const cplx<T>*)a.twP2;
  cplx<T>* X = twl + (TW_LDS ? M2 : 0);                  // umax*2 rows
  cplx<T>* nyq = X + (size_t)a.umax * 2 * STR;           // umax
  double* coef = (double*)(nyq + a.umax);                // coef_max
  double* red = coef + a.coef_max;                       // NWAVE * umax
  double* sdot = red + NWAVE * a.umax;                   // umax
  int* tab = (int*)(sdot + a.umax);                      // tab_max

  const int nrows = (k1 == 0 || 2 * k1 == M1) ? 1 : 2;
  auto row_of = [&](int rr) { return rr ? M1 - k1 : k1; };   // the two rows (no indexed array)
  const int Tp = sd.Tp;

  // everything this work item reads from HBM is requested up front, in the
  // order it is needed (completions are counted in issue order)
  const cplx<T>* Z1 = (const cplx<T>*)sd.Z1;
  // wavefront transforms: job j = (column j / nrows, row j mod nrows); wavefront
  // w takes jobs w, w + NWAVE, ..., holding the next job's row in registers
  // while it transforms the current one
  const int njobs = u * nrows;
  cplx<T> vcur[E], vnext[E];
  auto load_job = [&](int j, cplx<T>(&v)[E]) {
    const int c = j / nrows, rr = j - c * nrows;
    const cplx<T>* src = Z1 + ((size_t)c * M + (int64_t)row_of(rr) * M2 + lane);
#pragma unroll
    for (int e = 0; e < E; ++e) v[e] = ldg(src + 64 * e);
  };
  if constexpr (WAVE) {
    if (wave < njobs) load_job(wave, vcur);
    if (wave + NWAVE < njobs) load_job(wave + NWAVE, vnext);
  } else {
    const int nload = u * nrows * M2;
#pragma unroll 8
    for (int idx = tid; idx < nload; idx += NT) {
      int cr = idx / M2, k2 = idx - cr * M2;
      int c = cr / nrows, rr = cr - c * nrows;
      X[cr * STR + lds_pad(k2)] = ldg(Z1 + ((size_t)c * M + (int64_t)row_of(rr) * M2 + k2));
    }
  }
  if (TW_LDS) load_table<T, M2, NT>(twl, a.twP2);
  const int nunits = (k1 == 0) ? M2 / 2 + 1 : (nrows == 1 ? M2 / 2 : M2);
  const int64_t lmask = (int64_t(1) << a.b) - 1;
  // combine mapping: with few distinct columns (non-lean variant) two adjacent
  // lanes share a bin pair, one per bin; otherwise one thread per bin pair.
  // The longest rows keep the LDS mapping: the register mapping spilled there
  // and measured 7% slower.
  const bool split = !LEAN && M2 < 2048 && u <= kRowRegCols;
  cplx<T> wkh[CPT], wkl[CPT];   // w_L^k of this thread's combine units (two table halves)
  cplx<T> wvh[VPT], wvl[VPT];   // w_M^(j2 row) of this thread's outputs (conjugated at use)
  auto load_twiddles = [&]() {
#pragma unroll
    for (int i = 0; i < CPT; ++i) {
      int unit = split ? (tid + i * NT) >> 1 : tid + i * NT;
      int64_t e = k1 + (int64_t)M1 * unit;
      wkh[i] = unit < nunits ? ldg((const cplx<T>*)a.twLhi + (e >> a.b)) : czero<T>();
      wkl[i] = unit < nunits ? ldg((const cplx<T>*)a.twLlo + (e & lmask)) : czero<T>();
    }
#pragma unroll
    for (int i = 0; i < VPT; ++i) {
      // wavefront transforms: wavefront rr stores row rr, lane l value e is j2 = l + 64 e
      int idx = WAVE ? wave * M2 + lane + 64 * i : tid + i * NT;
      int rr = idx / M2, j2 = idx - rr * M2;
      int64_t e = (2 * (int64_t)j2 * row_of(rr == 1)) % a.L;
      wvh[i] = idx < nrows * M2 ? ldg((const cplx<T>*)a.twLhi + (e >> a.b)) : czero<T>();
      wvl[i] = idx < nrows * M2 ? ldg((const cplx<T>*)a.twLlo + (e & lmask)) : czero<T>();
    }
  };
  // wavefront transforms hold their rows in registers meanwhile: their twiddles
  // are requested after the forward transforms
  if constexpr (!WAVE) load_twiddles();
  for (int i = tid; i < sd.ntab; i += NT) tab[i] = ldg(sd.tab + i);
  for (int i = tid; i < Tp + sd.Tq; i += NT) coef[i] = ldg(sd.coef + i);
  if (k1 == 0) {   // partial dots of the column pass -> per-wave sums
    const int ngroups = M2 / a.g;
    for (int c = 0; c < u; ++c) {
      double sacc = 0.0;
      for (int q = tid; q < ngroups; q += NT) sacc += ldg(sd.dots + ((size_t)c * ngroups + q));
      sacc = wave_sum(sacc);
      if (lane == 0) red[wave * a.umax + c] = sacc;
    }
  }
  lds_barrier();
  if constexpr (WAVE) {
    // each job's row is transformed in registers, with the row's own LDS
    // region as exchange space, and lands there in natural order
    for (int j = wave; j < njobs; j += NWAVE) {
      fft_wave<T, M2, -1, StageRadix<T, M2>::value>(vcur, X + (size_t)j * STR, tw);
#pragma unroll
      for (int e = 0; e < E; ++e) X[(size_t)j * STR + lds_pad(lane + 64 * e)] = vcur[e];
      // (the next row always arrives in the second register set: reloading the
      // current set in place at the end of the loop body was miscompiled at
      // -O3 for this target, which clobbered the first stage's inputs)
      if (j + NWAVE < njobs) {
#pragma unroll
        for (int e = 0; e < E; ++e) vcur[e] = vnext[e];
        if (j + 2 * NWAVE < njobs) load_job(j + 2 * NWAVE, vnext);
      }
    }
    load_twiddles();
    lds_barrier();
  } else {
    fft_batch<T, M2, -1, NB, STR, NT, StageRadix<T, M2>::value>(X, u * nrows, tw);
  }

  // bins k = k1 + M1*iA and M - k, spectra of the real inputs, their weighted
  // products, and the even/odd packing of the real inverse; the gain-term
  // tables are read with scalar loads (uniform over the workgroup)
  const auto poff = uniform_ptr(sd.tab);
  const auto pids = uniform_ptr(sd.tab + sd.o_pids);
  const auto pcoef = uniform_ptr(sd.coef);
  const auto pfrom = uniform_ptr(sd.tab + sd.o_pfrom);
  const int Tpu = uniform_int(Tp);
  // bin pair of a unit: A = iA in row 0, B = its mirror (row rB)
  auto pair_of = [&](int unit, int& iB, int& rB) {
    if (k1 == 0) { iB = (M2 - unit) & (M2 - 1); rB = 0; }
    else if (nrows == 1) { iB = M2 - 1 - unit; rB = 0; }
    else { iB = M2 - 1 - unit; rB = 1; }
  };
  // spectrum of real input c at bins A and B from the packed half-length
  // spectrum Z: X(A) = E + t and X(B) = conj(E - t), E = (Z_A + conj Z_B)/2,
  // t = w_L^k * (-i)(Z_A - conj Z_B)/2; at the zero bin X(0) = Re+Im of Z_0
  // and the Nyquist value X(M) = Re-Im
  auto unpack = [&](int c, int iA, int iB, int rB, bool zero_bin, bool self, cplx<T> wk, cplx<T>& xa,
                    cplx<T>& xb) {
    const cplx<T> ZA = X[(c * nrows) * STR + lds_pad(iA)];
    const cplx<T> ZB = X[(c * nrows + rB) * STR + lds_pad(iB)];
    if (zero_bin) {
      xa = cplx<T>{ZA.re + ZA.im, Real<T>::zero()};
      xb = cplx<T>{ZA.re - ZA.im, Real<T>::zero()};
    } else {
      cplx<T> zc = cconj(ZB);
      cplx<T> E = cplx<T>{half_of(ZA.re + zc.re), half_of(ZA.im + zc.im)};
      cplx<T> dd = csub(ZA, zc);
      cplx<T> O = cplx<T>{half_of(dd.im), half_of(-dd.re)};   // -i*(ZA - conj ZB)/2
      cplx<T> t = cmul(wk, O);
      xa = cadd(E, t);
      xb = self ? xa : cconj(csub(E, t));
    }
  };
  // even/odd packing of the real inverse from the combined spectrum at A and B
  auto pack_a = [&](cplx<T> YA, cplx<T> YB, cplx<T> wk) {
    return cadd(cadd(YA, cconj(YB)), cmul_i(cmulc(csub(YA, cconj(YB)), wk)));
  };
  auto pack_b = [&](cplx<T> YA, cplx<T> YB, cplx<T> wk) {
    return cadd(cconj(cadd(YA, cconj(YB))), cmul_i(cmul(wk, cconj(csub(YA, cconj(YB))))));
  };
  if (split) {
    // few distinct columns: each lane keeps its bin's unpacked spectra in
    // registers and forms the products for that bin; the partner lane's sum
    // arrives by a lane exchange.  Both lanes read a pair's inputs with the same
    // LDS instructions before either writes, and the lanes of a wave run in
    // lockstep, so no barrier is needed.
#pragma unroll
    for (int i = 0; i < HPT; ++i) {
      const int h = tid + i * NT;
      const int unit = h >> 1, side = h & 1;
      const bool valid = unit < nunits;
      int iB, rB;
      pair_of(unit, iB, rB);
      const int iA = unit;
      const bool zero_bin = (k1 == 0 && iA == 0);
      const bool self = (rB == 0 && iB == iA);
      const cplx<T> wk = cmul(wkh[i], wkl[i]);
      cplx<T> x[kRowRegCols];
#pragma unroll
      for (int c = 0; c < kRowRegCols; ++c) {
        x[c] = czero<T>();
        if (valid && c < u) {
          cplx<T> xa, xb;
          unpack(c, iA, iB, rB, zero_bin, self, wk, xa, xb);
          x[c] = cnorm(side ? xb : xa);   // as stored by the LDS mapping
        }
      }
      // running product over the ids of each term (continued from the
      // previous term when that one is its prefix), times the coefficient
      cplx<T> Y = czero<T>(), P = czero<T>();
      for (int t = 0; t < Tpu; ++t) {
        const int oe = poff[t + 1];
        int o = pfrom[t];
        bool fresh = o == poff[t];
        for (; o < oe; ++o) {
          const int c = pids[o];
          cplx<T> f = x[0];
#pragma unroll
          for (int q = 1; q < kRowRegCols; ++q)
            if (c == q) f = x[q];
          P = fresh ? f : cmul(P, f);
          fresh = false;
        }
        Y = cadd(Y, cscale(P, Real<T>::from_d(pcoef[t])));
      }
      const cplx<T> Yp = lane_swap1(Y);
      if (valid) {
        const cplx<T> YA = side ? Yp : Y, YB = side ? Y : Yp;
        if (zero_bin) {
          if (side == 0) X[0] = cnorm(cplx<T>{YA.re + YB.re, YA.re - YB.re});
        } else if (side == 0) {
          X[lds_pad(iA)] = cnorm(pack_a(YA, YB, wk));
        } else if (!self) {
          X[rB * STR + lds_pad(iB)] = cnorm(pack_b(YA, YB, wk));
        }
      }
    }
  } else if (TS > 1 && u > kRowRegCols && Tpu >= 2 * TS) {
    // rows of at most 64 values with many gain terms (fewer bin pairs than
    // threads): a bin pair's terms are shared by TS adjacent lanes of one
    // wavefront in contiguous blocks; a block that starts inside a running
    // product recomputes its prefix with the same operations in the same order,
    // and the lanes' sums are added in lane order.  (Every launch variant takes
    // this path for such a slot: with more than kRowRegCols columns none keeps
    // the spectra in registers.)
    const int su = wave * (64 / TS) + lane / TS;   // this lane's bin pair
    const int sg = lane % TS, sbase = lane - sg;
    const bool on = su < nunits;
    int iB = 0, rB = 0;
    if (on) pair_of(su, iB, rB);
    const int iA = su;
    const bool zero_bin = (k1 == 0 && iA == 0);
    const bool self = (rB == 0 && iB == iA);
    cplx<T> wk = czero<T>();
    if (on) {
      const int64_t e = k1 + (int64_t)M1 * su;
      wk = cmul(ldg((const cplx<T>*)a.twLhi + (e >> a.b)), ldg((const cplx<T>*)a.twLlo + (e & lmask)));
      for (int c = sg; c < u; c += TS) {   // the pair's columns unpacked by its lanes in turn
        cplx<T> xa, xb;
        unpack(c, iA, iB, rB, zero_bin, self, wk, xa, xb);
        X[(c * nrows) * STR + lds_pad(iA)] = cnorm(xa);
        if (zero_bin) nyq[c] = cnorm(xb);
        else if (!self) X[(c * nrows + rB) * STR + lds_pad(iB)] = cnorm(xb);
      }
    }
    wave_lds_sync();   // a pair's lanes sit in one wavefront
    if (on) {
      cplx<T> YA = czero<T>(), YB = czero<T>(), PA = czero<T>(), PB = czero<T>();
      const int per = (Tpu + TS - 1) / TS;
      const int t0 = min(Tpu, sg * per), t1 = min(Tpu, t0 + per);
      for (int t = t0; t < t1; ++t) {
        const int oe = poff[t + 1];
        int o = t == t0 ? poff[t] : pfrom[t];
        bool fresh = o == poff[t];
        for (; o < oe; ++o) {
          int c = pids[o];
          const cplx<T> fa = X[(c * nrows) * STR + lds_pad(iA)];
          const cplx<T> fb = zero_bin ? nyq[c] : X[(c * nrows + rB) * STR + lds_pad(iB)];
          PA = fresh ? fa : cmul(PA, fa);
          PB = fresh ? fb : cmul(PB, fb);
          fresh = false;
        }
        const T cf = Real<T>::from_d(pcoef[t]);
        YA = cadd(YA, cscale(PA, cf));
        YB = cadd(YB, cscale(PB, cf));
      }
      cplx<T> SA = lane_read(YA, sbase), SB = lane_read(YB, sbase);
#pragma unroll
      for (int j = 1; j < TS; ++j) {
        SA = cadd(SA, lane_read(YA, sbase + j));
        SB = cadd(SB, lane_read(YB, sbase + j));
      }
      if (sg == 0) {
        if (zero_bin) {
          X[0] = cnorm(cplx<T>{SA.re + SB.re, SA.re - SB.re});
        } else {
          X[lds_pad(iA)] = cnorm(pack_a(SA, SB, wk));
          if (!self) X[rB * STR + lds_pad(iB)] = cnorm(pack_b(SA, SB, wk));
        }
      }
    }
  } else {
#pragma unroll
    for (int i = 0; i < UPT; ++i) {
      const int unit = tid + i * NT;
      if (unit >= nunits) continue;
      int iB, rB;
      pair_of(unit, iB, rB);
      const int iA = unit;
      const bool zero_bin = (k1 == 0 && iA == 0);
      const bool self = (rB == 0 && iB == iA);
      const cplx<T> wk = cmul(wkh[i], wkl[i]);
      for (int c = 0; c < u; ++c) {
        cplx<T> xa, xb;
        unpack(c, iA, iB, rB, zero_bin, self, wk, xa, xb);
        X[(c * nrows) * STR + lds_pad(iA)] = cnorm(xa);
        if (zero_bin) nyq[c] = cnorm(xb);
        else if (!self) X[(c * nrows + rB) * STR + lds_pad(iB)] = cnorm(xb);
      }
      cplx<T> YA = czero<T>(), YB = czero<T>(), PA = czero<T>(), PB = czero<T>();
      for (int t = 0; t < Tpu; ++t) {
        const int oe = poff[t + 1];
        int o = pfrom[t];
        bool fresh = o == poff[t];
        for (; o < oe; ++o) {
          int c = pids[o];
          const cplx<T> fa = X[(c * nrows) * STR + lds_pad(iA)];
          const cplx<T> fb = zero_bin ? nyq[c] : X[(c * nrows + rB) * STR + lds_pad(iB)];
          PA = fresh ? fa : cmul(PA, fa);
          PB = fresh ? fb : cmul(PB, fb);
          fresh = false;
        }
        const T cf = Real<T>::from_d(pcoef[t]);
        YA = cadd(YA, cscale(PA, cf));
        YB = cadd(YB, cscale(PB, cf));
      }
      if (zero_bin) {
        X[0] = cnorm(cplx<T>{YA.re + YB.re, YA.re - YB.re});
      } else {
        X[lds_pad(iA)] = cnorm(pack_a(YA, YB, wk));
        if (!self) X[rB * STR + lds_pad(iB)] = cnorm(pack_b(YA, YB, wk));
      }
    }
  }
  lds_barrier();
  cplx<T>* V = (cplx<T>*)sd.V;
  if constexpr (WAVE) {
    if (wave < nrows) {   // wavefront rr: inverse of row rr in registers, stored from them
      cplx<T> y[E];
#pragma unroll
      for (int e = 0; e < E; ++e) y[e] = X[(size_t)wave * STR + lds_pad(lane + 64 * e)];
      __builtin_amdgcn_wave_barrier();
      fft_wave<T, M2, +1, StageRadix<T, M2>::value>(y, X + (size_t)wave * STR, tw);
      cplx<T>* dst = V + (int64_t)row_of(wave) * M2 + lane;
#pragma unroll
      for (int e = 0; e < E; ++e) stg(dst + 64 * e, cnorm(cmulc(y[e], cmul(wvh[e], wvl[e]))));
    }
  } else {
    fft_batch<T, M2, +1, NB, STR, NT, StageRadix<T, M2>::value>(X, nrows, tw);
#pragma unroll
    for (int i = 0; i < VPT; ++i) {
      int idx = tid + i * NT;
      if (idx < nrows * M2) {
        int rr = idx / M2, j2 = idx - rr * M2;
        stg(V + ((int64_t)row_of(rr) * M2 + j2), cnorm(cmulc(X[rr * STR + lds_pad(j2)], cmul(wvh[i], wvl[i]))));
      }
    }
  }

  // loss-term weights of this evaluation: G_c = sum over loss terms with k-mode c
  // of coef * prod of the other modes' dot products
  if (k1 == 0) {
    if (tid < u) {
      double t = 0.0;
      for (int wv = 0; wv < NWAVE; ++wv) t += red[wv * a.umax + tid];
      sdot[tid] = t;
    }
    lds_barrier();
    if (tid < u) {
      const int* qoff = tab + sd.o_qoff;
      const int* qids = tab + sd.o_qids;
      const int* qkm = tab + sd.o_qkm;
      double Gc = 0.0;
      for (int t = 0; t < sd.Tq; ++t) {
        if (qkm[t] != tid) continue;
        double pr = coef[Tp + t];
        for (int o = qoff[t]; o < qoff[t + 1]; ++o) pr *= sdot[qids[o]];
        Gc += pr;
      }
      stg(sd.G + tid, Gc);
    }
  }
}

// ---------------------------------------------------------------------------
// Row pass in chunks, for kernel sets whose distinct columns do not all fit in
// LDS at the row length (many ranks at the longest transforms).  Work item and
// result are those of row_kernel.  The gain terms come grouped into chunks of
// at most a.cmax columns; per chunk the work item loads, transforms and unpacks
// that chunk's columns only and adds the chunk's terms to per-thread sums of
// the combined spectrum, which stay in registers across chunks.  The inverse
// transform and the loss-term weights follow the last chunk.  A slot without
// chunk tables runs as one chunk of all its columns.
// LDS: M2 twiddles (M2 <= 512), a.cmax*2 rows, a.cmax Nyquist values, the
// per-wave partial dots and the u dot products.
// ---------------------------------------------------------------------------
template <class T, int M2>
__global__ __launch_bounds__(kChunkThreads, 1) void row_chunk_kernel(LaunchArgs a) {
  constexpr int NT = kChunkThreads;
  constexpr bool TW_LDS = M2 <= 512;
  constexpr int NB = (4096 / M2) > 0 ? 4096 / M2 : 1;   // a butterfly per thread at radix 8
  constexpr int STR = lds_len(M2);
  constexpr int NWAVE = NT / 64;
  constexpr int UPT = (M2 + NT - 1) / NT;       // combine units (bin pairs) per thread
  constexpr int VPT = (2 * M2 + NT - 1) / NT;   // output values per thread
  extern __shared__ __align__(16) unsigned char smem[];

  const int M1 = a.M1;
  const int nwork = M1 / 2 + 1;
  const int lslot = blockIdx.x / nwork;
  const int k1 = blockIdx.x - lslot * nwork;
  const int slot = launch_slot(a, lslot);
  if (slot < 0) return;
  const SlotDesc sd = slot_desc(a, slot);
  int mode_unused, row_on;
  double dt_unused;
  slot_stage(a, sd, mode_unused, row_on, dt_unused);
  if (!row_on) return;
  const int u = sd.u;
  const int64_t M = (int64_t)M1 * M2;
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;

  cplx<T>* twl = (cplx<T>*)smem;                          // M2 when TW_LDS
  const cplx<T>* tw = TW_LDS ? twl : (const cplx<T>*)a.twP2;
  cplx<T>* X = twl + (TW_LDS ? M2 : 0);                   // cmax*2 rows
  cplx<T>* nyq = X + (size_t)a.cmax * 2 * STR;            // cmax
  double* red = (double*)(nyq + a.cmax);                  // NWAVE * umax
  double* sdot = red + NWAVE * a.umax;                    // umax

  const int nrows = (k1 == 0 || 2 * k1 == M1) ? 1 : 2;
  auto row_of = [&](int rr) { return rr ? M1 - k1 : k1; };
  const int nunits = (k1 == 0) ? M2 / 2 + 1 : (nrows == 1 ? M2 / 2 : M2);
  if (TW_LDS) load_table<T, M2, NT>(twl, a.twP2);
  cplx<T> wk[UPT];   // w_L^k of this thread's combine units
#pragma unroll
  for (int i = 0; i < UPT; ++i) {
    const int unit = tid + i * NT;
    wk[i] = unit < nunits ? twL<T>(a, k1 + (int64_t)M1 * unit) : czero<T>();
  }
  if (k1 == 0) {   // partial dots of the column pass -> per-wave sums
    const int ngroups = M2 / a.g;
    for (int c = 0; c < u; ++c) {
      double sacc = 0.0;
      for (int q = tid; q < ngroups; q += NT) sacc += ldg(sd.dots + ((size_t)c * ngroups + q));
      sacc = wave_sum(sacc);
      if (lane == 0) red[wave * a.umax + c] = sacc;
    }
  }

  const bool chunked = sd.nch > 0;
  const int nch = chunked ? uniform_int(sd.nch) : 1;
  const auto chc = uniform_ptr(sd.tab + sd.o_chc);
  const auto chcols = uniform_ptr(sd.tab + sd.o_chcols);
  const auto cht = uniform_ptr(sd.tab + sd.o_cht);
  const auto poff = uniform_ptr(sd.tab);
  const auto pids = uniform_ptr(sd.tab + sd.o_pids);
  const auto pcoef = uniform_ptr(sd.coef);
  const auto pfrom = uniform_ptr(sd.tab + sd.o_pfrom);
  const cplx<T>* Z1 = (const cplx<T>*)sd.Z1;
  auto pair_of = [&](int unit, int& iB, int& rB) {
    if (k1 == 0) { iB = (M2 - unit) & (M2 - 1); rB = 0; }
    else if (nrows == 1) { iB = M2 - 1 - unit; rB = 0; }
    else { iB = M2 - 1 - unit; rB = 1; }
  };

  cplx<T> YA[UPT], YB[UPT];
#pragma unroll
  for (int i = 0; i < UPT; ++i) YA[i] = YB[i] = czero<T>();
  // tensor-train kernels: the running row vector of a term's matrix chain at
  // the unit's two bins, carried across chunks (cores); rows of at most 512
  // values only (the planner's limit), so other lengths compile it out
  constexpr bool TTK = M2 <= 512;
  constexpr int TTU = TTK ? UPT : 1, TTR = TTK ? kTTMaxRank : 1;
  cplx<T> vA[TTU][TTR], vB[TTU][TTR];
  const bool tt = TTK && sd.tt > 0;
  const auto ttrec = uniform_ptr(sd.tab + sd.o_tt);
  const auto ttid = uniform_ptr(sd.tab);
  // rows of at most 256 values (fewer bin pairs than threads): the chain of a
  // bin pair is shared by TOS adjacent lanes of one wavefront, lane og of the
  // pair holding outputs og, og + TOS, ... of every core's product and reading
  // the product's inputs from the pair's other lanes; each output sums the
  // same products in the same order as a single thread would
  constexpr int TOS = !TTK ? 1 : (NT / M2 >= kTTMaxRank ? kTTMaxRank : (NT / M2 > 1 ? NT / M2 : 1));
  constexpr bool TSPLIT = TOS > 1;
  constexpr int TOJ = kTTMaxRank / TOS;             // outputs per lane
  const int tu = wave * (64 / TOS) + lane / TOS;    // this lane's bin pair
  const int tog = lane % TOS, tbase = lane - tog;   // its outputs, the pair's first lane
  const bool ton = TSPLIT && tt && tu < nunits;
  cplx<T> sA[TOJ], sB[TOJ], YAs = czero<T>(), YBs = czero<T>();
#pragma unroll
  for (int j = 0; j < TOJ; ++j) sA[j] = sB[j] = czero<T>();
  const cplx<T> wks = ton ? twL<T>(a, k1 + (int64_t)M1 * tu) : czero<T>();
  for (int h = 0; h < nch; ++h) {
    const int c0 = chunked ? chc[h] : 0;
    const int nc = chunked ? chc[h + 1] - c0 : uniform_int(u);
    const int t0 = chunked ? cht[h] : 0;
    const int t1 = chunked ? cht[h + 1] : uniform_int(sd.Tp);
    lds_barrier();   // the previous chunk's combine is done with X
    const int nload = nc * nrows * M2;
    // unrolled so that several loads are in flight before their LDS stores wait
#pragma unroll 8
    for (int idx = tid; idx < nload; idx += NT) {
      const int cr = idx / M2, k2 = idx - cr * M2;
      const int c = nrows == 2 ? cr >> 1 : cr, rr = cr - c * nrows;
      const int gc = chunked ? chcols[c0 + c] : c;
      X[cr * STR + lds_pad(k2)] = ldg(Z1 + ((size_t)gc * M + (int64_t)row_of(rr) * M2 + k2));
    }
    lds_barrier();
    fft_batch<T, M2, -1, NB, STR, NT, StageRadix<T, M2>::value>(X, nc * nrows, tw);
    if constexpr (TSPLIT) {
      if (tt) {
        int iB = 0, rB = 0;
        if (ton) pair_of(tu, iB, rB);
        const int iA = tu;
        const bool zero_bin = (k1 == 0 && iA == 0);
        const bool self = (rB == 0 && iB == iA);
        if (ton) {   // the pair's columns unpacked by its lanes in turn
          for (int c = tog; c < nc; c += TOS) {
            const cplx<T> ZA = X[(c * nrows) * STR + lds_pad(iA)];
            const cplx<T> ZB = X[(c * nrows + rB) * STR + lds_pad(iB)];
            cplx<T> xa, xb;
            if (zero_bin) {
              xa = cplx<T>{ZA.re + ZA.im, Real<T>::zero()};
              xb = cplx<T>{ZA.re - ZA.im, Real<T>::zero()};
            } else {
              const cplx<T> zc = cconj(ZB);
              const cplx<T> E = cplx<T>{half_of(ZA.re + zc.re), half_of(ZA.im + zc.im)};
              const cplx<T> dd = csub(ZA, zc);
              const cplx<T> t = cmul(wks, cplx<T>{half_of(dd.im), half_of(-dd.re)});
              xa = cadd(E, t);
              xb = self ? xa : cconj(csub(E, t));
            }
            X[(c * nrows) * STR + lds_pad(iA)] = cnorm(xa);
            if (zero_bin) nyq[c] = cnorm(xb);
            else if (!self) X[(c * nrows + rB) * STR + lds_pad(iB)] = cnorm(xb);
          }
        }
        wave_lds_sync();   // a pair's lanes sit in one wavefront
        if (ton) {
          auto xat = [&](int c, bool b) -> cplx<T> {
            if (c < 0) return czero<T>();
            if (!b) return X[(c * nrows) * STR + lds_pad(iA)];
            return zero_bin ? nyq[c] : X[(c * nrows + rB) * STR + lds_pad(iB)];
          };
          for (int k = t0; k < t1; ++k) {
            const int term = ttrec[7 * k], lam = ttrec[7 * k + 1], d = ttrec[7 * k + 2];
            const int rin = ttrec[7 * k + 3], rout = ttrec[7 * k + 4], lo = ttrec[7 * k + 5];
            cplx<T> inA[kTTMaxRank], inB[kTTMaxRank];   // the pair's vector, from its lanes
            if (lam > 1) {
#pragma unroll
              for (int a2 = 0; a2 < kTTMaxRank; ++a2) {
                if (a2 < rin) {
                  inA[a2] = lane_read(sA[a2 / TOS], tbase + a2 % TOS);
                  inB[a2] = lane_read(sB[a2 / TOS], tbase + a2 % TOS);
                }
              }
            }
#pragma unroll
            for (int j = 0; j < TOJ; ++j) {
              const int b = tog + j * TOS;
              cplx<T> nA = czero<T>(), nB = czero<T>();
              if (b < rout) {
                if (lam == 1) {
                  nA = xat(ttid[lo + b], false);
                  nB = xat(ttid[lo + b], true);
                } else {
#pragma unroll
                  for (int a2 = 0; a2 < kTTMaxRank; ++a2) {
                    if (a2 < rin) {
                      const int c = ttid[lo + a2 * rout + b];
                      if (c >= 0) {
                        nA = cadd(nA, cmul(inA[a2], xat(c, false)));
                        nB = cadd(nB, cmul(inB[a2], xat(c, true)));
                      }
                    }
                  }
                }
              }
              sA[j] = cnorm(nA);
              sB[j] = cnorm(nB);
            }
            if (lam == d && tog == 0) {
              const T cf = Real<T>::from_d(pcoef[2 * term]);
              YAs = cnorm(cadd(YAs, cscale(sA[0], cf)));
              YBs = cnorm(cadd(YBs, cscale(sB[0], cf)));
            }
          }
        }
        continue;
      }
    }
#pragma unroll
    for (int i = 0; i < UPT; ++i) {
      const int unit = tid + i * NT;
      if (unit >= nunits) continue;
      int iB, rB;
      pair_of(unit, iB, rB);
      const int iA = unit;
      const bool zero_bin = (k1 == 0 && iA == 0);
      const bool self = (rB == 0 && iB == iA);
      // spectra of the chunk's real inputs at bins A and B (in place: the two
      // positions of a bin pair belong to this thread alone)
      for (int c = 0; c < nc; ++c) {
        const cplx<T> ZA = X[(c * nrows) * STR + lds_pad(iA)];
        const cplx<T> ZB = X[(c * nrows + rB) * STR + lds_pad(iB)];
        cplx<T> xa, xb;
        if (zero_bin) {
          xa = cplx<T>{ZA.re + ZA.im, Real<T>::zero()};
          xb = cplx<T>{ZA.re - ZA.im, Real<T>::zero()};
        } else {
          const cplx<T> zc = cconj(ZB);
          const cplx<T> E = cplx<T>{half_of(ZA.re + zc.re), half_of(ZA.im + zc.im)};
          const cplx<T> dd = csub(ZA, zc);
          const cplx<T> t = cmul(wk[i], cplx<T>{half_of(dd.im), half_of(-dd.re)});
          xa = cadd(E, t);
          xb = self ? xa : cconj(csub(E, t));
        }
        X[(c * nrows) * STR + lds_pad(iA)] = cnorm(xa);
        if (zero_bin) nyq[c] = cnorm(xb);
        else if (!self) X[(c * nrows + rB) * STR + lds_pad(iB)] = cnorm(xb);
      }
      if constexpr (TTK && !TSPLIT) {
        if (tt) {
          // cores [t0, t1) of this chunk: v <- v * (the core's matrix of
          // spectra at this bin); the first core of a term starts v, the last
          // adds v[0] / d! to the gain
          auto xat = [&](int c, bool b) -> cplx<T> {
            if (c < 0) return czero<T>();
            if (!b) return X[(c * nrows) * STR + lds_pad(iA)];
            return zero_bin ? nyq[c] : X[(c * nrows + rB) * STR + lds_pad(iB)];
          };
          for (int k = t0; k < t1; ++k) {
            const int term = ttrec[7 * k], lam = ttrec[7 * k + 1], d = ttrec[7 * k + 2];
            const int rin = ttrec[7 * k + 3], rout = ttrec[7 * k + 4], lo = ttrec[7 * k + 5];
            cplx<T> nA[TTR], nB[TTR];
#pragma unroll
            for (int b = 0; b < TTR; ++b) {
              nA[b] = nB[b] = czero<T>();
              if (b < rout) {
                if (lam == 1) {
                  nA[b] = xat(ttid[lo + b], false);
                  nB[b] = xat(ttid[lo + b], true);
                } else {
#pragma unroll
                  for (int a2 = 0; a2 < TTR; ++a2) {
                    if (a2 < rin) {
                      const int c = ttid[lo + a2 * rout + b];
                      if (c >= 0) {
                        nA[b] = cadd(nA[b], cmul(vA[i][a2], xat(c, false)));
                        nB[b] = cadd(nB[b], cmul(vB[i][a2], xat(c, true)));
                      }
                    }
                  }
                }
              }
            }
#pragma unroll
            for (int b = 0; b < TTR; ++b) {
              vA[i][b] = cnorm(nA[b]);
              vB[i][b] = cnorm(nB[b]);
            }
            if (lam == d) {
              const T cf = Real<T>::from_d(pcoef[2 * term]);
              YA[i] = cnorm(cadd(YA[i], cscale(vA[i][0], cf)));
              YB[i] = cnorm(cadd(YB[i], cscale(vB[i][0], cf)));
            }
          }
          continue;
        }
      }
      cplx<T> PA = czero<T>(), PB = czero<T>();
      for (int t = t0; t < t1; ++t) {
        const int oe = poff[t + 1];
        int o = pfrom[t];
        bool fresh = o == poff[t];
        for (; o < oe; ++o) {
          const int c = pids[o];
          const cplx<T> fa = X[(c * nrows) * STR + lds_pad(iA)];
          const cplx<T> fb = zero_bin ? nyq[c] : X[(c * nrows + rB) * STR + lds_pad(iB)];
          PA = fresh ? fa : cmul(PA, fa);
          PB = fresh ? fb : cmul(PB, fb);
          fresh = false;
        }
        const T cf = Real<T>::from_d(pcoef[t]);
        YA[i] = cnorm(cadd(YA[i], cscale(PA, cf)));
        YB[i] = cnorm(cadd(YB[i], cscale(PB, cf)));
      }
    }
  }
  lds_barrier();   // every chunk's reads of X are done: rows 0-1 take the packed sum
  auto pack = [&](int unit, cplx<T> A, cplx<T> B, cplx<T> w) {
    int iB, rB;
    pair_of(unit, iB, rB);
    const int iA = unit;
    if (k1 == 0 && iA == 0) {
      X[0] = cnorm(cplx<T>{A.re + B.re, A.re - B.re});
    } else {
      const cplx<T> s = cadd(A, cconj(B)), df = csub(A, cconj(B));
      X[lds_pad(iA)] = cnorm(cadd(s, cmul_i(cmulc(df, w))));
      if (!(rB == 0 && iB == iA)) X[rB * STR + lds_pad(iB)] = cnorm(cadd(cconj(s), cmul_i(cmul(w, cconj(df)))));
    }
  };
  if (TSPLIT && tt) {
    if (ton && tog == 0) pack(tu, YAs, YBs, wks);
  } else {
#pragma unroll
    for (int i = 0; i < UPT; ++i) {
      const int unit = tid + i * NT;
      if (unit < nunits) pack(unit, YA[i], YB[i], wk[i]);
    }
  }
  lds_barrier();
  fft_batch<T, M2, +1, NB, STR, NT, StageRadix<T, M2>::value>(X, nrows, tw);

  cplx<T>* V = (cplx<T>*)sd.V;
#pragma unroll
  for (int i = 0; i < VPT; ++i) {
    const int idx = tid + i * NT;
    if (idx < nrows * M2) {
      const int rr = idx / M2, j2 = idx - rr * M2;
      const int64_t e = (2 * (int64_t)j2 * row_of(rr == 1)) % a.L;
      stg(V + ((int64_t)row_of(rr) * M2 + j2), cnorm(cmulc(X[rr * STR + lds_pad(j2)], twL<T>(a, e))));
    }
  }

  // loss-term weights G_c (as in row_kernel), tables read from device memory
  if (k1 == 0) {
    for (int c = tid; c < u; c += NT) {
      double t = 0.0;
      for (int wv = 0; wv < NWAVE; ++wv) t += red[wv * a.umax + c];
      sdot[c] = t;
    }
    lds_barrier();
    if (tt) {
      // tensor-train terms: w = the product of the first d-1 cores' matrices
      // of dot products (a row vector), then G_c += w_r / (d-1)! for core d's
      // column c = (r, 0) (one thread: a few small products)
      double* gacc = sdot + a.umax;
      for (int c = tid; c < u; c += NT) gacc[c] = 0.0;
      lds_barrier();
      if (tid == 0) {
        double w[kTTMaxRank];
        const int ncores = ldg(sd.tab + sd.o_cht + sd.nch);
        for (int k = 0; k < ncores; ++k) {
          const int* cr = sd.tab + sd.o_tt + 7 * k;
          const int term = ldg(cr), lam = ldg(cr + 1), d = ldg(cr + 2), rin = ldg(cr + 3), rout = ldg(cr + 4);
          const int* gid = sd.tab + ldg(cr + 6);
          if (lam == d) {
            const double cq = ldg(sd.coef + 2 * term + 1);
            for (int r = 0; r < rin; ++r) {
              const int c = ldg(gid + r * rout);
              if (c >= 0) gacc[c] += cq * w[r];
            }
            continue;
          }
          double nw[kTTMaxRank];
          for (int b = 0; b < rout; ++b) {
            double acc = 0.0;
            for (int r = 0; r < rin; ++r) {
              const int c = ldg(gid + r * rout + b);
              const double s = c >= 0 ? sdot[c] : 0.0;
              acc += (lam == 1 ? 1.0 : w[r]) * s;
            }
            nw[b] = acc;
          }
          for (int b = 0; b < rout; ++b) w[b] = nw[b];
        }
      }
      lds_barrier();
      for (int c = tid; c < u; c += NT) stg(sd.G + c, gacc[c]);
      return;
    }
    const int* qoff = sd.tab + sd.o_qoff;
    const int* qids = sd.tab + sd.o_qids;
    const int* qkm = sd.tab + sd.o_qkm;
    for (int c = tid; c < u; c += NT) {
      double Gc = 0.0;
      for (int t = 0; t < sd.Tq; ++t) {
        if (ldg(qkm + t) != c) continue;
        double pr = ldg(sd.coef + (sd.Tp + t));
        for (int o = ldg(qoff + t); o < ldg(qoff + t + 1); ++o) pr *= sdot[ldg(qids + o)];
        Gc += pr;
      }
      stg(sd.G + c, Gc);
    }
  }
}

// ---------------------------------------------------------------------------
// Elementwise Heun stages of the unfused (term-by-term) evaluation:
//   stage 1: n~ = n + dt k1        stage 2: n = n + dt/2 (k1 + k2)
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kThreads) void heun_kernel(int stage, double* n, const double* k1, const double* k2,
                                                        double* ntil, double dt, int64_t total) {
  for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < total; i += (int64_t)gridDim.x * kThreads) {
    if (stage == 1) ntil[i] = n[i] + dt * k1[i];
    else n[i] = n[i] + 0.5 * dt * (k1[i] + k2[i]);
  }
}

hipError_t launch_heun(int stage, double* n, const double* k1, const double* k2, double* ntil, double dt,
                       int64_t total, hipStream_t s) {
  int64_t blocks = (total + kThreads - 1) / kThreads;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(heun_kernel, dim3((unsigned)blocks), dim3(kThreads), 0, s, stage, n, k1, k2, ntil, dt, total);
  return hipGetLastError();
}

// The serving engine's tick counter: one increment per tick, after every
// launch of the tick (stream order).
__global__ void tick_kernel(int64_t* t) {
  if (threadIdx.x == 0) t[0] += 1;
}

hipError_t launch_tick(int64_t* t, hipStream_t s) {
  hipLaunchKernelGGL(tick_kernel, dim3(1), dim3(64), 0, s, t);
  return hipGetLastError();
}

__global__ __launch_bounds__(kThreads) void zero_kernel(double* x, int64_t total) {
  for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < total; i += (int64_t)gridDim.x * kThreads)
    x[i] = 0.0;
}

hipError_t launch_zero(double* x, int64_t total, hipStream_t s) {
  int64_t blocks = (total + kThreads - 1) / kThreads;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(zero_kernel, dim3((unsigned)blocks), dim3(kThreads), 0, s, x, total);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Moments M0 = sum n, M1 = sum k n, and a non-finite count (binary64).
// ---------------------------------------------------------------------------
// Compensated binary64 accumulation (Neumaier's variant of Kahan summation,
// with Knuth's TwoSum for the rounding error of each addition): s + c carries
// the sum with an error of about one rounding of the result, independent of
// the number of terms.
__device__ __forceinline__ void comp_add(double& s, double& c, double x) {
#pragma clang fp contract(off)
  const double t = s + x;
  const double bb = t - s;
  c += (s - (t - bb)) + (x - bb);
  s = t;
}

// Moments of a batch of states: per block the compensated sums of n_k and of
// k n_k (the product's rounding error, from an FMA, is added as a term of its
// own) and the count of non-finite values.  part[5b..5b+4] = (M0 sum, M0
// compensation, M1 sum, M1 compensation, non-finite count).
__global__ __launch_bounds__(kThreads) void moments_kernel(const double* n, int64_t total, int64_t N,
                                                          double* part) {
  // no contraction: the product k n_k must be the rounded one that the
  // compensated sum adds, its rounding error being added separately
#pragma clang fp contract(off)
  __shared__ double r[5][kThreads];
  double s0 = 0, c0 = 0, s1 = 0, c1 = 0, bad = 0;
  for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < total;
       i += (int64_t)gridDim.x * kThreads) {
    const double v = n[i];
    if (!isfinite(v)) { bad += 1.0; continue; }
    comp_add(s0, c0, v);
    const double k = (double)(i % N + 1);
    const double pr = k * v;
    comp_add(s1, c1, pr);
    c1 += __builtin_fma(k, v, -pr);
  }
  const int tid = threadIdx.x;
  r[0][tid] = s0; r[1][tid] = c0; r[2][tid] = s1; r[3][tid] = c1; r[4][tid] = bad;
  __syncthreads();
  for (int w = kThreads / 2; w > 0; w >>= 1) {
    if (tid < w) {
      double a = r[0][tid], ca = r[1][tid] + r[1][tid + w];
      comp_add(a, ca, r[0][tid + w]);
      r[0][tid] = a; r[1][tid] = ca;
      double b = r[2][tid], cb = r[3][tid] + r[3][tid + w];
      comp_add(b, cb, r[2][tid + w]);
      r[2][tid] = b; r[3][tid] = cb;
      r[4][tid] += r[4][tid + w];
    }
    __syncthreads();
  }
  if (tid < 5) part[5 * blockIdx.x + tid] = r[tid][0];
}

// ---------------------------------------------------------------------------
// Host launchers
// ---------------------------------------------------------------------------
template <class T, int M1, bool LEAN, bool TILT = false>
static hipError_t launch_col_v(const LaunchArgs& a, hipStream_t s, size_t smem, dim3 grid) {
  static bool attr_done = false;   // raise the dynamic LDS cap once per instantiation
  if (!attr_done) {
    hipError_t e = hipFuncSetAttribute((const void*)col_kernel<T, M1, LEAN, TILT>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024 - 4096);
    if (e != hipSuccess) return e;
    attr_done = true;
  }
  hipLaunchKernelGGL((col_kernel<T, M1, LEAN, TILT>), grid, dim3(kColThreads), smem, s, a);
  return hipGetLastError();
}

template <class T, int M1>
static hipError_t launch_col_t(const LaunchArgs& a, hipStream_t s) {
  constexpr int GMAX = (1024 / M1) > 0 ? 1024 / M1 : 1;
  const size_t tbuf = (size_t)a.ub * GMAX * lds_len(M1);   // transform buffer
  dim3 grid(a.nslots * (a.M2 / a.g) * (a.usplit > 1 ? a.usplit : 1));
  // from M1 = 1024 the register cap of the lean variant (two workgroups per CU)
  // spills the per-item state to scratch; those launches keep every register
  if constexpr (M1 <= kLeanMaxM1) {
    if (a.lean && a.tilt == 0.0) return launch_col_v<T, M1, true>(a, s, ((size_t)M1 + tbuf) * sizeof(cplx<T>), grid);
  }
  constexpr int nbuf = kColPingPong<T, M1, false> ? 2 : 1;
  if constexpr (std::is_same<T, float>::value) {   // tilted launches take the full variant
    if (a.tilt != 0.0) return launch_col_v<T, M1, false, true>(a, s, ((size_t)M1 + nbuf * tbuf) * sizeof(cplx<T>), grid);
  }
  return launch_col_v<T, M1, false>(a, s, ((size_t)M1 + nbuf * tbuf) * sizeof(cplx<T>), grid);
}

template <class T>
static hipError_t launch_col_p(const LaunchArgs& a, hipStream_t s) {
  switch (a.M1) {
    case 4: return launch_col_t<T, 4>(a, s);
    case 8: return launch_col_t<T, 8>(a, s);
    case 16: return launch_col_t<T, 16>(a, s);
    case 32: return launch_col_t<T, 32>(a, s);
    case 64: return launch_col_t<T, 64>(a, s);
    case 128: return launch_col_t<T, 128>(a, s);
    case 256: return launch_col_t<T, 256>(a, s);
    case 512: return launch_col_t<T, 512>(a, s);
    case 1024: return launch_col_t<T, 1024>(a, s);
    case 2048: return launch_col_t<T, 2048>(a, s);
    // mixed-radix lengths (the planner's supported set)
    case 96: return launch_col_t<T, 96>(a, s);
    case 192: return launch_col_t<T, 192>(a, s);
    case 384: return launch_col_t<T, 384>(a, s);
    case 768: return launch_col_t<T, 768>(a, s);
    case 1536: return launch_col_t<T, 1536>(a, s);
    case 160: return launch_col_t<T, 160>(a, s);
    case 320: return launch_col_t<T, 320>(a, s);
    case 640: return launch_col_t<T, 640>(a, s);
    case 1280: return launch_col_t<T, 1280>(a, s);
  }
  return hipErrorInvalidValue;
}

size_t row_smem_bytes(int prec, int umax, int M2, int tab_max, int coef_max) {
  size_t cs = prec == 1 ? 8 : 16;
  return (size_t)(M2 <= 512 ? M2 : 0) * cs + (size_t)umax * 2 * lds_len(M2) * cs + (size_t)umax * cs +
         (size_t)coef_max * 8 + (size_t)(2 * kThreads / 64 + 1) * umax * 8 + (size_t)tab_max * 4 + 16;
}

size_t row_chunk_smem_bytes(int prec, int cmax, int umax, int M2, int, int) {
  size_t cs = prec == 1 ? 8 : 16;
  // rows, Nyquist values, per-wave partial dots, dot products, loss weights (tensor-train terms)
  return (size_t)(M2 <= 512 ? M2 : 0) * cs + (size_t)cmax * 2 * lds_len(M2) * cs + (size_t)cmax * cs +
         (size_t)(2 * kThreads / 64 + 2) * umax * 8 + 16;
}

int col_batch(int prec, int M1, int u, int nworkgroups) {
  size_t cs = prec == 1 ? 8 : 16;
  size_t gmax = 1024 / M1 > 0 ? 1024 / M1 : 1;
  const bool lean = nworkgroups >= kLeanWorkgroups && M1 <= kLeanMaxM1;
  // the float-float full variant keeps a second transform buffer below the
  // longest columns
  size_t per = gmax * lds_len(M1) * cs * ((lean || M1 >= 2048 || prec != 2) ? 1 : 2);
  long ub = ((long)kColLdsBudget - (long)(M1 * cs)) / (long)per;
  if (ub < 1) ub = 1;
  if (ub > kColBatch) ub = kColBatch;
  if (ub > u) ub = u < 1 ? 1 : u;
  // a launch that already fills the GPU gains more from occupancy (small LDS
  // per workgroup) than from transforming several columns per workgroup,
  // except where its wavefronts transform one column each (columns of 256 and
  // 512 values): there a group of several columns keeps them all busy
  if (nworkgroups >= kLeanWorkgroups && !(lean && (M1 == 256 || M1 == 512))) ub = 1;
  return (int)ub;
}

template <class T, int M2>
static hipError_t launch_row_t(const LaunchArgs& a, hipStream_t s) {
  // saturating launches trade registers for several resident work groups per CU;
  // smaller ones keep every register (no spills) for the shortest chains
  if (a.cmax > 0) {
    const size_t smem = row_chunk_smem_bytes(sizeof(cplx<T>) == 8 ? 1 : 0, a.cmax, a.umax, a.M2, 0, 0);
    static bool chunk_attr = false;
    if (!chunk_attr) {
      hipError_t e = hipFuncSetAttribute((const void*)row_chunk_kernel<T, M2>,
                                         hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024 - 4096);
      if (e != hipSuccess) return e;
      chunk_attr = true;
    }
    if (smem > 160 * 1024 - 4096) return hipErrorInvalidValue;
    hipLaunchKernelGGL((row_chunk_kernel<T, M2>), dim3(a.nslots * (a.M1 / 2 + 1)), dim3(kChunkThreads), smem, s, a);
    return hipGetLastError();
  }
  constexpr bool kHasLean = M2 <= 512;
  const bool lean = kHasLean && (int64_t)a.nslots * (a.M1 / 2 + 1) >= kLeanWorkgroups;
  const size_t smem = row_smem_bytes(sizeof(cplx<T>) == 8 ? 1 : 0, a.umax, a.M2, a.tab_max, a.coef_max);
  const void* fn = lean ? (const void*)row_kernel<T, M2, kHasLean> : (const void*)row_kernel<T, M2, false>;
  static bool attr_done[2] = {false, false};   // raise the dynamic LDS cap once per instantiation
  if (!attr_done[lean]) {
    hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024 - 4096);
    if (e != hipSuccess) return e;
    attr_done[lean] = true;
  }
  dim3 grid(a.nslots * (a.M1 / 2 + 1));
  if (lean)
    hipLaunchKernelGGL((row_kernel<T, M2, kHasLean>), grid, dim3(RowThreads<M2, kHasLean>::value), smem, s, a);
  else
    hipLaunchKernelGGL((row_kernel<T, M2, false>), grid, dim3(RowThreads<M2, false>::value), smem, s, a);
  return hipGetLastError();
}

template <class T>
static hipError_t launch_row_p(const LaunchArgs& a, hipStream_t s) {
  switch (a.M2) {
    case 2: return launch_row_t<T, 2>(a, s);
    case 4: return launch_row_t<T, 4>(a, s);
    case 8: return launch_row_t<T, 8>(a, s);
    case 16: return launch_row_t<T, 16>(a, s);
    case 32: return launch_row_t<T, 32>(a, s);
    case 64: return launch_row_t<T, 64>(a, s);
    case 128: return launch_row_t<T, 128>(a, s);
    case 256: return launch_row_t<T, 256>(a, s);
    case 512: return launch_row_t<T, 512>(a, s);
    case 1024: return launch_row_t<T, 1024>(a, s);
    case 2048: return launch_row_t<T, 2048>(a, s);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_col(int prec, const LaunchArgs& a, hipStream_t s) {
  if (prec == 0) return launch_col_p<double>(a, s);
  if (prec == 1) return launch_col_p<float>(a, s);
  return launch_col_p<ff>(a, s);
}

hipError_t launch_row(int prec, const LaunchArgs& a, hipStream_t s) {
  if (prec == 0) return launch_row_p<double>(a, s);
  if (prec == 1) return launch_row_p<float>(a, s);
  return launch_row_p<ff>(a, s);
}

hipError_t launch_moments(const double* n, int64_t total, int64_t N, double* part, int nblocks,
                          hipStream_t s) {
  hipLaunchKernelGGL(moments_kernel, dim3(nblocks), dim3(kThreads), 0, s, n, total, N, part);
  return hipGetLastError();
}

}  // namespace agg
