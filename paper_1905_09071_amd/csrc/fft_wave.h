// Power-of-two FFTs held by one wavefront in registers.
//
// A transform of length P = 64 E lives in the E registers v[0..E) of the 64
// lanes of one wavefront: lane l, register e holds element l + 64 e
// ("lane-major", natural order), on entry and on exit.  The stages are those
// of the Stockham formulation used by fft_lds.h (span NS, radix R: butterfly b
// takes elements b + r P/R, twiddles input r by w_{NS R}^{(b mod NS) r}, and
// writes output r to (b div NS) NS R + b mod NS + r NS), with every radix R
// dividing E.  Butterfly b = l + 64 q (q < E/R) then reads registers
// q + r E/R of its own lane, so a stage needs no data movement on input; its
// outputs are moved back to lane-major order through a wavefront-private LDS
// region.  After the last stage (NS R = P) the outputs already sit in
// lane-major order.  A length-P transform thus costs log_R(P) - 1 exchanges,
// and no workgroup barrier: LDS operations of one wavefront complete in issue
// order, so each exchange only has to keep the compiler from moving its reads
// above its writes and wait for the writes (lgkmcnt).
#pragma once
#include "fft_lds.h"

namespace agg {

// Exchange region of a transform: P values at lds_pad positions (one pad slot
// after every 16, the layout of fft_lds.h), so a row already held in LDS can
// serve as its own exchange region.  The lane-major reads are conflict-free;
// the scattered stage writes (lane stride R) meet at most two lanes per bank
// group.

// Orders this wavefront's LDS writes before its following LDS reads (no
// workgroup barrier; waits for LDS only, not for outstanding global loads).
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

template <class T, int P, int E, int NS, int DIR, int RMAX>
__device__ __forceinline__ void fft_wave_stages(cplx<T> (&v)[E], cplx<T>* scr, const cplx<T>* __restrict__ tw) {
  static_assert(E == 2 || E == 4 || E == 8, "values per lane");
  static_assert(RMAX <= E && E % RMAX == 0, "the largest radix divides the values per lane");
  if constexpr (NS < P) {
    constexpr int REM = P / NS;
    constexpr int R = REM >= RMAX ? RMAX : REM;   // radix of this stage (divides E)
    constexpr int Q = E / R;                // butterflies per lane
    constexpr bool LAST = NS * R == P;
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      const int b = lane + 64 * q;
      cplx<T> x[R];
#pragma unroll
      for (int r = 0; r < R; ++r) x[r] = v[q + r * Q];
      const int j = b % NS;
      if constexpr (NS > 1) {
#pragma unroll
        for (int r = 1; r < R; ++r) x[r] = twiddle_apply<T, DIR>(x[r], tw[j * r * (P / (NS * R))]);
      }
      dftR<T, R, DIR>(x);
      if constexpr (LAST) {
        // renormalised like every stage output of fft_lds.h, so that both
        // formulations give the same values
#pragma unroll
        for (int r = 0; r < R; ++r) v[q + r * Q] = cnorm(x[r]);
      } else {
        const int base = (b / NS) * NS * R + j;
#pragma unroll
        for (int r = 0; r < R; ++r) scr[lds_pad(base + r * NS)] = cnorm(x[r]);
      }
    }
    if constexpr (!LAST) {
      wave_lds_sync();
#pragma unroll
      for (int e = 0; e < E; ++e) v[e] = scr[lds_pad(lane + 64 * e)];
      // the next stage's writes must not overtake these reads (same wavefront:
      // LDS order is issue order; this only pins the compiler's order)
      __builtin_amdgcn_wave_barrier();
      fft_wave_stages<T, P, E, NS * R, DIR, RMAX>(v, scr, tw);
    }
  }
}

// Transforms the lane-major sequence in v (length P = 64 E) in place, with the
// stage sequence of fft_batch<..., RMAX> (radix RMAX while at least RMAX
// remains, then the rest): the same operations on the same values, so the
// result is bit for bit that of fft_lds.h.  RMAX must divide E.
// scr: this wavefront's region of lds_len(P) values (LDS); tw[e] = w_P^e, e < P
// (any memory the wavefront can read; LDS in the kernels).  DIR = -1 forward,
// +1 the unnormalised inverse.
template <class T, int P, int DIR, int RMAX = P / 64>
__device__ __forceinline__ void fft_wave(cplx<T> (&v)[P / 64], cplx<T>* scr, const cplx<T>* __restrict__ tw) {
  static_assert(P >= 128 && P <= 512 && (P & (P - 1)) == 0, "2 to 8 values per lane");
  fft_wave_stages<T, P, P / 64, 1, DIR, RMAX>(v, scr, tw);
}

// The same transform for a sequence held in LDS at lds_pad positions of the
// region reg (natural order in and out): read lane-major, transformed in
// registers with reg as exchange space, written back renormalised.  The
// region must be visible to the wavefront (a barrier after other wavefronts
// wrote it); other wavefronts must not touch it until a barrier follows.
template <class T, int P, int DIR, int RMAX = P / 64>
__device__ __forceinline__ void fft_wave_lds(cplx<T>* reg, const cplx<T>* __restrict__ tw) {
  cplx<T> v[P / 64];
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int e = 0; e < P / 64; ++e) v[e] = reg[lds_pad(lane + 64 * e)];
  fft_wave<T, P, DIR, RMAX>(v, reg, tw);
#pragma unroll
  for (int e = 0; e < P / 64; ++e) reg[lds_pad(lane + 64 * e)] = v[e];
}

}  // namespace agg
