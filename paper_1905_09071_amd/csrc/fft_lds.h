// Batched power-of-two FFTs held in LDS, for one workgroup of NT threads.
//
// Stockham autosort formulation: stage s with radix R and span NS (product of
// the radices before it) takes butterfly b (0 <= b < P/R) from positions
// b + r*P/R, twiddles input r by w_{NS*R}^{(b mod NS)*r}, runs a length-R DFT
// in registers and writes output r to (b div NS)*NS*R + (b mod NS) + r*NS.
// After the last stage the data sit in natural order.  Each stage reads all
// of its inputs into registers, synchronises, then writes in place, so one LDS
// buffer suffices.  DIR = -1 is the forward transform exp(-2 pi i jk/P),
// DIR = +1 the unnormalised inverse.
#pragma once
#include "arith.h"

namespace agg {

constexpr int kThreads = 256;

// Workgroup barrier that orders LDS only.  Unlike __syncthreads() it does not
// wait for outstanding global loads and stores, so prefetched global data stays
// in flight across the LDS-only stages of a transform.
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// LDS position of element i of a transform: one pad slot after every 16
// elements.  Stockham stage writes land at stride R*16 bytes in the first
// stages, which without padding puts up to 32 lanes of a wave on one bank
// group; with it every stage stays at the 4-way minimum of 16-byte accesses.
__host__ __device__ constexpr int lds_pad(int i) { return i + (i >> 4); }
// padded length of one transform of P elements in LDS
__host__ __device__ constexpr int lds_len(int P) { return P + (P >> 4); }

// tw[e] = exp(-2 pi i e / P) in the working precision
template <class T, int DIR>
__device__ __forceinline__ cplx<T> twiddle_apply(cplx<T> v, cplx<T> w) {
  return DIR < 0 ? cmul(v, w) : cmulc(v, w);
}

template <class T, int DIR> __device__ __forceinline__ void dft2(cplx<T>* v) {
  cplx<T> a = v[0], b = v[1];
  v[0] = cadd(a, b);
  v[1] = csub(a, b);
}

template <class T, int DIR> __device__ __forceinline__ void dft4(cplx<T>* v) {
  cplx<T> a0 = cadd(v[0], v[2]), a1 = csub(v[0], v[2]);
  cplx<T> a2 = cadd(v[1], v[3]), d = csub(v[1], v[3]);
  cplx<T> a3 = DIR < 0 ? cmul_negi(d) : cmul_i(d);
  v[0] = cadd(a0, a2);
  v[2] = csub(a0, a2);
  v[1] = cadd(a1, a3);
  v[3] = csub(a1, a3);
}

// (x) * exp(DIR * 2 pi i / 8) = x * (1 + DIR i)/sqrt(2)
template <class T, int DIR> __device__ __forceinline__ cplx<T> rot8(cplx<T> x, T h) {
  return DIR < 0 ? cplx<T>{(x.re + x.im) * h, (x.im - x.re) * h}
                 : cplx<T>{(x.re - x.im) * h, (x.im + x.re) * h};
}

template <class T, int DIR> __device__ __forceinline__ void dft8(cplx<T>* v) {
  const T h = Real<T>::from_d(0.70710678118654752440084436210484903928);
  cplx<T> e[4] = {v[0], v[2], v[4], v[6]};
  cplx<T> o[4] = {v[1], v[3], v[5], v[7]};
  dft4<T, DIR>(e);
  dft4<T, DIR>(o);
  // twiddles w8^k, k = 0..3
  cplx<T> t1 = rot8<T, DIR>(o[1], h);
  cplx<T> t2 = DIR < 0 ? cmul_negi(o[2]) : cmul_i(o[2]);
  cplx<T> t3 = rot8<T, DIR>(DIR < 0 ? cmul_negi(o[3]) : cmul_i(o[3]), h);
  v[0] = cadd(e[0], o[0]);
  v[4] = csub(e[0], o[0]);
  v[1] = cadd(e[1], t1);
  v[5] = csub(e[1], t1);
  v[2] = cadd(e[2], t2);
  v[6] = csub(e[2], t2);
  v[3] = cadd(e[3], t3);
  v[7] = csub(e[3], t3);
}

template <class T, int R, int DIR> __device__ __forceinline__ void dftR(cplx<T>* v) {
  if constexpr (R == 2) dft2<T, DIR>(v);
  else if constexpr (R == 4) dft4<T, DIR>(v);
  else dft8<T, DIR>(v);
}

// One Stockham stage over `nfft` transforms (nfft <= NB) stored at stride STR.
template <class T, int P, int R, int NS, int DIR, int NB, int STR, int NT>
__device__ __forceinline__ void fft_stage(cplx<T>* buf, int nfft, const cplx<T>* __restrict__ tw) {
  constexpr int BPF = P / R;
  constexpr int TOT = NB * BPF;
  constexpr int K = (TOT + NT - 1) / NT;
  const int tid = threadIdx.x;
  const int nvalid = nfft * BPF;
  cplx<T> v[K][R];
#pragma unroll
  for (int kk = 0; kk < K; ++kk) {
    int bg = tid + kk * NT;
    if (bg < nvalid) {
      int f = bg / BPF, b = bg % BPF;
#pragma unroll
      for (int r = 0; r < R; ++r) v[kk][r] = buf[f * STR + lds_pad(b + r * BPF)];
    }
  }
  lds_barrier();
#pragma unroll
  for (int kk = 0; kk < K; ++kk) {
    int bg = tid + kk * NT;
    if (bg < nvalid) {
      int f = bg / BPF, b = bg % BPF;
      int j = b % NS;
      if constexpr (NS > 1) {
#pragma unroll
        for (int r = 1; r < R; ++r) {
          int e = j * r * (P / (NS * R));
          v[kk][r] = twiddle_apply<T, DIR>(v[kk][r], tw[e]);
        }
      }
      dftR<T, R, DIR>(v[kk]);
      int base = (b / NS) * NS * R + j;
#pragma unroll
      for (int r = 0; r < R; ++r) buf[f * STR + lds_pad(base + r * NS)] = cnorm(v[kk][r]);
    }
  }
  lds_barrier();
}

// The same stage reading from `src` and writing to a second buffer `dst`:
// no barrier is needed between the reads and the writes, one after them.
template <class T, int P, int R, int NS, int DIR, int NB, int STR, int NT>
__device__ __forceinline__ void fft_stage_pp(const cplx<T>* src, cplx<T>* dst, int nfft,
                                             const cplx<T>* __restrict__ tw) {
  constexpr int BPF = P / R;
  constexpr int TOT = NB * BPF;
  constexpr int K = (TOT + NT - 1) / NT;
  const int tid = threadIdx.x;
  const int nvalid = nfft * BPF;
#pragma unroll
  for (int kk = 0; kk < K; ++kk) {
    int bg = tid + kk * NT;
    if (bg < nvalid) {
      int f = bg / BPF, b = bg % BPF;
      cplx<T> v[R];
#pragma unroll
      for (int r = 0; r < R; ++r) v[r] = src[f * STR + lds_pad(b + r * BPF)];
      int j = b % NS;
      if constexpr (NS > 1) {
#pragma unroll
        for (int r = 1; r < R; ++r) {
          int e = j * r * (P / (NS * R));
          v[r] = twiddle_apply<T, DIR>(v[r], tw[e]);
        }
      }
      dftR<T, R, DIR>(v);
      int base = (b / NS) * NS * R + j;
#pragma unroll
      for (int r = 0; r < R; ++r) dst[f * STR + lds_pad(base + r * NS)] = cnorm(v[r]);
    }
  }
  lds_barrier();
}

// Number of Stockham stages of a length-P transform with radices up to RMAX,
// from span NS0 on.
__host__ __device__ constexpr int fft_nstages(int P, int RMAX, int NS0 = 1) {
  int n = 0;
  for (int ns = NS0; ns < P; ns *= (P / ns >= RMAX ? RMAX : P / ns)) ++n;
  return n;
}

template <class T, int P, int NS, int DIR, int NB, int STR, int NT, int RMAX>
__device__ __forceinline__ void fft_stages_pp(cplx<T>* a, cplx<T>* b, int nfft, const cplx<T>* __restrict__ tw) {
  if constexpr (NS < P) {
    constexpr int REM = P / NS;
    constexpr int R = REM >= RMAX ? RMAX : REM;
    fft_stage_pp<T, P, R, NS, DIR, NB, STR, NT>(a, b, nfft, tw);
    fft_stages_pp<T, P, NS * R, DIR, NB, STR, NT, RMAX>(b, a, nfft, tw);
  }
}

template <class T, int P, int NS, int DIR, int NB, int STR, int NT, int RMAX>
__device__ __forceinline__ void fft_stages(cplx<T>* buf, int nfft, const cplx<T>* __restrict__ tw) {
  if constexpr (NS < P) {
    constexpr int REM = P / NS;
    constexpr int R = REM >= RMAX ? RMAX : REM;
    fft_stage<T, P, R, NS, DIR, NB, STR, NT>(buf, nfft, tw);
    fft_stages<T, P, NS * R, DIR, NB, STR, NT, RMAX>(buf, nfft, tw);
  }
}

// Transforms `count` sequences of length P at stride STR (>= lds_len(P)),
// element i of sequence f at buf[f*STR + lds_pad(i)], NB at a time.  Every
// thread of the block must call this (it synchronises internally, on LDS only:
// the caller must have made its LDS input visible with lds_barrier() or
// __syncthreads() first).
// RMAX: largest radix per stage.  Radix 8 needs the fewest LDS passes (best
// when many workgroups share a CU); radix 4 gives shorter per-thread chains and
// more parallel butterflies (best when one workgroup per CU is latency-bound).
// NS0 > 1 starts after the first stage (the caller has written that stage's
// output itself, e.g. the broadcast of an input whose nonzeros all fall in
// the first radix-R block).
template <class T, int P, int DIR, int NB, int STR, int NT = kThreads, int RMAX = 8, int NS0 = 1>
__device__ __forceinline__ void fft_batch(cplx<T>* buf, int count, const cplx<T>* __restrict__ tw) {
  for (int c0 = 0; c0 < count; c0 += NB) {
    int nf = count - c0 < NB ? count - c0 : NB;
    fft_stages<T, P, NS0, DIR, NB, STR, NT, RMAX>(buf + c0 * STR, nf, tw);
  }
}

// fft_batch with a second buffer `alt` of the same layout: one barrier per
// stage instead of two.  The stages alternate between the buffers; the result
// is in the returned one (buf or alt, by the parity of the stage count).
template <class T, int P, int DIR, int NB, int STR, int NT = kThreads, int RMAX = 8, int NS0 = 1>
__device__ __forceinline__ cplx<T>* fft_batch_pp(cplx<T>* buf, cplx<T>* alt, int count,
                                                 const cplx<T>* __restrict__ tw) {
  for (int c0 = 0; c0 < count; c0 += NB) {
    int nf = count - c0 < NB ? count - c0 : NB;
    fft_stages_pp<T, P, NS0, DIR, NB, STR, NT, RMAX>(buf + c0 * STR, alt + c0 * STR, nf, tw);
  }
  return (fft_nstages(P, RMAX, NS0) & 1) ? alt : buf;
}

}  // namespace agg
