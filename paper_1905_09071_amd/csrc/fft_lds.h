// Batched FFTs of lengths 2^k, 3 2^k and 5 2^k held in LDS, for one
// workgroup of NT threads.
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

// multiplication by DIR * i
template <class T, int DIR> __device__ __forceinline__ cplx<T> mul_dir_i(cplx<T> x) {
  return DIR < 0 ? cmul_negi(x) : cmul_i(x);
}

// Length-3 DFT: y_0 = x_0 + a, y_{1,2} = x_0 - a/2 +- DIR i (sqrt(3)/2) b with
// a = x_1 + x_2, b = x_1 - x_2 (the roots w^1, w^2 = -1/2 +- DIR i sqrt(3)/2).
template <class T, int DIR> __device__ __forceinline__ void dft3(cplx<T>* v) {
  const T h = Real<T>::from_d(0.5);
  const T s3 = Real<T>::from_d(0.86602540378443864676372317075293618347);   // sqrt(3)/2
  const cplx<T> a = cadd(v[1], v[2]), b = csub(v[1], v[2]);
  const cplx<T> m = csub(v[0], cscale(a, h));
  const cplx<T> t = mul_dir_i<T, DIR>(cscale(b, s3));
  v[0] = cadd(v[0], a);
  v[1] = cadd(m, t);
  v[2] = csub(m, t);
}

// Length-5 DFT from the symmetric sums a_1 = x_1 + x_4, a_2 = x_2 + x_3 and
// differences b_1 = x_1 - x_4, b_2 = x_2 - x_3, with c_k = cos(2 pi k/5),
// s_k = sin(2 pi k/5):
//   y_0 = x_0 + a_1 + a_2
//   y_{1,4} = x_0 + c_1 a_1 + c_2 a_2 +- DIR i (s_1 b_1 + s_2 b_2)
//   y_{2,3} = x_0 + c_2 a_1 + c_1 a_2 +- DIR i (s_2 b_1 - s_1 b_2)
template <class T, int DIR> __device__ __forceinline__ void dft5(cplx<T>* v) {
  const T c1 = Real<T>::from_d(0.30901699437494742410229341718281905886);
  const T c2 = Real<T>::from_d(-0.80901699437494742410229341718281905886);
  const T s1 = Real<T>::from_d(0.95105651629515357211643933337938214340);
  const T s2 = Real<T>::from_d(0.58778525229247312916870595463907276860);
  const cplx<T> a1 = cadd(v[1], v[4]), b1 = csub(v[1], v[4]);
  const cplx<T> a2 = cadd(v[2], v[3]), b2 = csub(v[2], v[3]);
  const cplx<T> m1 = cadd(v[0], cadd(cscale(a1, c1), cscale(a2, c2)));
  const cplx<T> m2 = cadd(v[0], cadd(cscale(a1, c2), cscale(a2, c1)));
  const cplx<T> t1 = mul_dir_i<T, DIR>(cadd(cscale(b1, s1), cscale(b2, s2)));
  const cplx<T> t2 = mul_dir_i<T, DIR>(csub(cscale(b1, s2), cscale(b2, s1)));
  v[0] = cadd(v[0], cadd(a1, a2));
  v[1] = cadd(m1, t1);
  v[4] = csub(m1, t1);
  v[2] = cadd(m2, t2);
  v[3] = csub(m2, t2);
}

template <class T, int R, int DIR> __device__ __forceinline__ void dftR(cplx<T>* v) {
  if constexpr (R == 2) dft2<T, DIR>(v);
  else if constexpr (R == 3) dft3<T, DIR>(v);
  else if constexpr (R == 4) dft4<T, DIR>(v);
  else if constexpr (R == 5) dft5<T, DIR>(v);
  else dft8<T, DIR>(v);
}

// Radix of the stage at span NS of a length-P transform with largest
// power-of-two radix RMAX: lengths 3 2^k and 5 2^k take their odd factor in
// the first stage, then powers of two (radix RMAX while at least RMAX remains).
__host__ __device__ constexpr int stage_radix(int P, int NS, int RMAX) {
  return (NS == 1 && P % 5 == 0) ? 5 : (NS == 1 && P % 3 == 0) ? 3 : (P / NS >= RMAX ? RMAX : P / NS);
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
  for (int ns = NS0; ns < P; ns *= stage_radix(P, ns, RMAX)) ++n;
  return n;
}

template <class T, int P, int NS, int DIR, int NB, int STR, int NT, int RMAX>
__device__ __forceinline__ void fft_stages_pp(cplx<T>* a, cplx<T>* b, int nfft, const cplx<T>* __restrict__ tw) {
  if constexpr (NS < P) {
    constexpr int R = stage_radix(P, NS, RMAX);
    fft_stage_pp<T, P, R, NS, DIR, NB, STR, NT>(a, b, nfft, tw);
    fft_stages_pp<T, P, NS * R, DIR, NB, STR, NT, RMAX>(b, a, nfft, tw);
  }
}

template <class T, int P, int NS, int DIR, int NB, int STR, int NT, int RMAX>
__device__ __forceinline__ void fft_stages(cplx<T>* buf, int nfft, const cplx<T>* __restrict__ tw) {
  if constexpr (NS < P) {
    constexpr int R = stage_radix(P, NS, RMAX);
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
