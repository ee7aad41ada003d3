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

#include "fft_lds.h"
#include "kernels.h"

namespace agg {

template <class T>
__device__ __forceinline__ cplx<T> twL(const LaunchArgs& a, int64_t e) {
  const cplx<T>* lo = (const cplx<T>*)a.twLlo;
  const cplx<T>* hi = (const cplx<T>*)a.twLhi;
  int64_t mask = (int64_t(1) << a.b) - 1;
  return cmul(hi[e >> a.b], lo[e & mask]);
}

// ---------------------------------------------------------------------------
// Column pass.  Work item = (slot, group of g adjacent columns j2).
// ---------------------------------------------------------------------------
template <class T, int M1>
__global__ __launch_bounds__(kThreads) void col_kernel(LaunchArgs a) {
  constexpr int GMAX = (2048 / M1) > 0 ? 2048 / M1 : 1;
  constexpr int STR = M1;
  constexpr int CAP = GMAX * M1;
  constexpr int IPT = (CAP + kThreads - 1) / kThreads;
  __shared__ cplx<T> buf[CAP];
  __shared__ double red[kThreads];

  const int M2 = a.M2, g = a.g;
  const int ngroups = M2 / g;
  const int slot = blockIdx.x / ngroups;
  const int grp = blockIdx.x - slot * ngroups;
  const SlotDesc sd = a.slots[slot];
  const int mode = a.mode >= 0 ? a.mode : sd.mode;
  if (mode == CM_NONE) return;
  const double dt = a.mode >= 0 ? a.dt : sd.dt;
  const int64_t N = sd.N;
  const int64_t M = (int64_t)M1 * M2;
  const int j2_0 = grp * g;
  const int tid = threadIdx.x;
  const int nitems = g * M1;
  double* state = a.ext_state ? a.ext_state + (size_t)slot * N : sd.n_state;
  const cplx<T>* twP1 = (const cplx<T>*)a.twP1;

  double s0[IPT], s1[IPT];   // new state at sizes 2j and 2j+1 of each item

  if (mode_has_inverse(mode)) {
    const cplx<T>* V = (const cplx<T>*)sd.V;
#pragma unroll
    for (int it = 0; it < IPT; ++it) {
      int idx = tid + it * kThreads;
      if (idx < nitems) {
        int k1 = idx / g, jl = idx - k1 * g;
        buf[jl * STR + k1] = V[(int64_t)k1 * M2 + j2_0 + jl];
      }
    }
    __syncthreads();
    fft_batch<T, M1, +1, GMAX, STR>(buf, g, twP1);

    const double invL = 1.0 / (double)a.L;
    const bool stage2 = (mode == CM_H2 || mode == CM_H2_FWD);
    const double* ev = stage2 ? sd.ntil : state;   // state at which f is taken
    double* out = a.ext_out ? a.ext_out + (size_t)slot * N : sd.out;
    const int u = sd.u;
#pragma unroll
    for (int it = 0; it < IPT; ++it) {
      int idx = tid + it * kThreads;
      s0[it] = 0.0;
      s1[it] = 0.0;
      if (idx < nitems) {
        int j1 = idx / g, jl = idx - j1 * g;
        int64_t j = j2_0 + jl + (int64_t)M2 * j1;
        cplx<T> w = buf[jl * STR + j1];
        double y[2] = {Real<T>::to_d(w.re), Real<T>::to_d(w.im)};
#pragma unroll
        for (int e = 0; e < 2; ++e) {
          int64_t s = 2 * j + e;
          double val = 0.0;
          if (s >= 1 && s <= N) {
            double p = s >= 2 ? y[e] * invL : 0.0;
            double gk = 0.0;
            for (int c = 0; c < u; ++c) gk += sd.cols[(size_t)c * N + (s - 1)] * sd.G[c];
            double f = p - ev[s - 1] * gk;
            if (mode == CM_RHS) {
              out[s - 1] = f;
            } else if (mode == CM_H1) {
              sd.k1[s - 1] = f;
              val = state[s - 1] + dt * f;
              sd.ntil[s - 1] = val;
            } else {
              val = state[s - 1] + 0.5 * dt * (sd.k1[s - 1] + f);
              state[s - 1] = val;
            }
          }
          if (e == 0) s0[it] = val; else s1[it] = val;
        }
      }
    }
    __syncthreads();
  } else {
#pragma unroll
    for (int it = 0; it < IPT; ++it) {
      int idx = tid + it * kThreads;
      s0[it] = 0.0;
      s1[it] = 0.0;
      if (idx < nitems) {
        int j1 = idx / g, jl = idx - j1 * g;
        int64_t j = j2_0 + jl + (int64_t)M2 * j1;
        if (2 * j >= 1 && 2 * j <= N) s0[it] = state[2 * j - 1];
        if (2 * j + 1 <= N) s1[it] = state[2 * j];
      }
    }
  }

  if (!mode_has_forward(mode)) return;
  cplx<T>* Z1 = (cplx<T>*)sd.Z1;
  for (int c = 0; c < sd.u; ++c) {
    const double* col = sd.cols + (size_t)c * N;
    double dsum = 0.0;
#pragma unroll
    for (int it = 0; it < IPT; ++it) {
      int idx = tid + it * kThreads;
      if (idx < nitems) {
        int j1 = idx / g, jl = idx - j1 * g;
        int64_t j = j2_0 + jl + (int64_t)M2 * j1;
        double x0 = (2 * j >= 1 && 2 * j <= N) ? col[2 * j - 1] * s0[it] : 0.0;
        double x1 = (2 * j + 1 <= N) ? col[2 * j] * s1[it] : 0.0;
        buf[jl * STR + j1] = cplx<T>{Real<T>::from_d(x0), Real<T>::from_d(x1)};
        dsum += x0 + x1;
      }
    }
    __syncthreads();
    fft_batch<T, M1, -1, GMAX, STR>(buf, g, twP1);
#pragma unroll
    for (int it = 0; it < IPT; ++it) {
      int idx = tid + it * kThreads;
      if (idx < nitems) {
        int k1 = idx / g, jl = idx - k1 * g;
        int j2 = j2_0 + jl;
        int64_t e = (2 * (int64_t)j2 * k1) & (a.L - 1);
        Z1[(size_t)c * M + (int64_t)k1 * M2 + j2] = cmul(buf[jl * STR + k1], twL<T>(a, e));
      }
    }
    red[tid] = dsum;
    __syncthreads();
    for (int w = kThreads / 2; w > 0; w >>= 1) {
      if (tid < w) red[tid] += red[tid + w];
      __syncthreads();
    }
    if (tid == 0) sd.dots[(size_t)c * ngroups + grp] = red[0];
  }
}

// ---------------------------------------------------------------------------
// Row pass.  Work item = (slot, k1 in [0, M1/2]) covering rows k1 and M1-k1.
// ---------------------------------------------------------------------------
template <class T, int M2>
__global__ __launch_bounds__(kThreads) void row_kernel(LaunchArgs a) {
  constexpr int NB = (2048 / M2) > 0 ? 2048 / M2 : 1;
  constexpr int STR = M2;
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ double red[kThreads];

  const int M1 = a.M1;
  const int nwork = M1 / 2 + 1;
  const int slot = blockIdx.x / nwork;
  const int k1 = blockIdx.x - slot * nwork;
  const SlotDesc sd = a.slots[slot];
  const int row_on = a.mode >= 0 ? 1 : sd.row_on;
  if (!row_on) return;
  const int u = sd.u;
  const int64_t M = (int64_t)M1 * M2;
  const int tid = threadIdx.x;
  cplx<T>* X = (cplx<T>*)smem;                         // u * nrows rows
  cplx<T>* nyq = X + (size_t)a.umax * 2 * STR;         // u Nyquist values (bin k = M)
  double* sdot = (double*)(nyq + a.umax);              // u dot products

  // loss-term weights of this evaluation, from the column pass's partial dots
  if (k1 == 0) {
    const int ngroups = M2 / a.g;
    for (int c = 0; c < u; ++c) {
      double s = 0.0;
      for (int q = tid; q < ngroups; q += kThreads) s += sd.dots[(size_t)c * ngroups + q];
      red[tid] = s;
      __syncthreads();
      for (int w = kThreads / 2; w > 0; w >>= 1) {
        if (tid < w) red[tid] += red[tid + w];
        __syncthreads();
      }
      if (tid == 0) sdot[c] = red[0];
      __syncthreads();
    }
    if (tid == 0) {
      for (int c = 0; c < u; ++c) sd.G[c] = 0.0;
      for (int t = 0; t < sd.Tq; ++t) {
        double pr = sd.q_coef[t];
        for (int o = sd.q_off[t]; o < sd.q_off[t + 1]; ++o) pr *= sdot[sd.q_ids[o]];
        sd.G[sd.q_kmode[t]] += pr;
      }
    }
  }

  const int nrows = (k1 == 0 || 2 * k1 == M1) ? 1 : 2;
  const int rows[2] = {k1, M1 - k1};
  const cplx<T>* Z1 = (const cplx<T>*)sd.Z1;
  const int nload = u * nrows * M2;
  for (int idx = tid; idx < nload; idx += kThreads) {
    int cr = idx / M2, k2 = idx - cr * M2;
    int c = cr / nrows, rr = cr - c * nrows;
    X[cr * STR + k2] = Z1[(size_t)c * M + (int64_t)rows[rr] * M2 + k2];
  }
  __syncthreads();
  fft_batch<T, M2, -1, NB, STR>(X, u * nrows, (const cplx<T>*)a.twP2);

  // bins k = k1 + M1*iA and M - k, spectra of the real inputs, their weighted
  // products, and the even/odd packing of the real inverse
  const int nunits = (k1 == 0) ? M2 / 2 + 1 : (nrows == 1 ? M2 / 2 : M2);
  for (int unit = tid; unit < nunits; unit += kThreads) {
    const int iA = unit;
    int iB, rB;
    if (k1 == 0) { iB = (M2 - iA) & (M2 - 1); rB = 0; }
    else if (nrows == 1) { iB = M2 - 1 - iA; rB = 0; }
    else { iB = M2 - 1 - iA; rB = 1; }
    const bool zero_bin = (k1 == 0 && iA == 0);
    const bool self = (rB == 0 && iB == iA);
    const int64_t kA = k1 + (int64_t)M1 * iA;
    const cplx<T> wk = twL<T>(a, kA);
    for (int c = 0; c < u; ++c) {
      cplx<T>* pA = &X[(c * nrows) * STR + iA];
      cplx<T>* pB = &X[(c * nrows + rB) * STR + iB];
      cplx<T> ZA = *pA, ZB = *pB;
      if (zero_bin) {
        *pA = cplx<T>{ZA.re + ZA.im, Real<T>::zero()};
        nyq[c] = cplx<T>{ZA.re - ZA.im, Real<T>::zero()};
      } else {
        cplx<T> zc = cconj(ZB);
        cplx<T> E = cplx<T>{half_of(ZA.re + zc.re), half_of(ZA.im + zc.im)};
        cplx<T> dd = csub(ZA, zc);
        cplx<T> O = cplx<T>{half_of(dd.im), half_of(-dd.re)};   // -i*(ZA - conj ZB)/2
        cplx<T> t = cmul(wk, O);
        *pA = cadd(E, t);
        if (!self) *pB = cconj(csub(E, t));
      }
    }
    cplx<T> YA = czero<T>(), YB = czero<T>();
    for (int t = 0; t < sd.Tp; ++t) {
      T cf = Real<T>::from_d(sd.p_coef[t]);
      cplx<T> PA = cplx<T>{cf, Real<T>::zero()}, PB = PA;
      for (int o = sd.p_off[t]; o < sd.p_off[t + 1]; ++o) {
        int c = sd.p_ids[o];
        PA = cmul(PA, X[(c * nrows) * STR + iA]);
        PB = cmul(PB, zero_bin ? nyq[c] : X[(c * nrows + rB) * STR + iB]);
      }
      YA = cadd(YA, PA);
      YB = cadd(YB, PB);
    }
    if (zero_bin) {
      X[0] = cplx<T>{YA.re + YB.re, YA.re - YB.re};
    } else {
      cplx<T> F = cadd(YA, cconj(YB));
      cplx<T> Gd = csub(YA, cconj(YB));
      X[iA] = cadd(F, cmul_i(cmulc(Gd, wk)));
      if (!self) X[rB * STR + iB] = cadd(cconj(F), cmul_i(cmul(wk, cconj(Gd))));
    }
  }
  __syncthreads();
  fft_batch<T, M2, +1, NB, STR>(X, nrows, (const cplx<T>*)a.twP2);

  cplx<T>* V = (cplx<T>*)sd.V;
  for (int idx = tid; idx < nrows * M2; idx += kThreads) {
    int rr = idx / M2, j2 = idx - rr * M2;
    int64_t row = rows[rr];
    int64_t e = (2 * (int64_t)j2 * row) & (a.L - 1);
    V[row * M2 + j2] = cmulc(X[rr * STR + j2], twL<T>(a, e));
  }
}

// ---------------------------------------------------------------------------
// Moments M0 = sum n, M1 = sum k n, and a non-finite count (binary64).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kThreads) void moments_kernel(const double* n, int64_t total, int64_t N,
                                                          double* part) {
  __shared__ double r0[kThreads], r1[kThreads], r2[kThreads];
  double a0 = 0, a1 = 0, a2 = 0;
  for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < total;
       i += (int64_t)gridDim.x * kThreads) {
    double v = n[i];
    if (!isfinite(v)) { a2 += 1.0; continue; }
    a0 += v;
    a1 += (double)(i % N + 1) * v;
  }
  int tid = threadIdx.x;
  r0[tid] = a0; r1[tid] = a1; r2[tid] = a2;
  __syncthreads();
  for (int w = kThreads / 2; w > 0; w >>= 1) {
    if (tid < w) { r0[tid] += r0[tid + w]; r1[tid] += r1[tid + w]; r2[tid] += r2[tid + w]; }
    __syncthreads();
  }
  if (tid == 0) {
    part[3 * blockIdx.x] = r0[0];
    part[3 * blockIdx.x + 1] = r1[0];
    part[3 * blockIdx.x + 2] = r2[0];
  }
}

// ---------------------------------------------------------------------------
// Host launchers
// ---------------------------------------------------------------------------
template <class T, int M1>
static hipError_t launch_col_t(const LaunchArgs& a, hipStream_t s) {
  dim3 grid(a.nslots * (a.M2 / a.g));
  hipLaunchKernelGGL((col_kernel<T, M1>), grid, dim3(kThreads), 0, s, a);
  return hipGetLastError();
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
  }
  return hipErrorInvalidValue;
}

size_t row_smem_bytes(int prec, int umax, int M2) {
  size_t cs = prec == 1 ? 8 : 16;
  return (size_t)umax * 2 * M2 * cs + (size_t)umax * cs + (size_t)umax * 8;
}

template <class T, int M2>
static hipError_t launch_row_t(const LaunchArgs& a, hipStream_t s, size_t smem) {
  static bool attr_done = false;   // raise the dynamic LDS cap once per instantiation
  if (!attr_done) {
    hipError_t e = hipFuncSetAttribute((const void*)row_kernel<T, M2>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024 - 4096);
    if (e != hipSuccess) return e;
    attr_done = true;
  }
  dim3 grid(a.nslots * (a.M1 / 2 + 1));
  hipLaunchKernelGGL((row_kernel<T, M2>), grid, dim3(kThreads), smem, s, a);
  return hipGetLastError();
}

template <class T>
static hipError_t launch_row_p(const LaunchArgs& a, hipStream_t s, size_t smem) {
  switch (a.M2) {
    case 2: return launch_row_t<T, 2>(a, s, smem);
    case 4: return launch_row_t<T, 4>(a, s, smem);
    case 8: return launch_row_t<T, 8>(a, s, smem);
    case 16: return launch_row_t<T, 16>(a, s, smem);
    case 32: return launch_row_t<T, 32>(a, s, smem);
    case 64: return launch_row_t<T, 64>(a, s, smem);
    case 128: return launch_row_t<T, 128>(a, s, smem);
    case 256: return launch_row_t<T, 256>(a, s, smem);
    case 512: return launch_row_t<T, 512>(a, s, smem);
    case 1024: return launch_row_t<T, 1024>(a, s, smem);
    case 2048: return launch_row_t<T, 2048>(a, s, smem);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_col(int prec, const LaunchArgs& a, hipStream_t s) {
  if (prec == 0) return launch_col_p<double>(a, s);
  if (prec == 1) return launch_col_p<float>(a, s);
  return launch_col_p<ff>(a, s);
}

hipError_t launch_row(int prec, const LaunchArgs& a, hipStream_t s) {
  size_t smem = row_smem_bytes(prec, a.umax, a.M2);
  if (prec == 0) return launch_row_p<double>(a, s, smem);
  if (prec == 1) return launch_row_p<float>(a, s, smem);
  return launch_row_p<ff>(a, s, smem);
}

hipError_t launch_moments(const double* n, int64_t total, int64_t N, double* part, int nblocks,
                          hipStream_t s) {
  hipLaunchKernelGGL(moments_kernel, dim3(nblocks), dim3(kThreads), 0, s, n, total, N, part);
  return hipGetLastError();
}

}  // namespace agg
