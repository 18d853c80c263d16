// Device kernels of the AIMx matvec and of the batched Krylov solver, for
// gfx950 (CDNA4: 64-lane wavefronts, 160 KB LDS per CU).
//
// Matvec (eq. LAIMx): y = P^T IFFT( H_hat * FFT( pad(P x) ) ) + C x
//   project        q = P x with P assembled at set-up and sorted by grid node;
//                  each thread owns one node and sums its row in a fixed
//                  order (reproducible, no atomics);
//   fft_row/col    register-resident Stockham passes (radix 8 or 16 with
//                  one smaller stage, exchanges through LDS), pruned: forward passes read only the non-zero half
//                  of each padded line, inverse passes write only the half that
//                  is kept; column passes move whole 128-byte row segments so
//                  the strided y/z lines are read and written coalesced;
//                  the z pass multiplies by the kernel spectrum between its
//                  forward and inverse transforms without leaving LDS;
//   interp_near    rows of P^T (stencil potentials of each triangle) plus the
//                  rows of the real CSR near-field correction, one pass over y.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <mutex>
#include <vector>

#include "aim_internal.h"

namespace aim {

// ---------------------------------------------------------------------------
// complex helpers
// ---------------------------------------------------------------------------
template <typename T>
struct CxT;
template <>
struct CxT<double> {
  using t = double2;
};
template <>
struct CxT<float> {
  using t = float2;
};
template <typename T>
using cx = typename CxT<T>::t;

template <typename T>
__device__ __forceinline__ cx<T> mkc(T re, T im) {
  cx<T> r;
  r.x = re;
  r.y = im;
  return r;
}
template <typename C>
__device__ __forceinline__ C cadd(C a, C b) {
  C r;
  r.x = a.x + b.x;
  r.y = a.y + b.y;
  return r;
}
template <typename C>
__device__ __forceinline__ C csub(C a, C b) {
  C r;
  r.x = a.x - b.x;
  r.y = a.y - b.y;
  return r;
}
template <typename C>
__device__ __forceinline__ C cmul(C a, C b) {
  C r;
  r.x = a.x * b.x - a.y * b.y;
  r.y = a.x * b.y + a.y * b.x;
  return r;
}
template <typename C, typename S>
__device__ __forceinline__ C cscale(C a, S s) {
  C r;
  r.x = a.x * s;
  r.y = a.y * s;
  return r;
}

constexpr int ilog2(int v) { return v <= 1 ? 0 : 1 + ilog2(v / 2); }

// ---------------------------------------------------------------------------
// radix-R DFTs on registers (forward sign e^{-2 pi i/R}; INV uses e^{+})
// ---------------------------------------------------------------------------
template <typename T, bool INV>
__device__ __forceinline__ cx<T> rot90(cx<T> a) {  // * (-i) forward, * (+i) inverse
  return INV ? mkc<T>(-a.y, a.x) : mkc<T>(a.y, -a.x);
}

// HALF_IN: the upper half of the inputs (v[R/2] .. v[R-1]) is zero and is
// not read, which drops the butterflies that would only add zeros (the first
// forward stage of a zero-padded line).
template <typename T, int R, bool INV, bool HALF_IN = false>
struct Dft;

template <typename T, bool INV, bool HALF_IN>
struct Dft<T, 2, INV, HALF_IN> {
  static __device__ __forceinline__ void run(cx<T>* v) {
    const cx<T> a = v[0];
    if constexpr (HALF_IN) {
      v[1] = a;
    } else {
      v[0] = cadd(a, v[1]);
      v[1] = csub(a, v[1]);
    }
  }
};

template <typename T, bool INV, bool HALF_IN>
struct Dft<T, 4, INV, HALF_IN> {
  static __device__ __forceinline__ void run(cx<T>* v) {
    if constexpr (HALF_IN) {
      const cx<T> a0 = v[0], a1 = v[1], r = rot90<T, INV>(a1);
      v[0] = cadd(a0, a1);
      v[2] = csub(a0, a1);
      v[1] = cadd(a0, r);
      v[3] = csub(a0, r);
    } else {
      const cx<T> t0 = cadd(v[0], v[2]), t1 = csub(v[0], v[2]);
      const cx<T> t2 = cadd(v[1], v[3]), t3 = rot90<T, INV>(csub(v[1], v[3]));
      v[0] = cadd(t0, t2);
      v[2] = csub(t0, t2);
      v[1] = cadd(t1, t3);
      v[3] = csub(t1, t3);
    }
  }
};

template <typename T, bool INV, bool HALF_IN>
struct Dft<T, 8, INV, HALF_IN> {
  static __device__ __forceinline__ void run(cx<T>* v) {
    // even and odd inputs; with HALF_IN only their first two are non-zero
    cx<T> e[4] = {v[0], v[2], v[4], v[6]};
    cx<T> o[4] = {v[1], v[3], v[5], v[7]};
    Dft<T, 4, INV, HALF_IN>::run(e);
    Dft<T, 4, INV, HALF_IN>::run(o);
    const T r2 = T(0.70710678118654752440);
    // o1 *= w8, o2 *= w8^2, o3 *= w8^3 with w8 = e^{-/+ i pi/4}
    const cx<T> a = o[1], c = o[3];
    if (INV) {
      o[1] = mkc<T>((a.x - a.y) * r2, (a.x + a.y) * r2);
      o[3] = mkc<T>(-(c.x + c.y) * r2, (c.x - c.y) * r2);
    } else {
      o[1] = mkc<T>((a.x + a.y) * r2, (a.y - a.x) * r2);
      o[3] = mkc<T>((c.y - c.x) * r2, -(c.x + c.y) * r2);
    }
    o[2] = rot90<T, INV>(o[2]);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      v[k] = cadd(e[k], o[k]);
      v[k + 4] = csub(e[k], o[k]);
    }
  }
};

// 16 points as 4 x 4: n = 4 n1 + n2, k = k1 + 4 k2; 4-point DFTs over n1,
// twiddles W16^(n2 k1), 4-point DFTs over n2
template <typename T, bool INV, bool HALF_IN>
struct Dft<T, 16, INV, HALF_IN> {
  static __device__ __forceinline__ cx<T> tw(cx<T> a, T c, T sf) {  // a * (c + i sf), sf forward
    return cmul(a, mkc<T>(c, INV ? -sf : sf));
  }
  static __device__ __forceinline__ void run(cx<T>* v) {
    const T c1 = T(0.92387953251128675613), s1 = T(0.38268343236508977173);
    const T r2 = T(0.70710678118654752440);
    cx<T> a[4][4];
#pragma unroll
    for (int n2 = 0; n2 < 4; ++n2) {
      cx<T> u[4] = {v[n2], v[4 + n2], v[8 + n2], v[12 + n2]};
      Dft<T, 4, INV, HALF_IN>::run(u);  // inputs n < 8: n1 < 2
#pragma unroll
      for (int k1 = 0; k1 < 4; ++k1) a[n2][k1] = u[k1];
    }
    a[1][1] = tw(a[1][1], c1, -s1);   // W^1
    a[1][2] = tw(a[1][2], r2, -r2);   // W^2
    a[1][3] = tw(a[1][3], s1, -c1);   // W^3
    a[2][1] = tw(a[2][1], r2, -r2);   // W^2
    a[2][2] = rot90<T, INV>(a[2][2]); // W^4
    a[2][3] = tw(a[2][3], -r2, -r2);  // W^6
    a[3][1] = tw(a[3][1], s1, -c1);   // W^3
    a[3][2] = tw(a[3][2], -r2, -r2);  // W^6
    a[3][3] = tw(a[3][3], -c1, s1);   // W^9
#pragma unroll
    for (int k1 = 0; k1 < 4; ++k1) {
      cx<T> u[4] = {a[0][k1], a[1][k1], a[2][k1], a[3][k1]};
      Dft<T, 4, INV>::run(u);
#pragma unroll
      for (int k2 = 0; k2 < 4; ++k2) v[k1 + 4 * k2] = u[k2];
    }
  }
};

// 32 points as 4 x 8: n = 8 n1 + n2, k = k1 + 4 k2; 4-point DFTs over n1,
// twiddles W32^(n2 k1), 8-point DFTs over n2
constexpr double kCos32[8] = {1.0, 0.9807852804032304, 0.9238795325112867, 0.8314696123025452,
                              0.7071067811865476, 0.5555702330196023, 0.38268343236508984,
                              0.19509032201612833};  // cos(2 pi r / 32)
constexpr double kSin32[8] = {0.0, 0.19509032201612825, 0.3826834323650898, 0.5555702330196022,
                              0.7071067811865475, 0.8314696123025452, 0.9238795325112867,
                              0.9807852804032304};   // sin(2 pi r / 32)
template <typename T, bool INV, bool HALF_IN>
struct Dft<T, 32, INV, HALF_IN> {
  // a * W32^m (e^{-2 pi i m / 32} forward): the first-octant twiddle of
  // m mod 8, then a quarter turn for each 8 in m
  static __device__ __forceinline__ cx<T> w(cx<T> a, int m) {
    const int r = m % 8, q = m / 8;
    if (r != 0) a = cmul(a, mkc<T>(T(kCos32[r]), INV ? T(kSin32[r]) : -T(kSin32[r])));
    for (int i = 0; i < q; ++i) a = rot90<T, INV>(a);
    return a;
  }
  static __device__ __forceinline__ void run(cx<T>* v) {
    cx<T> a[8][4];
#pragma unroll
    for (int n2 = 0; n2 < 8; ++n2) {
      cx<T> u[4] = {v[n2], v[8 + n2], v[16 + n2], v[24 + n2]};
      Dft<T, 4, INV, HALF_IN>::run(u);  // inputs n < 16: n1 < 2
#pragma unroll
      for (int k1 = 0; k1 < 4; ++k1) a[n2][k1] = w(u[k1], n2 * k1);
    }
#pragma unroll
    for (int k1 = 0; k1 < 4; ++k1) {
      cx<T> u[8];
#pragma unroll
      for (int n2 = 0; n2 < 8; ++n2) u[n2] = a[n2][k1];
      Dft<T, 8, INV>::run(u);
#pragma unroll
      for (int k2 = 0; k2 < 8; ++k2) v[k1 + 4 * k2] = u[k2];
    }
  }
};

// ---------------------------------------------------------------------------
// Register-resident Stockham FFT.  A length-L line is shared by NT threads;
// each holds E = L/NT elements in registers.  Stage s with radix R treats
// butterfly j (= t + i NT) as elements j + r L/R, twiddles them by
// W_{Ns R}^{r (j mod Ns)}, runs the R-point DFT and leaves element
// (j div Ns) Ns R + (j mod Ns) + r Ns, with Ns the product of the earlier
// radices.  Elements move through LDS only between stages; the first stage
// reads straight from memory (skipping the zero padding) and the last writes
// straight to memory (skipping the discarded half).  Forward passes put the
// small radix (2 or 4) first and inverse passes last, so a forward transform
// ends, and an inverse one starts, with radix 8 and the same element
// ownership: the spectral multiply between them needs no exchange.
// ---------------------------------------------------------------------------
template <int L, bool SMALL_FIRST, int RMAX>
struct Sched {
  static constexpr int P = ilog2(L);
  static constexpr int Q = ilog2(RMAX);                 // bits per full stage (3 or 4)
  static constexpr int REM = P % Q;
  static constexpr int SMALL = 1 << REM;               // the one smaller radix, if any
  static constexpr int NST = P / Q + (REM ? 1 : 0);
  static constexpr int radix(int st) {
    return REM == 0 ? RMAX : (SMALL_FIRST ? (st == 0 ? SMALL : RMAX)
                                          : (st == NST - 1 ? SMALL : RMAX));
  }
  static constexpr int lgns(int st) {
    int a = 0;
    for (int q = 0; q < st; ++q) a += ilog2(radix(q));
    return a;
  }
};

template <typename T, int L, int NT, bool INV, int R, int LGNS, bool HALF_IN = false>
__device__ __forceinline__ void stage_compute(cx<T>* v, int t, const cx<T>* tw) {
  constexpr int NB = L / (R * NT);
  static_assert(NB >= 1, "too many threads per line for this radix");
  constexpr int twsh = ilog2(L) - LGNS - ilog2(R);  // log2(L / (Ns R))
#pragma unroll
  for (int i = 0; i < NB; ++i) {
    if constexpr (LGNS > 0) {
      const int k = (t + i * NT) & ((1 << LGNS) - 1);
#pragma unroll
      for (int r = 1; r < R; ++r) {
        cx<T> w = tw[(r * k) << twsh];
        if (INV) w.y = -w.y;
        v[i * R + r] = cmul(v[i * R + r], w);
      }
    }
    Dft<T, R, INV, HALF_IN>::run(v + i * R);
  }
}

template <typename T, int L, int NT, int R, int LGNS, int R2>
__device__ __forceinline__ void exchange(cx<T>* v, cx<T>* s, int es, int t) {
  constexpr int NB = L / (R * NT), NB2 = L / (R2 * NT);
  constexpr int lgR = ilog2(R), Ns = 1 << LGNS;
#pragma unroll
  for (int i = 0; i < NB; ++i) {
    const int j = t + i * NT;
    const int d = ((j >> LGNS) << (LGNS + lgR)) + (j & (Ns - 1));
#pragma unroll
    for (int r = 0; r < R; ++r) s[(d + r * Ns) * es] = v[i * R + r];
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < NB2; ++i) {
    const int j = t + i * NT;
#pragma unroll
    for (int r = 0; r < R2; ++r) v[i * R2 + r] = s[(j + r * (L / R2)) * es];
  }
  __syncthreads();
}

// HALF_IN: the second half of the line is zero (a zero-padded forward
// transform); only the first stage sees that
template <typename T, int L, int NT, bool INV, bool SF, int RMAX, int ST, bool HALF_IN = false>
__device__ __forceinline__ void run_stages(cx<T>* v, cx<T>* s, int es, int t, const cx<T>* tw) {
  using Sc = Sched<L, SF, RMAX>;
  constexpr int R = Sc::radix(ST), LG = Sc::lgns(ST);
  stage_compute<T, L, NT, INV, R, LG, HALF_IN && ST == 0>(v, t, tw);
  if constexpr (ST + 1 < Sc::NST) {
    exchange<T, L, NT, R, LG, Sc::radix(ST + 1)>(v, s, es, t);
    run_stages<T, L, NT, INV, SF, RMAX, ST + 1>(v, s, es, t, tw);
  }
}

// ---------------------------------------------------------------------------
// FFT pass kernel.  Lines are addressed as (line >> lg_nli) * os + e * es +
// (line & (2^lg_nli - 1)) * p0: column passes (y, z) have lg_nli = log2(Mx)
// and p0 = 1 so that consecutive lines are consecutive x positions (coalesced
// rows of TL elements); row passes (x) have lg_nli = log2(rows per plane),
// p0 = row pitch, os = plane pitch and es = 1.
// MODE 0: forward, 1: inverse, 2: forward * spectrum then inverse, 3: the x
// forward pass with its input lines computed as the projection q = P x.
//
// MODE 3: a workgroup's TL lines are TL * (L/2) consecutive grid nodes, i.e.
// consecutive rows of P sorted by node, so their entries form one contiguous
// range.  The range is streamed in chunks through the LDS line buffer as the
// products w x[col] (coalesced entry loads, the x gathers of 256 or more
// threads in flight together), and every thread sums, in entry order, the
// rows of the elements it then transforms: the projected values never go
// to memory, and the result does not depend on the chunking.
// HALF (the convolution's passes): a forward transform reads only the first
// half of its line (the rest is the zero padding, known at compile time, so
// the first stage skips it) and an inverse transform keeps only the first
// half; otherwise (the kernel spectrum) whole lines, Lin and Lout elements.
// ---------------------------------------------------------------------------
struct PassArgs {
  int64_t nlines;
  int lg_nli;
  int64_t in_es, in_os, out_es, out_os;
  int64_t in_p0, out_p0;  // stride of the inner line index (1 for column passes)
  int64_t in_bs, out_bs;  // per right-hand-side strides
  int Lin, Lout;          // leading elements read / written per line
  // spectral multiply (fused z pass): line (li, lo) = (kx, ky), element = kz
  const void* spec;
  int64_t spec_fs;        // per-frequency stride of the folded spectrum
  const int32_t* rhs_freq;
  int Mx, Nx, My, Ny, Mz, Nz;
  // projection fused into the x forward pass (MODE 3): P by grid node and
  // the mesh vector x ([nrhs][px_bs])
  const int32_t* prow;
  const int32_t* pcol;
  const void* pval;
  const void* px;
  int64_t px_bs;
  // the double layer's cross-product z pass: stride between the three
  // channels' grids, and between the three folded gradient spectra
  int64_t ch_bs;
  int64_t spec_cs;
};

template <typename T, int L, int TL, int NT, int MODE, bool COL, int RMAX, bool HALF>
__global__ __launch_bounds__(TL* NT) void fft_pass_kernel(const cx<T>* in, cx<T>* out,
                                                          const cx<T>* __restrict__ twg,
                                                          PassArgs a) {
  constexpr int E = L / NT;
  constexpr int NTH = TL * NT;
  __shared__ cx<T> s[COL ? L * TL : TL * (L + 1)];
  __shared__ cx<T> tw[L];
  __shared__ int32_t rp[MODE == 3 ? TL * (L / 2) + 1 : 1];
  const int tid = threadIdx.x;
  const int rhs = blockIdx.y;
  if constexpr (MODE != 3) in += rhs * a.in_bs;
  out += rhs * a.out_bs;
  const int l = COL ? (tid & (TL - 1)) : (tid / NT);
  const int t = COL ? (tid / TL) : (tid & (NT - 1));
  int64_t line0 = int64_t(blockIdx.x) * TL;
  if constexpr (MODE == 2) {
    // XCD-aware order: workgroups are dealt round-robin to the 8 XCDs, so
    // hardware block b runs on XCD b % 8.  Give each XCD a contiguous run of
    // logical blocks, and order rows as 0, 1, My-1, 2, My-2, ..., My/2: the
    // rows ky and My-ky (and, within a row, kx and Mx-kx) read the same folded
    // spectrum plane, which then stays in that XCD's L2.
    if (a.Mx >= TL) {                                // a block stays within one row
      const int nbx = a.Mx / TL;                     // both powers of two
      const int nb = nbx * a.My;
      const int b = int(blockIdx.x);
      const int lb = (nb % 8 == 0) ? (b % 8) * (nb / 8) + b / 8 : b;
      const int rowpos = lb / nbx, g = lb % nbx;
      const int h = a.My / 2;
      const int ky = rowpos == 0 ? 0
                   : rowpos == a.My - 1 ? h
                   : (rowpos & 1) ? (rowpos + 1) / 2 : a.My - rowpos / 2;
      line0 = int64_t(ky) * a.Mx + int64_t(g) * TL;
    }
  }
  const int64_t line = line0 + l;
  const bool valid = line < a.nlines;
  const int64_t mask = (int64_t(1) << a.lg_nli) - 1;
  const int64_t li = line & mask, lo = line >> a.lg_nli;
  const cx<T>* src = MODE == 3 ? nullptr : in + lo * a.in_os + li * a.in_p0;
  cx<T>* dst = out + lo * a.out_os + li * a.out_p0;
  cx<T>* sl = COL ? s + l : s + l * (L + 1);
  const int es = COL ? TL : 1;

  constexpr bool FWD = MODE == 0 || MODE == 3;
  constexpr bool SF = MODE != 1;
  constexpr bool HALF_IN = HALF && MODE != 1, HALF_OUT = HALF && !FWD;
  static_assert(RMAX <= E, "a thread must hold a whole butterfly");
  static_assert(MODE != 3 || (!COL && HALF), "the fused projection feeds the x forward pass");
  using S0 = Sched<L, SF, RMAX>;
  constexpr int R0 = S0::radix(0), NB0 = L / (R0 * NT);
  cx<T> v[E];
  if constexpr (MODE == 3) {
    constexpr int NX = L / 2;
    const int64_t u0 = line0 * NX, ng = a.nlines * NX;
    for (int i = tid; i <= TL * NX; i += NTH)
      rp[i] = a.prow[u0 + i < ng ? u0 + i : ng];
#pragma unroll
    for (int k = 0; k < E; ++k) v[k] = mkc<T>(T(0), T(0));
    __syncthreads();
    const T* pv = static_cast<const T*>(a.pval);
    const cx<T>* xr = static_cast<const cx<T>*>(a.px) + rhs * a.px_bs;
    const int32_t k0 = rp[0], k1 = rp[TL * NX];
    constexpr int CH = TL * (L + 1);
    for (int32_t cb = k0; cb < k1; cb += CH) {
      const int32_t ce = k1 - cb < CH ? k1 : cb + CH;
      for (int32_t k = cb + tid; k < ce; k += NTH) {
        const T w = pv[k];
        const cx<T> xv = xr[a.pcol[k]];
        s[k - cb] = mkc<T>(w * xv.x, w * xv.y);
      }
      __syncthreads();
#pragma unroll
      for (int i = 0; i < NB0; ++i)
#pragma unroll
        for (int r = 0; r < R0 / 2; ++r) {  // the nonzero half: e < L/2
          const int lr = l * NX + t + i * NT + r * (L / R0);
          const int32_t b0 = rp[lr] > cb ? rp[lr] : cb, b1 = rp[lr + 1] < ce ? rp[lr + 1] : ce;
          // four independent partial sums (four LDS reads in flight), then
          // combined in a fixed order
          T ax[4] = {T(0), T(0), T(0), T(0)}, ay[4] = {T(0), T(0), T(0), T(0)};
          int32_t k = b0;
          for (; k + 4 <= b1; k += 4)
#pragma unroll
            for (int j = 0; j < 4; ++j) {
              ax[j] += s[k + j - cb].x;
              ay[j] += s[k + j - cb].y;
            }
          for (int j = 0; k < b1; ++k, ++j) {
            ax[j] += s[k - cb].x;
            ay[j] += s[k - cb].y;
          }
          cx<T> acc = v[i * R0 + r];
          acc.x += (ax[0] + ax[1]) + (ax[2] + ax[3]);
          acc.y += (ay[0] + ay[1]) + (ay[2] + ay[3]);
          v[i * R0 + r] = acc;
        }
      __syncthreads();
    }
  } else {
#pragma unroll
    for (int i = 0; i < NB0; ++i)
#pragma unroll
      for (int r = 0; r < R0; ++r) {
        const int e = t + i * NT + r * (L / R0);
        if constexpr (HALF_IN)  // e < L/2 exactly when r < R0/2
          v[i * R0 + r] = (valid && r < R0 / 2) ? src[e * a.in_es] : mkc<T>(T(0), T(0));
        else
          v[i * R0 + r] = (valid && e < a.Lin) ? src[e * a.in_es] : mkc<T>(T(0), T(0));
      }
  }
  // fused z pass: the spectrum values this thread multiplies after its
  // forward transform depend only on (kx, ky) and the element index, so they
  // are loaded here, in flight together with the line itself
  using Fw = Sched<L, true, RMAX>;
  constexpr int RM = Fw::radix(Fw::NST - 1);
  constexpr int NSP = MODE == 2 ? E : 1;
  cx<T> spv[NSP];
  if constexpr (MODE == 2) {
    static_assert(RM == Sched<L, false, RMAX>::radix(0),
                  "the forward transform must end with the radix the inverse starts with");
    if (valid) {
      const int kx = int(li), ky = int(lo);
      const int fx = kx <= a.Nx ? kx : a.Mx - kx;
      const int fy = ky <= a.Ny ? ky : a.My - ky;
      // folded spectrum layout [fy][fz][fx]: one contiguous plane per fy
      const cx<T>* sp = static_cast<const cx<T>*>(a.spec) + int64_t(a.rhs_freq[rhs]) * a.spec_fs +
                        int64_t(fy) * (a.Nz + 1) * (a.Nx + 1) + fx;
      const int64_t zst = int64_t(a.Nx + 1);
#pragma unroll
      for (int i = 0; i < L / (RM * NT); ++i)
#pragma unroll
        for (int r = 0; r < RM; ++r) {
          const int e = t + i * NT + r * (L / RM);
          const int fz = e <= a.Nz ? e : a.Mz - e;
          spv[i * RM + r] = sp[fz * zst];
        }
    }
  }
  // the twiddle table after the line and spectrum loads, so that their
  // latencies overlap
  for (int m = tid; m < L; m += NTH) tw[m] = twg[m];
  __syncthreads();
  run_stages<T, L, NT, MODE == 1, SF, RMAX, 0, HALF_IN>(v, sl, es, t, tw);
  if constexpr (MODE == 2) {
    if (valid) {
#pragma unroll
      for (int k = 0; k < E; ++k) v[k] = cmul(v[k], spv[k]);
    }
    run_stages<T, L, NT, true, false, RMAX, 0>(v, sl, es, t, tw);
  }
  using Sf = Sched<L, FWD, RMAX>;
  // outputs that the next pass streams (the forward passes and the y
  // inverse) are stored non-temporally, keeping them out of the way in the
  // caches; the in-place z pass and the x inverse, whose output the
  // interpolation gathers, store normally (measured both ways)
  constexpr bool kStreamOut = FWD || (MODE == 1 && COL);
  constexpr int Rf = Sf::radix(Sf::NST - 1), NBf = L / (Rf * NT);
  if (valid) {
#pragma unroll
    for (int i = 0; i < NBf; ++i)
#pragma unroll
      for (int r = 0; r < Rf; ++r) {
        const int e = t + i * NT + r * (L / Rf);
        if (HALF_OUT ? r < Rf / 2 : e < a.Lout) {  // e < L/2 exactly when r < Rf/2
          if constexpr (kStreamOut) {
            __builtin_nontemporal_store(v[i * Rf + r].x, &dst[e * a.out_es].x);
            __builtin_nontemporal_store(v[i * Rf + r].y, &dst[e * a.out_es].y);
          } else {
            dst[e * a.out_es] = v[i * Rf + r];
          }
        }
      }
  }
}

// ---------------------------------------------------------------------------
// z pass of the double-layer operators (Sec. III-B, eq. KAIMx) with the
// spectra K^_a of the three components of grad G (each odd along its own
// axis: the folded entry times -1 where the frequency along that axis lies
// above N).  A workgroup takes the z lines at TL positions (kx, ky) of all
// three channels, transforms them forward and forms
//   DOT false (RWG double layer): V^ = K^ x J^, three products;
//   DOT true (scalar double layer): -(K^ . q^), the channels q_a = n_a x
//   convolved with dG/dr'_a = -K_a and summed, one product,
// transforms the products back and writes the first Nz elements of each
// line into `out` (in place when out == in; the DOT product goes to channel
// 0).  The forward and inverse transforms, the element ownership and the
// XCD-aware order of the rows are those of the fused z pass
// (fft_pass_kernel, MODE 2).
// ---------------------------------------------------------------------------
template <typename T, int L, int TL, int NT, int RMAX, bool DOT>
__global__ __launch_bounds__(TL* NT) void zcross_kernel(const cx<T>* in, cx<T>* out,
                                                       const cx<T>* __restrict__ twg,
                                                       PassArgs a) {
  constexpr int NOUT = DOT ? 1 : 3;
  constexpr int E = L / NT;
  __shared__ cx<T> s[L * TL];
  __shared__ cx<T> tw[L];
  const int tid = threadIdx.x;
  const int rhs = blockIdx.y;
  in += rhs * a.in_bs;
  out += rhs * a.out_bs;
  const int l = tid & (TL - 1);
  const int t = tid / TL;
  int64_t line0 = int64_t(blockIdx.x) * TL;
  if (a.Mx >= TL) {  // the fused z pass's order: mirrored rows on one XCD
    const int nbx = a.Mx / TL;
    const int nb = nbx * a.My;
    const int b = int(blockIdx.x);
    const int lb = (nb % 8 == 0) ? (b % 8) * (nb / 8) + b / 8 : b;
    const int rowpos = lb / nbx, g = lb % nbx;
    const int h = a.My / 2;
    const int ky = rowpos == 0 ? 0
                 : rowpos == a.My - 1 ? h
                 : (rowpos & 1) ? (rowpos + 1) / 2 : a.My - rowpos / 2;
    line0 = int64_t(ky) * a.Mx + int64_t(g) * TL;
  }
  const int64_t line = line0 + l;
  const bool valid = line < a.nlines;
  const int64_t mask = (int64_t(1) << a.lg_nli) - 1;
  const int64_t li = line & mask, lo = line >> a.lg_nli;
  const cx<T>* src = in + lo * a.in_os + li * a.in_p0;
  cx<T>* dst = out + lo * a.out_os + li * a.out_p0;
  cx<T>* sl = s + l;
  using S0 = Sched<L, true, RMAX>;
  constexpr int R0 = S0::radix(0), NB0 = L / (R0 * NT);
  cx<T> v[3][E];
#pragma unroll
  for (int c = 0; c < 3; ++c)
#pragma unroll
    for (int i = 0; i < NB0; ++i)
#pragma unroll
      for (int r = 0; r < R0; ++r) {
        const int e = t + i * NT + r * (L / R0);
        v[c][i * R0 + r] = (valid && r < R0 / 2) ? src[c * a.ch_bs + e * a.in_es]
                                                 : mkc<T>(T(0), T(0));
      }
  using Fw = Sched<L, true, RMAX>;
  constexpr int RM = Fw::radix(Fw::NST - 1);
  static_assert(RM == Sched<L, false, RMAX>::radix(0),
                "the forward transform must end with the radix the inverse starts with");
  cx<T> kv[3][E];
  if (valid) {
    const int kx = int(li), ky = int(lo);
    const bool ox = kx > a.Nx, oy = ky > a.Ny;
    const int fx = ox ? a.Mx - kx : kx;
    const int fy = oy ? a.My - ky : ky;
    const cx<T>* sp = static_cast<const cx<T>*>(a.spec) + int64_t(a.rhs_freq[rhs]) * a.spec_fs +
                      int64_t(fy) * (a.Nz + 1) * (a.Nx + 1) + fx;
    const int64_t zst = int64_t(a.Nx + 1);
#pragma unroll
    for (int i = 0; i < L / (RM * NT); ++i)
#pragma unroll
      for (int r = 0; r < RM; ++r) {
        const int e = t + i * NT + r * (L / RM);
        const bool oz = e > a.Nz;
        const int64_t o = int64_t(oz ? a.Mz - e : e) * zst;
        cx<T> k0 = sp[o], k1 = sp[a.spec_cs + o], k2 = sp[2 * a.spec_cs + o];
        if (ox) k0 = mkc<T>(-k0.x, -k0.y);
        if (oy) k1 = mkc<T>(-k1.x, -k1.y);
        if (oz) k2 = mkc<T>(-k2.x, -k2.y);
        kv[0][i * RM + r] = k0;
        kv[1][i * RM + r] = k1;
        kv[2][i * RM + r] = k2;
      }
  }
  for (int m = tid; m < L; m += TL * NT) tw[m] = twg[m];
  __syncthreads();
#pragma unroll
  for (int c = 0; c < 3; ++c) run_stages<T, L, NT, false, true, RMAX, 0, true>(v[c], sl, TL, t, tw);
  if (valid && DOT) {
#pragma unroll
    for (int k = 0; k < E; ++k) {
      const cx<T> a0 = cmul(kv[0][k], v[0][k]), a1 = cmul(kv[1][k], v[1][k]),
                  a2 = cmul(kv[2][k], v[2][k]);
      v[0][k] = mkc<T>(-((a0.x + a1.x) + a2.x), -((a0.y + a1.y) + a2.y));
    }
  } else if (valid) {
#pragma unroll
    for (int k = 0; k < E; ++k) {
      const cx<T> jx = v[0][k], jy = v[1][k], jz = v[2][k];
      const cx<T> ax = cmul(kv[1][k], jz), bx = cmul(kv[2][k], jy);
      const cx<T> ay = cmul(kv[2][k], jx), by = cmul(kv[0][k], jz);
      const cx<T> az = cmul(kv[0][k], jy), bz = cmul(kv[1][k], jx);
      v[0][k] = mkc<T>(ax.x - bx.x, ax.y - bx.y);
      v[1][k] = mkc<T>(ay.x - by.x, ay.y - by.y);
      v[2][k] = mkc<T>(az.x - bz.x, az.y - bz.y);
    }
  }
#pragma unroll
  for (int c = 0; c < NOUT; ++c) run_stages<T, L, NT, true, false, RMAX, 0>(v[c], sl, TL, t, tw);
  using Sf = Sched<L, false, RMAX>;
  constexpr int Rf = Sf::radix(Sf::NST - 1), NBf = L / (Rf * NT);
  if (valid) {
#pragma unroll
    for (int c = 0; c < NOUT; ++c)
#pragma unroll
      for (int i = 0; i < NBf; ++i)
#pragma unroll
        for (int r = 0; r < Rf / 2; ++r) {  // the kept half: e < L/2
          const int e = t + i * NT + r * (L / Rf);
          dst[c * a.ch_bs + e * a.out_es] = v[c][i * Rf + r];
        }
  }
}

// ---------------------------------------------------------------------------
// launch shapes.  Each pass can run with one of kFftVariants (TL lines per
// block, NT threads per line) shapes; the autotuner picks one per pass.
// Column passes keep TL * sizeof(complex) >= 64 bytes so that each row of a
// block is one or two whole cache lines; row passes read whole lines.
// ---------------------------------------------------------------------------
constexpr int cmin(int a, int b) { return a < b ? a : b; }
constexpr int cmax(int a, int b) { return a > b ? a : b; }

template <typename T, int L, bool COL, int V>
struct Shape {
  static constexpr int kTL = sizeof(T) == 8 ? 8 : 16;  // 128-byte row segments
  // V 0-3: 8 elements per thread (radix-8 stages); V 4-5 and 7: 16 (radix 16;
  // V 7 with 512 threads, e.g. 16 lines of complex64 at L = 512, i.e.
  // 128-byte column rows); V 6: 32 (radix 32: one exchange for L = 512 =
  // 32 x 16)
  static constexpr int NT = V == 6 ? cmax(1, L / 32)
                          : V >= 4 ? cmax(1, L / 16)
                          : COL ? (V == 0 ? cmin(L / 8, 256 / kTL)
                                  : V == 1 ? cmin(L / 8, 512 / kTL)
                                  : V == 2 ? cmin(L / 8, 256 / (2 * kTL))
                                           : cmin(L / 8, 512 / (2 * kTL)))
                                : (V == 0 ? cmin(L / 8, 64)
                                  : V == 1 ? cmin(L / 8, 128)
                                  : V == 2 ? cmin(L / 8, 32)
                                           : cmin(L / 8, 64));
  static constexpr int TL = V == 6 ? cmax(1, 256 / NT)
                          : V >= 4 ? cmax(1, (V == 4 ? 256 : V == 5 ? 128 : 512) / NT)
                          : COL ? (V == 0 ? 256 / cmin(L / 8, 256 / kTL)
                                  : V == 1 ? 512 / cmin(L / 8, 512 / kTL)
                                  : V == 2 ? 256 / cmin(L / 8, 256 / (2 * kTL))
                                           : 512 / cmin(L / 8, 512 / (2 * kTL)))
                                : (V == 3 ? 512 / NT : cmax(1, 256 / NT));
  // radix-16 stages for the 16-element shapes: one exchange fewer per
  // transform for L = 128 and 256
  static constexpr int RMAX = V == 6 ? (L >= 32 ? 32 : 8) : V >= 4 && L >= 16 ? 16 : 8;
  static constexpr int THREADS = TL * NT;
  static constexpr size_t LDS = sizeof(cx<T>) * (COL ? size_t(L) * TL : size_t(TL) * (L + 1)) +
                                sizeof(cx<T>) * L;
  static constexpr bool OK = THREADS >= 64 && THREADS <= 1024 && LDS <= 160 * 1024 &&
                             (TL & (TL - 1)) == 0 &&
                             (V < 4 || (L >= 16 && (!COL || TL * sizeof(T) * 2 >= 64))) &&
                             (V != 6 || L >= 32);
};

template <typename T, int L, bool COL, int V>
void launch_shape(int mode, const cx<T>* i, cx<T>* o, const cx<T>* w, const PassArgs& a,
                  int nrhs, hipStream_t s) {
  using S = Shape<T, L, COL, V>;
  if constexpr (!S::OK) {
    throw Error(AIM_ERR_INVALID_ARG, "FFT launch shape not available for this length");
  } else {
    dim3 grid(unsigned((a.nlines + S::TL - 1) / S::TL), unsigned(nrhs));
    AIM_REQUIRE(mode == 2 ? (a.Lin == L / 2 && a.Lout == L / 2)
                          : (mode == 0 || mode == 3) ? (a.Lin == L / 2 && a.Lout == L)
                                                     : (a.Lin == L && a.Lout == L / 2),
                AIM_ERR_INVALID_ARG, "convolution FFT pass: lines must be half zero padding");
    if (mode == 3) {
      if constexpr (!COL)
        hipLaunchKernelGGL((fft_pass_kernel<T, L, S::TL, S::NT, 3, false, S::RMAX, true>), grid, dim3(S::THREADS), 0, s, i, o, w, a);
      else
        throw Error(AIM_ERR_INVALID_ARG, "the fused projection is a row pass");
    } else if (mode == 0)
      hipLaunchKernelGGL((fft_pass_kernel<T, L, S::TL, S::NT, 0, COL, S::RMAX, true>), grid, dim3(S::THREADS), 0, s, i, o, w, a);
    else if (mode == 1)
      hipLaunchKernelGGL((fft_pass_kernel<T, L, S::TL, S::NT, 1, COL, S::RMAX, true>), grid, dim3(S::THREADS), 0, s, i, o, w, a);
    else if constexpr (COL)
      hipLaunchKernelGGL((fft_pass_kernel<T, L, S::TL, S::NT, 2, COL, S::RMAX, true>), grid, dim3(S::THREADS), 0, s, i, o, w, a);
    else
      throw Error(AIM_ERR_INVALID_ARG, "row passes have no spectral multiply");
  }
}

template <typename T, int L>
void pass_L(bool col, int mode, int variant, const void* in, void* out, const void* tw,
            const PassArgs& a, int nrhs, hipStream_t s) {
  const cx<T>* i = static_cast<const cx<T>*>(in);
  cx<T>* o = static_cast<cx<T>*>(out);
  const cx<T>* w = static_cast<const cx<T>*>(tw);
  switch (variant * 2 + (col ? 1 : 0)) {
    case 0: launch_shape<T, L, false, 0>(mode, i, o, w, a, nrhs, s); break;
    case 1: launch_shape<T, L, true, 0>(mode, i, o, w, a, nrhs, s); break;
    case 2: launch_shape<T, L, false, 1>(mode, i, o, w, a, nrhs, s); break;
    case 3: launch_shape<T, L, true, 1>(mode, i, o, w, a, nrhs, s); break;
    case 4: launch_shape<T, L, false, 2>(mode, i, o, w, a, nrhs, s); break;
    case 5: launch_shape<T, L, true, 2>(mode, i, o, w, a, nrhs, s); break;
    case 6: launch_shape<T, L, false, 3>(mode, i, o, w, a, nrhs, s); break;
    case 7: launch_shape<T, L, true, 3>(mode, i, o, w, a, nrhs, s); break;
    case 8: launch_shape<T, L, false, 4>(mode, i, o, w, a, nrhs, s); break;
    case 9: launch_shape<T, L, true, 4>(mode, i, o, w, a, nrhs, s); break;
    case 10: launch_shape<T, L, false, 5>(mode, i, o, w, a, nrhs, s); break;
    case 11: launch_shape<T, L, true, 5>(mode, i, o, w, a, nrhs, s); break;
    case 12: launch_shape<T, L, false, 6>(mode, i, o, w, a, nrhs, s); break;
    case 13: launch_shape<T, L, true, 6>(mode, i, o, w, a, nrhs, s); break;
    case 14: launch_shape<T, L, false, 7>(mode, i, o, w, a, nrhs, s); break;
    case 15: launch_shape<T, L, true, 7>(mode, i, o, w, a, nrhs, s); break;
    default: throw Error(AIM_ERR_INVALID_ARG, "FFT launch shape out of range");
  }
}

template <typename T>
void fft_pass(int L, bool col, int mode, const void* in, void* out, const void* tw,
              const PassArgs& a, int nrhs, hipStream_t s, int variant = 0) {
  switch (L) {
    case 16: pass_L<T, 16>(col, mode, variant, in, out, tw, a, nrhs, s); break;
    case 32: pass_L<T, 32>(col, mode, variant, in, out, tw, a, nrhs, s); break;
    case 64: pass_L<T, 64>(col, mode, variant, in, out, tw, a, nrhs, s); break;
    case 128: pass_L<T, 128>(col, mode, variant, in, out, tw, a, nrhs, s); break;
    case 256: pass_L<T, 256>(col, mode, variant, in, out, tw, a, nrhs, s); break;
    case 512: pass_L<T, 512>(col, mode, variant, in, out, tw, a, nrhs, s); break;
    default: throw Error(AIM_ERR_GRID, "unsupported FFT length");
  }
  AIM_HIP(hipGetLastError());
}

// whole-line forward transform (the kernel spectrum), launch shape 0
template <typename T, int L, bool COL>
void full_forward_L(const void* in, void* out, const void* tw, const PassArgs& a, hipStream_t s) {
  using S = Shape<T, L, COL, 0>;
  static_assert(S::OK, "shape 0 exists for every length");
  dim3 grid(unsigned((a.nlines + S::TL - 1) / S::TL), 1u);
  hipLaunchKernelGGL((fft_pass_kernel<T, L, S::TL, S::NT, 0, COL, S::RMAX, false>), grid,
                     dim3(S::THREADS), 0, s, static_cast<const cx<T>*>(in), static_cast<cx<T>*>(out),
                     static_cast<const cx<T>*>(tw), a);
}

template <typename T>
void fft_full_forward(int L, bool col, const void* in, void* out, const void* tw,
                      const PassArgs& a, hipStream_t s) {
  switch (L * 2 + (col ? 1 : 0)) {
    case 32: full_forward_L<T, 16, false>(in, out, tw, a, s); break;
    case 33: full_forward_L<T, 16, true>(in, out, tw, a, s); break;
    case 64: full_forward_L<T, 32, false>(in, out, tw, a, s); break;
    case 65: full_forward_L<T, 32, true>(in, out, tw, a, s); break;
    case 128: full_forward_L<T, 64, false>(in, out, tw, a, s); break;
    case 129: full_forward_L<T, 64, true>(in, out, tw, a, s); break;
    case 256: full_forward_L<T, 128, false>(in, out, tw, a, s); break;
    case 257: full_forward_L<T, 128, true>(in, out, tw, a, s); break;
    case 512: full_forward_L<T, 256, false>(in, out, tw, a, s); break;
    case 513: full_forward_L<T, 256, true>(in, out, tw, a, s); break;
    case 1024: full_forward_L<T, 512, false>(in, out, tw, a, s); break;
    case 1025: full_forward_L<T, 512, true>(in, out, tw, a, s); break;
    default: throw Error(AIM_ERR_GRID, "unsupported FFT length");
  }
  AIM_HIP(hipGetLastError());
}

template <typename T, int L>
bool shape_ok_L(bool col, int v) {
  switch (v * 2 + (col ? 1 : 0)) {
    case 0: return Shape<T, L, false, 0>::OK;
    case 1: return Shape<T, L, true, 0>::OK;
    case 2: return Shape<T, L, false, 1>::OK;
    case 3: return Shape<T, L, true, 1>::OK;
    case 4: return Shape<T, L, false, 2>::OK;
    case 5: return Shape<T, L, true, 2>::OK;
    case 6: return Shape<T, L, false, 3>::OK;
    case 7: return Shape<T, L, true, 3>::OK;
    case 8: return Shape<T, L, false, 4>::OK;
    case 9: return Shape<T, L, true, 4>::OK;
    case 10: return Shape<T, L, false, 5>::OK;
    case 11: return Shape<T, L, true, 5>::OK;
    case 12: return Shape<T, L, false, 6>::OK;
    case 13: return Shape<T, L, true, 6>::OK;
    case 14: return Shape<T, L, false, 7>::OK;
    case 15: return Shape<T, L, true, 7>::OK;
    default: return false;
  }
}

template <typename T>
bool fft_shape_ok(int L, bool col, int v) {
  switch (L) {
    case 16: return shape_ok_L<T, 16>(col, v);
    case 32: return shape_ok_L<T, 32>(col, v);
    case 64: return shape_ok_L<T, 64>(col, v);
    case 128: return shape_ok_L<T, 128>(col, v);
    case 256: return shape_ok_L<T, 256>(col, v);
    case 512: return shape_ok_L<T, 512>(col, v);
    default: return false;
  }
}

// ---------------------------------------------------------------------------
// Fused z pass, persistent and software-pipelined (z-pass shapes 8 and up).
// A set is TL adjacent z lines (kx .. kx+TL-1 of one row ky).  Each workgroup
// walks a strided list of sets and, while it transforms one set, has the
// loads of the next one in flight, so the memory pipe keeps streaming during
// the butterflies and LDS exchanges (a workgroup of the one-set-per-launch
// kernel above leaves it idle for that time).  The twiddle table is loaded
// once per workgroup, after the first set's loads are issued.  The pass
// length L = Mz = 2 Nz is fixed at compile time: the forward transform reads
// only z < L/2 (the rest is the zero padding) and the inverse stores only
// z < L/2.  Sets are dealt to XCDs in contiguous runs, rows in the order 0,
// 1, My-1, 2, My-2, ... so that rows sharing a folded spectrum plane run on
// the same XCD (as in the kernel above).
// ---------------------------------------------------------------------------
struct ZconvArgs {
  int64_t es;  // element stride along z (plane pitch of the work grid)
  int64_t bs;  // per right-hand-side stride of the work grid
  const void* spec;
  int64_t spec_fs;  // per-frequency stride of the folded spectrum
  const int32_t* rhs_freq;
  int Mx, Nx, My, Ny, Nz;
  int nsets;  // Mx My / TL
};

template <typename T, int L, int TL, int NT, int RMAX>
__global__ __launch_bounds__(TL* NT) void zconv_kernel(cx<T>* B, const cx<T>* __restrict__ twg,
                                                       ZconvArgs a) {
  constexpr int E = L / NT, NTH = TL * NT;
  static_assert(RMAX <= E, "a thread must hold a whole butterfly");
  __shared__ cx<T> s[L * TL];
  __shared__ cx<T> tw[L];
  const int tid = threadIdx.x;
  const int l = tid & (TL - 1), t = tid / TL;
  B += int64_t(blockIdx.y) * a.bs;
  const cx<T>* spec =
      static_cast<const cx<T>*>(a.spec) + int64_t(a.rhs_freq[blockIdx.y]) * a.spec_fs;
  // sets first, first + step, ... below last
  const int G = int(gridDim.x), b = int(blockIdx.x);
  int first = b, step = G, last = a.nsets;
  if (G % 8 == 0 && a.nsets % 8 == 0) {
    const int per = a.nsets / 8;
    first = (b % 8) * per + b / 8;
    step = G / 8;
    last = (b % 8 + 1) * per;
  }
  const int nbx = a.Mx / TL, hy = a.My / 2;
  auto row_of = [&](int si) {
    const int rowpos = si / nbx;
    return rowpos == 0 ? 0
         : rowpos == a.My - 1 ? hy
         : (rowpos & 1) ? (rowpos + 1) / 2 : a.My - rowpos / 2;
  };
  auto col_of = [&](int si) { return (si % nbx) * TL + l; };
  // first forward stage: radix R0 over elements t + i NT + r L/R0; those
  // with r >= R0/2 lie in the zero padding
  using Fw = Sched<L, true, RMAX>;
  using Iv = Sched<L, false, RMAX>;
  constexpr int R0 = Fw::radix(0), NB0 = L / (R0 * NT), RH = R0 / 2;
  constexpr int RM = Fw::radix(Fw::NST - 1);
  static_assert(RM == Iv::radix(0),
                "the forward transform must end with the radix the inverse starts with");
  constexpr int Rf = Iv::radix(Iv::NST - 1), NBf = L / (Rf * NT);
  cx<T> nx[NB0 * RH];
  auto load = [&](int si) {
    const cx<T>* src = B + int64_t(row_of(si)) * a.Mx + col_of(si);
#pragma unroll
    for (int i = 0; i < NB0; ++i)
#pragma unroll
      for (int r = 0; r < RH; ++r) nx[i * RH + r] = src[int64_t(t + i * NT + r * (L / R0)) * a.es];
  };
  int si = first;
  if (si < last) load(si);
  for (int m = tid; m < L; m += NTH) tw[m] = twg[m];
  __syncthreads();
  cx<T>* sl = s + l;
  for (; si < last; si += step) {
    cx<T> v[E];
#pragma unroll
    for (int i = 0; i < NB0; ++i)
#pragma unroll
      for (int r = 0; r < R0; ++r) v[i * R0 + r] = r < RH ? nx[i * RH + r] : mkc<T>(T(0), T(0));
    const int ky = row_of(si), kx = col_of(si);
    // this set's spectrum values (needed after the forward transform), then
    // the next set's loads: both in flight during the forward transform
    cx<T> spv[E];
    {
      const int fx = kx <= a.Nx ? kx : a.Mx - kx;
      const int fy = ky <= a.Ny ? ky : a.My - ky;
      const cx<T>* sp = spec + int64_t(fy) * (a.Nz + 1) * (a.Nx + 1) + fx;
      const int64_t zst = int64_t(a.Nx + 1);
#pragma unroll
      for (int i = 0; i < L / (RM * NT); ++i)
#pragma unroll
        for (int r = 0; r < RM; ++r) {
          const int e = t + i * NT + r * (L / RM);
          const int fz = e <= a.Nz ? e : L - e;
          spv[i * RM + r] = sp[fz * zst];
        }
    }
    // (the last set reloads itself, unused: no branch, so the waits on these
    // loads are counted exactly)
    load(si + step < last ? si + step : si);
    run_stages<T, L, NT, false, true, RMAX, 0, true>(v, sl, TL, t, tw);
#pragma unroll
    for (int k = 0; k < E; ++k) v[k] = cmul(v[k], spv[k]);
    run_stages<T, L, NT, true, false, RMAX, 0>(v, sl, TL, t, tw);
    cx<T>* dst = B + int64_t(ky) * a.Mx + kx;
#pragma unroll
    for (int i = 0; i < NBf; ++i)
#pragma unroll
      for (int r = 0; r < Rf / 2; ++r)
        dst[int64_t(t + i * NT + r * (L / Rf)) * a.es] = v[i * Rf + r];
  }
}

// z-pass shapes 8 .. 8 + kZconvShapes - 1 (lines per set TL, threads per
// line NT, largest radix)
template <typename T, int L, int V>
struct ZShape {
  static constexpr int kTL = sizeof(T) == 8 ? 8 : 16;  // 128-byte row segments
  // V 0: radix 8, 8 elements per thread where the 512-thread cap allows;
  // V 1: radix 16, 256 threads; V 2: radix 16, 512 threads; V 3: radix 8,
  // 256 threads (short lines: more lines per set, at most 64, so that a
  // workgroup has at least one wave)
  static constexpr int NT = V == 0 ? cmin(L / 8, 512 / kTL)
                          : V == 1 ? cmax(1, L / 16)
                          : V == 2 ? cmax(1, L / 16)
                                   : cmin(L / 8, 256 / kTL);
  static constexpr int TL = V == 1 ? cmin(64, cmax(kTL, 256 / NT))
                          : V == 2 ? cmin(64, cmax(kTL, 512 / NT))
                                   : cmin(64, cmax(kTL, 64 / NT));
  static constexpr int RMAX = (V == 1 || V == 2) && L >= 16 ? 16 : 8;
  static constexpr int THREADS = TL * NT;
  static constexpr size_t LDS = sizeof(cx<T>) * (size_t(L) * TL + L);
  static constexpr bool OK = L >= 16 && L / NT >= RMAX && THREADS >= 64 && THREADS <= 1024 &&
                             LDS <= 160 * 1024;
};

template <typename T, int L, int V>
void launch_zshape(cx<T>* B, const cx<T>* w, ZconvArgs a, int nrhs, hipStream_t s) {
  using S = ZShape<T, L, V>;
  if constexpr (!S::OK) {
    throw Error(AIM_ERR_INVALID_ARG, "z-pass shape not available for this length");
  } else {
    AIM_REQUIRE(a.Mx % S::TL == 0 && a.My % 2 == 0, AIM_ERR_INVALID_ARG,
                "z-pass shape needs the padded x length to be a multiple of its lines per set");
    a.nsets = int(int64_t(a.Mx) * a.My / S::TL);
    auto kern = zconv_kernel<T, L, S::TL, S::NT, S::RMAX>;
    // one wave of workgroups: as many as can be resident on the device
    static int resident = 0;
    if (resident == 0) {
      int dev = 0, ncu = 0, per = 0;
      AIM_HIP(hipGetDevice(&dev));
      AIM_HIP(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
      AIM_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, kern, S::THREADS, 0));
      resident = std::max(8, (ncu * std::max(per, 1)) / 8 * 8);
    }
    const int G = std::min(resident, a.nsets);
    hipLaunchKernelGGL(kern, dim3(unsigned(G), unsigned(nrhs)), dim3(S::THREADS), 0, s, B, w, a);
  }
}

template <typename T, int L>
void zconv_L(int v, cx<T>* B, const cx<T>* w, const ZconvArgs& a, int nrhs, hipStream_t s) {
  switch (v) {
    case 0: launch_zshape<T, L, 0>(B, w, a, nrhs, s); break;
    case 1: launch_zshape<T, L, 1>(B, w, a, nrhs, s); break;
    case 2: launch_zshape<T, L, 2>(B, w, a, nrhs, s); break;
    case 3: launch_zshape<T, L, 3>(B, w, a, nrhs, s); break;
    default: throw Error(AIM_ERR_INVALID_ARG, "z-pass shape out of range");
  }
}

template <typename T>
void zconv(int L, int v, void* B, const void* tw, const ZconvArgs& a, int nrhs, hipStream_t s) {
  cx<T>* b = static_cast<cx<T>*>(B);
  const cx<T>* w = static_cast<const cx<T>*>(tw);
  switch (L) {
    case 16: zconv_L<T, 16>(v, b, w, a, nrhs, s); break;
    case 32: zconv_L<T, 32>(v, b, w, a, nrhs, s); break;
    case 64: zconv_L<T, 64>(v, b, w, a, nrhs, s); break;
    case 128: zconv_L<T, 128>(v, b, w, a, nrhs, s); break;
    case 256: zconv_L<T, 256>(v, b, w, a, nrhs, s); break;
    case 512: zconv_L<T, 512>(v, b, w, a, nrhs, s); break;
    default: throw Error(AIM_ERR_GRID, "unsupported FFT length");
  }
  AIM_HIP(hipGetLastError());
}

template <typename T, int L>
bool zshape_ok_L(int v, int Mx) {
  switch (v) {
    case 0: return ZShape<T, L, 0>::OK && Mx % ZShape<T, L, 0>::TL == 0;
    case 1: return ZShape<T, L, 1>::OK && Mx % ZShape<T, L, 1>::TL == 0;
    case 2: return ZShape<T, L, 2>::OK && Mx % ZShape<T, L, 2>::TL == 0;
    case 3: return ZShape<T, L, 3>::OK && Mx % ZShape<T, L, 3>::TL == 0;
    default: return false;
  }
}

template <typename T>
bool zshape_ok(int L, int v, int Mx) {
  switch (L) {
    case 16: return zshape_ok_L<T, 16>(v, Mx);
    case 32: return zshape_ok_L<T, 32>(v, Mx);
    case 64: return zshape_ok_L<T, 64>(v, Mx);
    case 128: return zshape_ok_L<T, 128>(v, Mx);
    case 256: return zshape_ok_L<T, 256>(v, Mx);
    case 512: return zshape_ok_L<T, 512>(v, Mx);
    default: return false;
  }
}

bool fft_variant_ok(bool dbl, const GridShape& g, int pass, int v) {
  static const int axis[5] = {0, 1, 2, 1, 0};
  const int L = g.M[axis[pass]];
  if (v >= kFftShapesPerLine) {  // persistent shapes: the fused z pass only
    if (pass != 2 || v >= kFftVariants) return false;
    return dbl ? zshape_ok<double>(L, v - kFftShapesPerLine, g.M[0])
               : zshape_ok<float>(L, v - kFftShapesPerLine, g.M[0]);
  }
  const bool col = pass >= 1 && pass <= 3;
  return dbl ? fft_shape_ok<double>(L, col, v) : fft_shape_ok<float>(L, col, v);
}

// row (x) pass over nplanes x rows lines: line (z, y) starts at
// z * ps + y * ls
template <typename T>
void row_pass(int L, bool inv, const void* in, void* out, const void* tw, int64_t nplanes,
              int rows, int64_t in_ls, int64_t out_ls, int64_t in_ps, int64_t out_ps,
              int64_t in_bs, int64_t out_bs, int Lin, int Lout, int nrhs, hipStream_t s,
              int variant = 0, const CsrDevice* P = nullptr, const void* x = nullptr,
              int64_t n = 0) {
  PassArgs a{};
  a.nlines = nplanes * rows;
  a.lg_nli = ilog2(rows);
  a.in_es = a.out_es = 1;
  a.in_os = in_ps;
  a.out_os = out_ps;
  a.in_p0 = in_ls;
  a.out_p0 = out_ls;
  a.in_bs = in_bs;
  a.out_bs = out_bs;
  a.Lin = Lin;
  a.Lout = Lout;
  if (P) {  // the input lines are q = P x, computed in the pass
    AIM_REQUIRE(!inv && in_ls == Lin && in_ps == int64_t(rows) * Lin, AIM_ERR_INVALID_ARG,
                "the fused projection reads unpadded grid rows");
    a.prow = P->rowptr;
    a.pcol = P->col;
    a.pval = P->val;
    a.px = x;
    a.px_bs = n;
  }
  fft_pass<T>(L, false, P ? 3 : (inv ? 1 : 0), in, out, tw, a, nrhs, s, variant);
}

// ---------------------------------------------------------------------------
// convolution phi = H q: pruned forward FFT, spectral multiply, pruned inverse
// work layout per right-hand side: B = [Nz][My][Mx] (4 Ng) followed by
// A = [Nz][Ny][Mx] (2 Ng), each z plane padded by the layout's pad so that
// the z lines (one element per plane) do not all fall on the same memory
// channel when the plane size is a large power of two.
// ---------------------------------------------------------------------------
int64_t work_elems(const GridShape& g, int layout, size_t elem_bytes) {
  const int64_t pad = kLayoutPadBytes[layout] / int64_t(elem_bytes);
  return int64_t(g.N[2]) * (int64_t(g.M[1]) * g.M[0] + pad + int64_t(g.N[1]) * g.M[0] + pad);
}

template <typename T>
void launch_convolve(const GridShape& g, const void* q, void* work, void* phi, const void* spec,
                     const int32_t* rhs_freq, int nrhs, const void* const* tw, hipStream_t s,
                     hipEvent_t* between, const int* sched, int repeat, const CsrDevice* P,
                     const void* x, int64_t n, int stages) {
  static const int kDefault[kSchedLen] = {0, 0, 0, 0, 0, 0, 0};
  if (!sched) sched = kDefault;
  auto mark = [&](int i) {
    if (between) AIM_HIP(hipEventRecord(between[i], s));
  };
  const int Nx = g.N[0], Ny = g.N[1], Nz = g.N[2];
  const int Mx = g.M[0], My = g.M[1], Mz = g.M[2];
  const int64_t Ng = g.Ng;
  const int64_t pad = kLayoutPadBytes[sched[5]] / int64_t(sizeof(cx<T>));
  const int64_t PB = int64_t(My) * Mx + pad, PA = int64_t(Ny) * Mx + pad;  // plane pitches
  const int64_t W = work_elems(g, sched[5], sizeof(cx<T>));                 // per right-hand side
  cx<T>* B = static_cast<cx<T>*>(work);
  cx<T>* A = B + int64_t(Nz) * PB;
  auto col_args = [&](int64_t nlines, int64_t in_es, int64_t in_os, int64_t out_es,
                      int64_t out_os, int Lin, int Lout) {
    PassArgs a{};
    a.nlines = nlines;
    a.lg_nli = ilog2(Mx);
    a.in_es = in_es;
    a.in_os = in_os;
    a.out_es = out_es;
    a.out_os = out_os;
    a.in_p0 = a.out_p0 = 1;
    a.in_bs = a.out_bs = W;
    a.Lin = Lin;
    a.Lout = Lout;
    return a;
  };
  if (stages & 1) {
    // x forward: rows (y, z) of q, Nx -> Mx, into A [Nz][Ny][Mx]
    for (int r = 0; r < repeat; ++r)
      row_pass<T>(Mx, false, q, A, tw[0], Nz, Ny, Nx, Mx, int64_t(Ny) * Nx, PA, Ng, W, Nx, Mx,
                  nrhs, s, sched[0], P, x, n);
    mark(0);
    // y forward: A [Nz][Ny][Mx] -> B [Nz][My][Mx]
    {
      const PassArgs a = col_args(int64_t(Mx) * Nz, Mx, PA, Mx, PB, Ny, My);
      for (int r = 0; r < repeat; ++r)
        fft_pass<T>(My, true, 0, A, B, tw[1], a, nrhs, s, sched[1]);
    }
    mark(1);
  }
  // z forward * spectrum * z inverse, in place on B, keeping z < Nz
  if (stages & 2) {
    PassArgs a = col_args(int64_t(Mx) * My, PB, Mx, PB, Mx, Nz, Nz);
    a.spec = spec;
    a.spec_fs = g.Nfold;
    a.rhs_freq = rhs_freq;
    a.Mx = Mx;
    a.Nx = Nx;
    a.My = My;
    a.Ny = Ny;
    a.Mz = Mz;
    a.Nz = Nz;
    if (sched[2] >= kFftShapesPerLine) {
      ZconvArgs z{};
      z.es = PB;
      z.bs = W;
      z.spec = spec;
      z.spec_fs = g.Nfold;
      z.rhs_freq = rhs_freq;
      z.Mx = Mx;
      z.Nx = Nx;
      z.My = My;
      z.Ny = Ny;
      z.Nz = Nz;
      for (int r = 0; r < repeat; ++r)
        zconv<T>(Mz, sched[2] - kFftShapesPerLine, B, tw[2], z, nrhs, s);
    } else {
      for (int r = 0; r < repeat; ++r)
        fft_pass<T>(Mz, true, 2, B, B, tw[2], a, nrhs, s, sched[2]);
    }
  }
  mark(2);
  if (stages & 4) {
    // y inverse: B [Nz][My][Mx] -> A [Nz][Ny][Mx]
    {
      const PassArgs a = col_args(int64_t(Mx) * Nz, Mx, PB, Mx, PA, My, Ny);
      for (int r = 0; r < repeat; ++r)
        fft_pass<T>(My, true, 1, B, A, tw[1], a, nrhs, s, sched[3]);
    }
    mark(3);
    // x inverse: rows of A (Mx) -> phi (Nx)
    for (int r = 0; r < repeat; ++r)
      row_pass<T>(Mx, true, A, phi, tw[0], Nz, Ny, Mx, Nx, PA, int64_t(Ny) * Nx, W, Ng, Mx, Nx,
                  nrhs, s, sched[4]);
  }
}

// the gradient z pass over nvec vectors' three channels (channel c of
// vector r is workspace grid c nvec + r in both buffers)
template <typename T, int L, int V>
void zcross_shape(bool dot, const cx<T>* i, cx<T>* o, const cx<T>* w, const PassArgs& a,
                  int nvec, hipStream_t s) {
  using S = Shape<T, L, true, V>;
  if constexpr (!S::OK || S::RMAX != 8) {
    throw Error(AIM_ERR_INVALID_ARG, "gradient z pass: launch shape not available");
  } else {
    const dim3 grid(unsigned((a.nlines + S::TL - 1) / S::TL), unsigned(nvec));
    if (dot)
      hipLaunchKernelGGL((zcross_kernel<T, L, S::TL, S::NT, S::RMAX, true>), grid,
                         dim3(S::THREADS), 0, s, i, o, w, a);
    else
      hipLaunchKernelGGL((zcross_kernel<T, L, S::TL, S::NT, S::RMAX, false>), grid,
                         dim3(S::THREADS), 0, s, i, o, w, a);
  }
}

template <typename T, int L>
int zcross_elems(int v) {  // elements per thread of column shape v (0 if unavailable)
  switch (v) {
    case 0: return Shape<T, L, true, 0>::OK ? L / Shape<T, L, true, 0>::NT : 0;
    case 1: return Shape<T, L, true, 1>::OK ? L / Shape<T, L, true, 1>::NT : 0;
    case 2: return Shape<T, L, true, 2>::OK ? L / Shape<T, L, true, 2>::NT : 0;
    case 3: return Shape<T, L, true, 3>::OK ? L / Shape<T, L, true, 3>::NT : 0;
    default: return 0;
  }
}

template <typename T, int L>
void zcross_L(bool dot, int pref, const cx<T>* i, cx<T>* o, const cx<T>* w, const PassArgs& a,
              int nvec, hipStream_t s) {
  // the z pass's own shape when it is a radix-8 one holding at most 64
  // bytes of each channel per thread, else the available radix-8 shape with
  // the fewest elements per thread (six lines' worth of registers per thread)
  constexpr int kMaxBytes = 64;
  int v = -1;
  if (pref >= 0 && pref < 4) {
    const int e = zcross_elems<T, L>(pref);
    if (e > 0 && e * int(sizeof(T)) <= kMaxBytes) v = pref;
  }
  if (v < 0) {
    int best = 0;
    for (int c = 0; c < 4; ++c) {
      const int e = zcross_elems<T, L>(c);
      if (e > 0 && (v < 0 || e < best)) v = c, best = e;
    }
  }
  switch (v) {
    case 0: zcross_shape<T, L, 0>(dot, i, o, w, a, nvec, s); break;
    case 1: zcross_shape<T, L, 1>(dot, i, o, w, a, nvec, s); break;
    case 2: zcross_shape<T, L, 2>(dot, i, o, w, a, nvec, s); break;
    case 3: zcross_shape<T, L, 3>(dot, i, o, w, a, nvec, s); break;
    default: throw Error(AIM_ERR_GRID, "no launch shape for the cross-product z pass");
  }
}

template <typename T>
void launch_zcross(const GridShape& g, const void* work_in, void* work_out, const void* spec3,
                   const int32_t* vec_freq, int nvec, const void* const* tw, hipStream_t s,
                   const int* sched, bool dot) {
  static const int kDefault[kSchedLen] = {0, 0, 0, 0, 0, 0, 0};
  if (!sched) sched = kDefault;
  const int Nx = g.N[0], Ny = g.N[1], Nz = g.N[2];
  const int Mx = g.M[0], My = g.M[1], Mz = g.M[2];
  const int64_t pad = kLayoutPadBytes[sched[5]] / int64_t(sizeof(cx<T>));
  const int64_t PB = int64_t(My) * Mx + pad;
  const int64_t W = work_elems(g, sched[5], sizeof(cx<T>));
  PassArgs a{};
  a.nlines = int64_t(Mx) * My;
  a.lg_nli = ilog2(Mx);
  a.in_es = a.out_es = PB;
  a.in_os = a.out_os = Mx;
  a.in_p0 = a.out_p0 = 1;
  a.in_bs = a.out_bs = W;
  a.Lin = a.Lout = Nz;
  a.ch_bs = int64_t(nvec) * W;
  a.spec = spec3;
  a.spec_cs = g.Nfold;
  a.spec_fs = 3 * g.Nfold;
  a.rhs_freq = vec_freq;
  a.Mx = Mx;
  a.Nx = Nx;
  a.My = My;
  a.Ny = Ny;
  a.Mz = Mz;
  a.Nz = Nz;
  const cx<T>* i = static_cast<const cx<T>*>(work_in);
  cx<T>* o = static_cast<cx<T>*>(work_out);
  const cx<T>* w = static_cast<const cx<T>*>(tw[2]);
  const int pref = sched[2] < kFftShapesPerLine ? sched[2] : -1;
  switch (Mz) {
    case 16: zcross_L<T, 16>(dot, pref, i, o, w, a, nvec, s); break;
    case 32: zcross_L<T, 32>(dot, pref, i, o, w, a, nvec, s); break;
    case 64: zcross_L<T, 64>(dot, pref, i, o, w, a, nvec, s); break;
    case 128: zcross_L<T, 128>(dot, pref, i, o, w, a, nvec, s); break;
    case 256: zcross_L<T, 256>(dot, pref, i, o, w, a, nvec, s); break;
    case 512: zcross_L<T, 512>(dot, pref, i, o, w, a, nvec, s); break;
    default: throw Error(AIM_ERR_GRID, "unsupported FFT length");
  }
  AIM_HIP(hipGetLastError());
}

template void launch_zcross<double>(const GridShape&, const void*, void*, const void*,
                                    const int32_t*, int, const void* const*, hipStream_t,
                                    const int*, bool);
template void launch_zcross<float>(const GridShape&, const void*, void*, const void*,
                                   const int32_t*, int, const void* const*, hipStream_t,
                                   const int*, bool);

template void launch_convolve<double>(const GridShape&, const void*, void*, void*, const void*,
                                      const int32_t*, int, const void* const*, hipStream_t,
                                      hipEvent_t*, const int*, int, const CsrDevice*,
                                      const void*, int64_t, int);
template void launch_convolve<float>(const GridShape&, const void*, void*, void*, const void*,
                                     const int32_t*, int, const void* const*, hipStream_t,
                                     hipEvent_t*, const int*, int, const CsrDevice*, const void*,
                                     int64_t, int);

// ---------------------------------------------------------------------------
// kernel spectrum: circulant embedding of G on the padded grid, full 3-D FFT,
// folded to its (Nx+1)(Ny+1)(Nz+1) distinct entries (the embedding is even in
// every axis), scaled by 1/(Mx My Mz) and stored [fy][fz][fx]
// ---------------------------------------------------------------------------
__global__ void green_sample_kernel(double2* c, int Nx, int Ny, int Nz, double k, double h,
                                    int kind) {
  const int Mx = 2 * Nx, My = 2 * Ny, Mz = 2 * Nz;
  const int64_t total = int64_t(Mx) * My * Mz;
  for (int64_t idx = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; idx < total;
       idx += int64_t(gridDim.x) * blockDim.x) {
    const int ix = int(idx % Mx);
    const int iy = int((idx / Mx) % My);
    const int iz = int(idx / (int64_t(Mx) * My));
    double2 v;
    v.x = 0.0;
    v.y = 0.0;
    if (ix != Nx && iy != Ny && iz != Nz) {
      const double dx = ix < Nx ? ix : ix - Mx;
      const double dy = iy < Ny ? iy : iy - My;
      const double dz = iz < Nz ? iz : iz - Mz;
      const double d2 = dx * dx + dy * dy + dz * dz;
      const double inv4pi = 0.07957747154594766788;  // 1/(4 pi)
      if (kind >= 1) {
        // kind 1: F = h (1 + jkR) e^{-jkR} / (4 pi R^3); kinds 2, 3, 4: the
        // gradient of G with respect to the observation point, component
        // a = kind - 2, i.e. -d_a F with d in node units; 0 at the origin
        if (d2 != 0.0) {
          const double R = h * sqrt(d2);
          double sn, cs;
          sincos(k * R, &sn, &cs);
          double a = h * inv4pi / (R * R * R);
          if (kind >= 2) a *= -(kind == 2 ? dx : kind == 3 ? dy : dz);
          const double kr = k * R;
          v.x = (cs + kr * sn) * a;
          v.y = (kr * cs - sn) * a;
        }
      } else if (d2 == 0.0) {
        v.y = -k * inv4pi;  // -jk/(4 pi): modified self term
      } else {
        const double R = h * sqrt(d2);
        double sn, cs;
        sincos(k * R, &sn, &cs);
        const double a = inv4pi / R;
        v.x = cs * a;
        v.y = -sn * a;
      }
    }
    c[idx] = v;
  }
}

__global__ void fold_spectrum_kernel(const double2* full, double2* s64, float2* s32, int Nx,
                                     int Ny, int Nz, double scale, int odd) {
  const int Fx = Nx + 1, Fy = Ny + 1, Fz = Nz + 1;
  const int64_t total = int64_t(Fx) * Fy * Fz;
  const int Mx = 2 * Nx, My = 2 * Ny;
  for (int64_t idx = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; idx < total;
       idx += int64_t(gridDim.x) * blockDim.x) {
    // output layout [fy][fz][fx]
    const int fx = int(idx % Fx), fz = int((idx / Fx) % Fz), fy = int(idx / (int64_t(Fx) * Fz));
    double2 v = full[(int64_t(fz) * My + fy) * Mx + fx];
    v.x *= scale;
    v.y *= scale;
    // a kernel odd along one axis has a spectrum odd along it, exactly zero
    // at its frequencies 0 and N (there the transform only holds rounding)
    const int fo = odd == 0 ? fx : odd == 1 ? fy : fz, no = odd == 0 ? Nx : odd == 1 ? Ny : Nz;
    if (odd >= 0 && (fo == 0 || fo == no)) v.x = v.y = 0.0;
    s64[idx] = v;
    if (s32) {
      float2 w;
      w.x = float(v.x);
      w.y = float(v.y);
      s32[idx] = w;
    }
  }
}

void launch_spectrum(const GridShape& g, double k, double h, void* full_work, void* spec64,
                     void* spec32, const void* const* tw64, hipStream_t s, int kind) {
  const int Nx = g.N[0], Ny = g.N[1], Nz = g.N[2];
  const int Mx = g.M[0], My = g.M[1], Mz = g.M[2];
  double2* F = static_cast<double2*>(full_work);
  hipLaunchKernelGGL(green_sample_kernel, dim3(4096), dim3(256), 0, s, F, Nx, Ny, Nz, k, h,
                     kind);
  AIM_HIP(hipGetLastError());
  const int64_t Np = int64_t(Mx) * My * Mz;
  {  // rows (y, z) of the whole padded grid
    PassArgs a{};
    a.nlines = int64_t(Mz) * My;
    a.lg_nli = ilog2(My);
    a.in_es = a.out_es = 1;
    a.in_os = a.out_os = int64_t(My) * Mx;
    a.in_p0 = a.out_p0 = Mx;
    a.Lin = a.Lout = Mx;
    fft_full_forward<double>(Mx, false, F, F, tw64[0], a, s);
  }
  {
    PassArgs a{};
    a.nlines = int64_t(Mx) * Mz;
    a.lg_nli = ilog2(Mx);
    a.in_p0 = a.out_p0 = 1;
    a.in_es = a.out_es = Mx;
    a.in_os = a.out_os = int64_t(My) * Mx;
    a.Lin = a.Lout = My;
    fft_full_forward<double>(My, true, F, F, tw64[1], a, s);
  }
  {
    PassArgs a{};
    a.nlines = int64_t(Mx) * My;
    a.lg_nli = ilog2(Mx);
    a.in_p0 = a.out_p0 = 1;
    a.in_es = a.out_es = int64_t(My) * Mx;
    a.in_os = a.out_os = Mx;
    a.Lin = a.Lout = Mz;
    fft_full_forward<double>(Mz, true, F, F, tw64[2], a, s);
  }
  hipLaunchKernelGGL(fold_spectrum_kernel, dim3(2048), dim3(256), 0, s, F,
                     static_cast<double2*>(spec64), static_cast<float2*>(spec32), Nx, Ny, Nz,
                     1.0 / double(Np), kind >= 2 ? kind - 2 : -1);
  AIM_HIP(hipGetLastError());
}

std::vector<double> twiddles64(int L) {
  std::vector<double> t(2 * L);
  for (int m = 0; m < L; ++m) {
    // exp(-2 pi i m / L) in long double, rounded once
    const long double ang = -2.0L * 3.141592653589793238462643383279502884L * m / L;
    t[2 * m] = double(cosl(ang));
    t[2 * m + 1] = double(sinl(ang));
  }
  return t;
}

// ---------------------------------------------------------------------------
// projection q = P x
//
// P is assembled once at set-up (the quadrature-point stencil weights of each
// triangle merged into one row per grid node, sorted by node) and cut into
// blocks of consecutive rows holding at most kProjNnz non-zeros.  A block
// loads all its non-zeros and row starts at once (coalesced loads, then
// independent gathers of x, every load in flight before the first is used),
// forms the products in LDS, then each thread sums whole rows from LDS in a
// fixed order (four interleaved partial sums), so the
// result is reproducible and no atomics are needed.  Nodes that no stencil
// reaches get their zero written by the same pass; long runs of them form
// blocks of their own that only store zeros.
// ---------------------------------------------------------------------------
template <typename T, int PR>
__global__ __launch_bounds__(256) void project_kernel(const cx<T>* __restrict__ x,
                                                      cx<T>* __restrict__ q,
                                                      const int32_t* __restrict__ rowptr,
                                                      const int32_t* __restrict__ col,
                                                      const T* __restrict__ val,
                                                      const int32_t* __restrict__ blk, int64_t n,
                                                      int64_t Ng, int nrhs, int rb) {
  constexpr int PER = kProjNnz / 256, RPER = kProjRows / 256 + 1;
  // PR right-hand sides side by side: their gathers in flight together, their
  // products in PR slices of LDS
  __shared__ cx<T> prod[PR * kProjNnz];
  __shared__ union {
    T red[2 * 256];           // long row
    int rp[kProjRows + 1];    // row starts of the block, relative to its first non-zero
  } sh;
  const int tid = threadIdx.x;
  const int r0 = blk[blockIdx.x], r1 = blk[blockIdx.x + 1];
  const int k0 = rowptr[r0], k1 = rowptr[r1];
  // rb right-hand sides per block (a multiple of PR): the block's rows of P
  // are read once and applied to each of them
  const int rhs_end = min(nrhs, int(blockIdx.y + 1) * rb);
  if (k0 == k1) {  // nodes no stencil reaches: zeros, without reading rowptr per row
    for (int rhs = int(blockIdx.y) * rb; rhs < rhs_end; ++rhs) {
      cx<T>* qr = q + rhs * Ng;
      for (int r = r0 + tid; r < r1; r += 256) qr[r] = mkc<T>(T(0), T(0));
    }
    return;
  }
  if (k1 - k0 > kProjNnz) {  // one long row: strided partial sums, block reduction
    for (int rhs = int(blockIdx.y) * rb; rhs < rhs_end; ++rhs) {
      const cx<T>* xr = x + rhs * n;
      T ar = T(0), ai = T(0);
      for (int k = k0 + tid; k < k1; k += 256) {
        const T w = val[k];
        const cx<T> xv = xr[col[k]];
        ar += w * xv.x;
        ai += w * xv.y;
      }
      sh.red[tid] = ar;
      sh.red[256 + tid] = ai;
      __syncthreads();
      for (int o = 128; o > 0; o >>= 1) {
        if (tid < o) {
          sh.red[tid] += sh.red[tid + o];
          sh.red[256 + tid] += sh.red[256 + tid + o];
        }
        __syncthreads();
      }
      if (tid == 0) q[rhs * Ng + r0] = mkc<T>(sh.red[0], sh.red[256]);
      __syncthreads();  // red is reused by the next right-hand side
    }
    return;
  }
  // the block's entries of P (PER per thread) and row starts: every load
  // issued before any is used
  T w[PER];
  int c[PER];
#pragma unroll
  for (int i = 0; i < PER; ++i) {
    const int k = k0 + tid + i * 256;
    w[i] = k < k1 ? val[k] : T(0);
    c[i] = k < k1 ? col[k] : 0;
  }
#pragma unroll
  for (int i = 0; i < RPER; ++i) {
    const int j = tid + i * 256;
    if (j <= r1 - r0) sh.rp[j] = rowptr[r0 + j] - k0;
  }
  const int R = r1 - r0;
  for (int rhs0 = int(blockIdx.y) * rb; rhs0 < rhs_end; rhs0 += PR) {
    const int nr = min(PR, rhs_end - rhs0);
    cx<T> xv[PR][PER];
#pragma unroll
    for (int j = 0; j < PR; ++j)
      if (j < nr) {
        const cx<T>* xr = x + (rhs0 + j) * n;
#pragma unroll
        for (int i = 0; i < PER; ++i) xv[j][i] = xr[c[i]];
      }
#pragma unroll
    for (int j = 0; j < PR; ++j)
      if (j < nr) {
#pragma unroll
        for (int i = 0; i < PER; ++i) {
          const int k = tid + i * 256;
          if (k < k1 - k0) prod[j * kProjNnz + k] = mkc<T>(w[i] * xv[j][i].x, w[i] * xv[j][i].y);
        }
      }
    __syncthreads();
    // row sums from LDS, four interleaved partial sums per row (fixed order),
    // one (row, right-hand side) pair per thread at a time
    for (int idx = tid; idx < R * nr; idx += 256) {
      const int j = idx / R, rr = idx - j * R;
      const cx<T>* pj = prod + j * kProjNnz;
      const int e = sh.rp[rr + 1];
      int k = sh.rp[rr];
      T ar[4] = {T(0), T(0), T(0), T(0)}, ai[4] = {T(0), T(0), T(0), T(0)};
      for (; k + 4 <= e; k += 4) {
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          ar[u] += pj[k + u].x;
          ai[u] += pj[k + u].y;
        }
      }
      for (int u = 0; k < e; ++k, ++u) {
        ar[u] += pj[k].x;
        ai[u] += pj[k].y;
      }
      q[(rhs0 + j) * Ng + r0 + rr] =
          mkc<T>((ar[0] + ar[1]) + (ar[2] + ar[3]), (ai[0] + ai[1]) + (ai[2] + ai[3]));
    }
    __syncthreads();  // prod is reused by the next group of right-hand sides
  }
}

// right-hand sides per workgroup: the largest power of two (at most 8, at
// most nrhs) that still leaves 1024 workgroups in the launch, else 1.  Each
// matrix entry is then loaded once and applied to that many vectors.
inline int rhs_per_block(int64_t blocks_per_rhs, int nrhs) {
  int rb = 1;
  while (rb < 8 && 2 * rb <= nrhs && blocks_per_rhs * ((nrhs + 2 * rb - 1) / (2 * rb)) >= 1024)
    rb *= 2;
  return rb;
}

// the projection serves several right-hand sides per workgroup (its rows of
// P then come from cache after the first) only on operators large enough that
// one right-hand side already fills 1024 workgroups; on small ones the rows
// are cache-resident anyway and the parallelism matters more
inline int project_rhs_per_block(int64_t blocks_per_rhs, int nrhs) {
  if (blocks_per_rhs < 1024) return 1;
  int rb = 1;
  while (rb < 8 && 2 * rb <= nrhs) rb *= 2;
  return rb;
}

template <typename T>
void launch_project(const GridShape& g, const CsrDevice& P, const int32_t* blk, int nblk,
                    const void* x, int64_t n, void* q, int nrhs, hipStream_t s) {
  // large operators: rb right-hand sides one after another per workgroup; small
  // ones with many right-hand sides: up to 4 (complex64) or 2 (complex128) side
  // by side, while the launch keeps 1024 workgroups
  int rb = project_rhs_per_block(nblk, nrhs), pr = 1;
  if (rb == 1) {
    const int pmax = sizeof(T) == 4 ? 4 : 2;
    while (pr < pmax && 2 * pr <= nrhs && int64_t(nblk) * ((nrhs + 2 * pr - 1) / (2 * pr)) >= 1024)
      pr *= 2;
    rb = pr;
  }
  const dim3 grid(unsigned(nblk), unsigned((nrhs + rb - 1) / rb));
  const cx<T>* xi = static_cast<const cx<T>*>(x);
  cx<T>* qo = static_cast<cx<T>*>(q);
  const T* v = static_cast<const T*>(P.val);
  if (pr == 4)
    hipLaunchKernelGGL((project_kernel<T, 4>), grid, dim3(256), 0, s, xi, qo, P.rowptr, P.col, v,
                       blk, n, g.Ng, nrhs, rb);
  else if (pr == 2)
    hipLaunchKernelGGL((project_kernel<T, 2>), grid, dim3(256), 0, s, xi, qo, P.rowptr, P.col, v,
                       blk, n, g.Ng, nrhs, rb);
  else
    hipLaunchKernelGGL((project_kernel<T, 1>), grid, dim3(256), 0, s, xi, qo, P.rowptr, P.col, v,
                       blk, n, g.Ng, nrhs, rb);
  AIM_HIP(hipGetLastError());
}

template void launch_project<double>(const GridShape&, const CsrDevice&, const int32_t*, int,
                                     const void*, int64_t, void*, int, hipStream_t);
template void launch_project<float>(const GridShape&, const CsrDevice&, const int32_t*, int,
                                    const void*, int64_t, void*, int, hipStream_t);

// ---------------------------------------------------------------------------
// interpolation y = P^T phi and near correction y += C x
//
// LPR lanes share one basis function: they stride over its row of P^T
// (grid potentials at the stencil nodes of its three quadrature points) and
// then over its row of C, and a reduction across the LPR lanes gives y_i.
// ---------------------------------------------------------------------------
template <int LPR, typename T>
__device__ __forceinline__ T group_sum(T v) {
#pragma unroll
  for (int o = LPR / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Lane sub of LPR lanes accumulates its share of the sparse row [k0, k1) of
// (col, val) against RB vectors v_j = base + j * stride: entries k0 + sub,
// k0 + sub + LPR, ... taken kRowBatch at a time, their indices and values
// loaded together, then the RB kRowBatch gathers, so a batch costs one
// exposed latency instead of one per entry.  The order of the sums is fixed.
constexpr int kRowBatch = 4;
template <typename T, int LPR, int RB>
__device__ __forceinline__ void row_gather(int k0, int k1, int sub, const int32_t* __restrict__ col,
                                           const T* __restrict__ val, const cx<T>* __restrict__ base,
                                           int64_t stride, int nr, T* ar, T* ai) {
  for (int kb = k0 + sub; kb < k1; kb += LPR * kRowBatch) {
    T w[kRowBatch];
    int c[kRowBatch];
#pragma unroll
    for (int u = 0; u < kRowBatch; ++u) {
      const int k = kb + u * LPR;
      w[u] = k < k1 ? val[k] : T(0);
      c[u] = k < k1 ? col[k] : 0;
    }
#pragma unroll
    for (int j = 0; j < RB; ++j)
      if (j < nr) {
        cx<T> v[kRowBatch];
#pragma unroll
        for (int u = 0; u < kRowBatch; ++u) v[u] = base[j * stride + c[u]];
#pragma unroll
        for (int u = 0; u < kRowBatch; ++u) {
          ar[j] += w[u] * v[u].x;
          ai[j] += w[u] * v[u].y;
        }
      }
  }
}

template <typename T, int LPR, bool INTERP, bool NEARC, int RB>
__global__ __launch_bounds__(256) void interp_near_kernel(
    const cx<T>* __restrict__ phi, const cx<T>* __restrict__ x, cx<T>* __restrict__ y,
    const int32_t* __restrict__ prow, const int32_t* __restrict__ pcol, const T* __restrict__ pval,
    const int32_t* __restrict__ rowptr, const int32_t* __restrict__ col,
    const T* __restrict__ val, int64_t n, int64_t Ng, int nrhs) {
  const int sub = threadIdx.x % LPR;
  const int64_t i = (int64_t(blockIdx.x) * blockDim.x + threadIdx.x) / LPR;
  // RB right-hand sides per workgroup: each matrix entry is loaded once
  const int rhs0 = int(blockIdx.y) * RB;
  const int nr = min(RB, nrhs - rhs0);
  T ar[RB], ai[RB];
#pragma unroll
  for (int j = 0; j < RB; ++j) ar[j] = ai[j] = T(0);
  if (i < n) {  // entries taken kRowBatch at a time (see row_gather)
    if constexpr (INTERP)
      row_gather<T, LPR, RB>(prow[i], prow[i + 1], sub, pcol, pval, phi + rhs0 * Ng, Ng, nr, ar,
                             ai);
    if constexpr (NEARC)
      row_gather<T, LPR, RB>(rowptr[i], rowptr[i + 1], sub, col, val, x + rhs0 * n, n, nr, ar,
                             ai);
  }
#pragma unroll
  for (int j = 0; j < RB; ++j) {
    const T sr = group_sum<LPR>(ar[j]), si = group_sum<LPR>(ai[j]);
    if (sub == 0 && i < n && j < nr) y[(rhs0 + j) * n + i] = mkc<T>(sr, si);
  }
}

// y += Cc x for a complex CSR matrix: LPR lanes per row, fixed summation
// order, one vector per blockIdx.y
template <typename T, int LPR>
__global__ __launch_bounds__(256) void near_complex_kernel(const int32_t* __restrict__ rowptr,
                                                           const int32_t* __restrict__ col,
                                                           const cx<T>* __restrict__ val,
                                                           const cx<T>* __restrict__ x,
                                                           cx<T>* __restrict__ y, int64_t n) {
  const int sub = threadIdx.x % LPR;
  const int64_t i = (int64_t(blockIdx.x) * blockDim.x + threadIdx.x) / LPR;
  const int64_t off = int64_t(blockIdx.y) * n;
  T ar = T(0), ai = T(0);
  if (i < n) {
    for (int k = rowptr[i] + sub; k < rowptr[i + 1]; k += LPR) {
      const cx<T> c = val[k];
      const cx<T> v = x[off + col[k]];
      ar += c.x * v.x - c.y * v.y;
      ai += c.x * v.y + c.y * v.x;
    }
  }
  ar = group_sum<LPR>(ar);
  ai = group_sum<LPR>(ai);
  if (sub == 0 && i < n) {
    cx<T> o = y[off + i];
    o.x += ar;
    o.y += ai;
    y[off + i] = o;
  }
}

template <typename T>
void launch_near_complex(const int32_t* rowptr, const int32_t* col, const void* val,
                         const void* x, void* y, int64_t n, int nrhs, hipStream_t s) {
  constexpr int LPR = 8;
  const dim3 grid(unsigned((n * LPR + 255) / 256), unsigned(nrhs));
  hipLaunchKernelGGL((near_complex_kernel<T, LPR>), grid, dim3(256), 0, s, rowptr, col,
                     static_cast<const cx<T>*>(val), static_cast<const cx<T>*>(x),
                     static_cast<cx<T>*>(y), n);
  AIM_HIP(hipGetLastError());
}

template void launch_near_complex<double>(const int32_t*, const int32_t*, const void*,
                                          const void*, void*, int64_t, int, hipStream_t);
template void launch_near_complex<float>(const int32_t*, const int32_t*, const void*, const void*,
                                         void*, int64_t, int, hipStream_t);

template <typename T>
void launch_interp_near(const GridShape& g, const CsrDevice& Pt, const CsrDevice& csr,
                        const void* phi, const void* x, void* y, int nrhs, bool do_interp,
                        bool do_near, hipStream_t s) {
  constexpr int LPR = 16;
  const int64_t n = csr.n;
  const int64_t gx = (n * LPR + 255) / 256;
  const int rb = rhs_per_block(gx, nrhs);
  dim3 grid(unsigned(gx), unsigned((nrhs + rb - 1) / rb));
  const cx<T>* ph = static_cast<const cx<T>*>(phi);
  const cx<T>* xi = static_cast<const cx<T>*>(x);
  cx<T>* yo = static_cast<cx<T>*>(y);
  const T* pv = static_cast<const T*>(Pt.val);
  const T* v = static_cast<const T*>(csr.val);
#define AIM_IN_LAUNCH(I, NR, R)                                                                  \
  hipLaunchKernelGGL((interp_near_kernel<T, LPR, I, NR, R>), grid, dim3(256), 0, s, ph, xi, yo,  \
                     Pt.rowptr, Pt.col, pv, csr.rowptr, csr.col, v, n, g.Ng, nrhs)
#define AIM_IN_RB(I, NR)                         \
  switch (rb) {                                  \
    case 1: AIM_IN_LAUNCH(I, NR, 1); break;      \
    case 2: AIM_IN_LAUNCH(I, NR, 2); break;      \
    case 4: AIM_IN_LAUNCH(I, NR, 4); break;      \
    default: AIM_IN_LAUNCH(I, NR, 8); break;     \
  }
  if (do_interp && do_near) AIM_IN_RB(true, true)
  else if (do_interp) AIM_IN_RB(true, false)
  else AIM_IN_RB(false, true)
#undef AIM_IN_RB
#undef AIM_IN_LAUNCH
  AIM_HIP(hipGetLastError());
}

// ---------------------------------------------------------------------------
// interpolation without the assembled P^T: y_i = sum over the triangle's three
// quadrature points q and their (n+1)^3 stencil nodes of
// w_q (Lx Ly Lz)(node) phi(node), with the tensor Lagrange weights recomputed
// from the stored local coordinates (36 bytes per point instead of ~12 bytes
// per merged non-zero), plus the near-field rows of C.  Order 3: 16 lanes per
// triangle, lane = (ix, iy), covering the three points and iz; order 2: 32
// lanes, lane = (q, ix, iy), covering iz.  A lane computes its weights and
// grid offsets once and reuses them for every right-hand side of its block.
// Blocks are dealt to the XCDs in contiguous runs of triangles, so the phi
// bricks a run gathers stay in one L2.
// ---------------------------------------------------------------------------
template <typename T, int ORDER>
__device__ __forceinline__ T lagrange_at(T u, int a) {
  T w = T(1);
#pragma unroll
  for (int b = 0; b <= ORDER; ++b)
    if (b != a) w = w * (u - T(b)) / T(a - b);
  return w;
}

template <typename T, int ORDER, bool NEARC>
__global__ __launch_bounds__(256) void interp_implicit_kernel(
    const cx<T>* __restrict__ phi, const cx<T>* __restrict__ x, cx<T>* __restrict__ y,
    const int32_t* __restrict__ qorigin, const T* __restrict__ qlocal, const T* __restrict__ qw,
    const int32_t* __restrict__ rowptr, const int32_t* __restrict__ col,
    const T* __restrict__ val, int64_t n, int Nx, int Ny, int64_t Ng, int nrhs, int rb) {
  constexpr int S = ORDER + 1, PER = S * S;
  constexpr bool QLANES = 3 * PER <= 32;  // one lane per (point, ix, iy)
  constexpr int LPR = QLANES ? 32 : 16;
  constexpr int NTERM = QLANES ? S : 3 * S;  // gathers per lane and right-hand side
  static_assert(QLANES || PER == 16, "order 3 uses 16 lanes per triangle");
  const int nb = int(gridDim.x), b = int(blockIdx.x);
  const int lb = (nb % 8 == 0) ? (b % 8) * (nb / 8) + b / 8 : b;
  const int sub = threadIdx.x % LPR;
  const int64_t i = (int64_t(lb) * blockDim.x + threadIdx.x) / LPR;
  T wts[NTERM];
  int64_t off[NTERM];
#pragma unroll
  for (int t = 0; t < NTERM; ++t) {
    wts[t] = T(0);
    off[t] = 0;
  }
  const bool active = i < n && (!QLANES || sub < 3 * PER);
  if (active) {
    const int64_t plane = int64_t(Nx) * Ny;
    auto point = [&](int q, int ix, int iy, int t0) {
      const int64_t p = 3 * i + q;
      const T* u = qlocal + 3 * p;
      const T wq = qw[p];
      const T lxy = lagrange_at<T, ORDER>(u[0], ix) * lagrange_at<T, ORDER>(u[1], iy);
      const int64_t base = int64_t(qorigin[p]) + int64_t(iy) * Nx + ix;
#pragma unroll
      for (int iz = 0; iz < S; ++iz) {
        wts[t0 + iz] = wq * (lxy * lagrange_at<T, ORDER>(u[2], iz));
        off[t0 + iz] = base + iz * plane;
      }
    };
    if constexpr (QLANES) {
      const int q = sub / PER, r = sub % PER;
      point(q, r % S, r / S, 0);
    } else {
#pragma unroll
      for (int q = 0; q < 3; ++q) point(q, sub % S, sub / S, q * S);
    }
  }
  const int rhs_end = min(nrhs, int(blockIdx.y + 1) * rb);
  for (int rhs = int(blockIdx.y) * rb; rhs < rhs_end; ++rhs) {
    T ar = T(0), ai = T(0);
    if (active) {
      const cx<T>* ph = phi + rhs * Ng;
#pragma unroll
      for (int t = 0; t < NTERM; ++t) {
        const cx<T> v = ph[off[t]];
        ar += wts[t] * v.x;
        ai += wts[t] * v.y;
      }
    }
    if constexpr (NEARC) {
      if (i < n) {
        const cx<T>* xr = x + rhs * n;
        for (int k = rowptr[i] + sub; k < rowptr[i + 1]; k += LPR) {
          const T v = val[k];
          const cx<T> xv = xr[col[k]];
          ar += v * xv.x;
          ai += v * xv.y;
        }
      }
    }
    ar = group_sum<LPR>(ar);
    ai = group_sum<LPR>(ai);
    if (sub == 0 && i < n) y[rhs * n + i] = mkc<T>(ar, ai);
  }
}

template <typename T>
void launch_interp_implicit(const GridShape& g, const QpDevice& qp, const CsrDevice& csr,
                            const void* phi, const void* x, void* y, int nrhs, bool do_near,
                            hipStream_t s) {
  const int64_t n = csr.n;
  const int lpr = qp.order == 3 ? 16 : 32;
  const int64_t gx = (n * lpr + 255) / 256;
  const int rb = rhs_per_block(gx, nrhs);
  dim3 grid(unsigned(gx), unsigned((nrhs + rb - 1) / rb));
  const cx<T>* ph = static_cast<const cx<T>*>(phi);
  const cx<T>* xi = static_cast<const cx<T>*>(x);
  cx<T>* yo = static_cast<cx<T>*>(y);
  const T* lc = static_cast<const T*>(qp.local);
  const T* w = static_cast<const T*>(qp.w);
  const T* v = static_cast<const T*>(csr.val);
#define AIM_II_LAUNCH(O, NR)                                                                    \
  hipLaunchKernelGGL((interp_implicit_kernel<T, O, NR>), grid, dim3(256), 0, s, ph, xi, yo,    \
                     qp.origin, lc, w, csr.rowptr, csr.col, v, n, g.N[0], g.N[1], g.Ng, nrhs,  \
                     rb)
  if (qp.order == 3) {
    if (do_near) AIM_II_LAUNCH(3, true);
    else AIM_II_LAUNCH(3, false);
  } else if (qp.order == 2) {
    if (do_near) AIM_II_LAUNCH(2, true);
    else AIM_II_LAUNCH(2, false);
  } else {
    throw Error(AIM_ERR_STATE, "implicit interpolation is built for orders 2 and 3");
  }
#undef AIM_II_LAUNCH
  AIM_HIP(hipGetLastError());
}

template void launch_interp_implicit<double>(const GridShape&, const QpDevice&, const CsrDevice&,
                                             const void*, const void*, void*, int, bool,
                                             hipStream_t);
template void launch_interp_implicit<float>(const GridShape&, const QpDevice&, const CsrDevice&,
                                            const void*, const void*, void*, int, bool,
                                            hipStream_t);

template void launch_interp_near<double>(const GridShape&, const CsrDevice&, const CsrDevice&,
                                         const void*, const void*, void*, int, bool, bool,
                                         hipStream_t);
template void launch_interp_near<float>(const GridShape&, const CsrDevice&, const CsrDevice&,
                                        const void*, const void*, void*, int, bool, bool,
                                        hipStream_t);

// ---------------------------------------------------------------------------
// excitation b_i = sum_p (A_i/3) u_inc(r_ip)
// ---------------------------------------------------------------------------
__global__ void excitation_kernel(int kind, const double* __restrict__ qp_xyz,
                                  const double* __restrict__ qp_w, int64_t n,
                                  const double* __restrict__ params, int np,
                                  const double* __restrict__ kvals,
                                  const int32_t* __restrict__ rhs_freq, double2* __restrict__ b) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  const int rhs = blockIdx.y;
  if (i >= n) return;
  const double* pr = params + int64_t(rhs) * np;
  const double k = kvals[rhs_freq[rhs]];
  double re = 0.0, im = 0.0;
  for (int q = 0; q < 3; ++q) {
    const int64_t p = 3 * i + q;
    const double* r = qp_xyz + 3 * p;
    const double w = qp_w[p];
    if (kind == 0) {
      const double ph = k * (pr[0] * r[0] + pr[1] * r[1] + pr[2] * r[2]);
      double sn, cs;
      sincos(ph, &sn, &cs);
      re += w * cs;
      im -= w * sn;
    } else {
      const double dx = r[0] - pr[0], dy = r[1] - pr[1], dz = r[2] - pr[2];
      re += w * exp(-(dx * dx + dy * dy + dz * dz) / (2.0 * pr[3] * pr[3]));
    }
  }
  double2 v;
  v.x = re;
  v.y = im;
  b[int64_t(rhs) * n + i] = v;
}

void launch_excitation(int kind, const double* qp_xyz, const double* qp_w, int64_t n,
                       const double* params, int n_params, const double* kvals,
                       const int32_t* rhs_freq, int nrhs, void* b, hipStream_t s) {
  dim3 grid(unsigned((n + 255) / 256), unsigned(nrhs));
  hipLaunchKernelGGL(excitation_kernel, grid, dim3(256), 0, s, kind, qp_xyz, qp_w, n, params,
                     n_params, kvals, rhs_freq, static_cast<double2*>(b));
  AIM_HIP(hipGetLastError());
}

// ---------------------------------------------------------------------------
// Krylov helpers (complex128)
// ---------------------------------------------------------------------------
__global__ void cast_c128_c64_kernel(const double2* in, float2* out, int64_t cnt) {
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < cnt;
       i += int64_t(gridDim.x) * blockDim.x) {
    float2 v;
    v.x = float(in[i].x);
    v.y = float(in[i].y);
    out[i] = v;
  }
}
__global__ void cast_c64_c128_kernel(const float2* in, double2* out, int64_t cnt) {
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < cnt;
       i += int64_t(gridDim.x) * blockDim.x) {
    double2 v;
    v.x = in[i].x;
    v.y = in[i].y;
    out[i] = v;
  }
}

static unsigned grid_for(int64_t cnt, int per = 256) {
  int64_t g = (cnt + per - 1) / per;
  if (g > 8192) g = 8192;
  if (g < 1) g = 1;
  return unsigned(g);
}

void launch_cast_c128_to_c64(const void* in, void* out, int64_t cnt, hipStream_t s) {
  hipLaunchKernelGGL(cast_c128_c64_kernel, dim3(grid_for(cnt)), dim3(256), 0, s,
                     static_cast<const double2*>(in), static_cast<float2*>(out), cnt);
  AIM_HIP(hipGetLastError());
}
void launch_cast_c64_to_c128(const void* in, void* out, int64_t cnt, hipStream_t s) {
  hipLaunchKernelGGL(cast_c64_c128_kernel, dim3(grid_for(cnt)), dim3(256), 0, s,
                     static_cast<const float2*>(in), static_cast<double2*>(out), cnt);
  AIM_HIP(hipGetLastError());
}

constexpr int kDotChunk = 4096;  // elements per partial sum

// block reduction of a double2 over 256 threads
__device__ __forceinline__ double2 block_sum2(double2 v, double2* sh) {
  const int tid = threadIdx.x;
  sh[tid] = v;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (tid < o) {
      sh[tid].x += sh[tid + o].x;
      sh[tid].y += sh[tid + o].y;
    }
    __syncthreads();
  }
  return sh[0];
}

// partial[r][i][c] = sum over chunk c of conj(V[r][i]) w[r]
__global__ __launch_bounds__(256) void block_dot_kernel(const double2* __restrict__ V, int64_t si,
                                                        int64_t sr, const double2* __restrict__ w,
                                                        int64_t n, int nv, int nchunk,
                                                        double2* partial,
                                                        const GivensState* __restrict__ gst,
                                                        const int32_t* __restrict__ rows) {
  __shared__ double2 sh[256];
  const int c = blockIdx.x, i = blockIdx.y, r = blockIdx.z;
  const int64_t nr = rows ? int64_t(rows[r]) : n;
  // frozen systems and chunks past the system's rows (uniform over the block)
  if ((gst && gst[r].frozen) || int64_t(c) * kDotChunk >= nr) {
    if (threadIdx.x == 0) partial[(int64_t(r) * nv + i) * nchunk + c] = make_double2(0.0, 0.0);
    return;
  }
  const double2* vi = V + (int64_t(i) * si + int64_t(r) * sr) * n;
  const double2* wr = w + int64_t(r) * n;
  double2 acc;
  acc.x = 0.0;
  acc.y = 0.0;
  const int64_t b = int64_t(c) * kDotChunk, e = min(nr, b + kDotChunk);
  for (int64_t k = b + threadIdx.x; k < e; k += 256) {
    const double2 a = vi[k], x = wr[k];
    acc.x += a.x * x.x + a.y * x.y;
    acc.y += a.x * x.y - a.y * x.x;
  }
  const double2 s = block_sum2(acc, sh);
  if (threadIdx.x == 0) partial[(int64_t(r) * nv + i) * nchunk + c] = s;
}

// w[r] -/+= sum_{i < nv_r} h[r][i] V[r][i] (SUB: a Gram-Schmidt update; !SUB:
// the restart update x += Z y), nv_r = min(nv, gst[r].len) when the cycle
// state is given, else nv: one element per thread (the launch covers
// every element, so all CUs take part), four basis vectors loaded together
// per step; the order of the terms is fixed
template <bool SUB>
__global__ __launch_bounds__(128) void basis_axpy_kernel(const double2* __restrict__ V,
                                                         int64_t si, int64_t sr,
                                                         double2* __restrict__ w, int64_t n,
                                                         int nv, const double2* __restrict__ h,
                                                         int64_t ldh,
                                                         const GivensState* __restrict__ gst,
                                                         const int32_t* __restrict__ rows) {
  const int r = blockIdx.y;
  const int64_t k = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (k >= (rows ? int64_t(rows[r]) : n)) return;
  // each system's own basis length: columns past it may never have been
  // written (systems stopped before or during the cycle)
  if (gst) nv = min(nv, gst[r].len);
  const double2* hr = h + int64_t(r) * ldh;
  const double2* vr = V + int64_t(r) * sr * n + k;
  const int64_t vs = si * n;
  double2 acc = w[int64_t(r) * n + k];
  auto term = [&](double2 c, double2 a) {
    const double re = c.x * a.x - c.y * a.y, im = c.x * a.y + c.y * a.x;
    if (SUB) {
      acc.x -= re;
      acc.y -= im;
    } else {
      acc.x += re;
      acc.y += im;
    }
  };
  int i = 0;
  for (; i + 4 <= nv; i += 4) {
    double2 a[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) a[u] = vr[int64_t(i + u) * vs];
#pragma unroll
    for (int u = 0; u < 4; ++u) term(hr[i + u], a[u]);
  }
  for (; i < nv; ++i) term(hr[i], vr[int64_t(i) * vs]);
  w[int64_t(r) * n + k] = acc;
}

// One Arnoldi step's Gram-Schmidt update straight from the dot partials:
// h[r][i] = sum_c part[(r nv + i) nchunk + c] is summed by every workgroup
// into LDS (chunks in order, so every workgroup has the same value to the
// bit), then w[r] -= sum_i h[r][i] V_i,r as in basis_axpy_kernel; workgroup
// 0 of each system also stores h in h_out for the Givens step.  No separate
// reduction launch.
constexpr int kMaxBasis = 256;
int dot_chunks(int64_t n) { return int((n + kDotChunk - 1) / kDotChunk); }

__global__ __launch_bounds__(128) void gs_update_kernel(const double2* __restrict__ V, int64_t si,
                                                        int64_t sr, double2* __restrict__ w,
                                                        int64_t n, int nv,
                                                        const double2* __restrict__ part,
                                                        int nchunk, double2* __restrict__ h_out,
                                                        const GivensState* __restrict__ gst,
                                                        const int32_t* __restrict__ rows) {
  __shared__ double2 hs[kMaxBasis];
  const int r = blockIdx.y;
  const int64_t nr = rows ? int64_t(rows[r]) : n;
  if (gst && gst[r].frozen) return;  // uniform over the block
  // workgroups past the system's rows (uniform); workgroup 0 always stays,
  // it stores h
  if (blockIdx.x > 0 && int64_t(blockIdx.x) * blockDim.x >= nr) return;
  for (int i = threadIdx.x; i < nv; i += blockDim.x) {
    const double2* pp = part + (int64_t(r) * nv + i) * nchunk;
    double2 sum = make_double2(0.0, 0.0);
    for (int c0 = 0; c0 < nchunk; c0 += 8) {  // loads in flight together, sums in order
      double2 v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) v[u] = c0 + u < nchunk ? pp[c0 + u] : make_double2(0.0, 0.0);
#pragma unroll
      for (int u = 0; u < 8; ++u)
        if (c0 + u < nchunk) {
          sum.x += v[u].x;
          sum.y += v[u].y;
        }
    }
    hs[i] = sum;
    if (blockIdx.x == 0) h_out[int64_t(r) * nv + i] = sum;
  }
  __syncthreads();
  const int64_t k = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (k >= nr) return;
  const double2* vr = V + int64_t(r) * sr * n + k;
  const int64_t vs = si * n;
  double2 acc = w[int64_t(r) * n + k];
  auto term = [&](double2 c, double2 a) {
    acc.x -= c.x * a.x - c.y * a.y;
    acc.y -= c.x * a.y + c.y * a.x;
  };
  int i = 0;
  for (; i + 4 <= nv; i += 4) {
    double2 a[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) a[u] = vr[int64_t(i + u) * vs];
#pragma unroll
    for (int u = 0; u < 4; ++u) term(hs[i + u], a[u]);
  }
  for (; i < nv; ++i) term(hs[i], vr[int64_t(i) * vs]);
  w[int64_t(r) * n + k] = acc;
}

void launch_block_dot_partials(const void* V, int64_t si, int64_t sr, const void* w, int64_t n,
                               int nv, int nrhs, void* partial, hipStream_t s,
                               const GivensState* gst, const int32_t* rows) {
  const int nchunk = dot_chunks(n);
  hipLaunchKernelGGL(block_dot_kernel, dim3(nchunk, nv, nrhs), dim3(256), 0, s,
                     static_cast<const double2*>(V), si, sr, static_cast<const double2*>(w), n, nv,
                     nchunk, static_cast<double2*>(partial), gst, rows);
  AIM_HIP(hipGetLastError());
}

void launch_gs_update(const void* V, int64_t si, int64_t sr, void* w, int64_t n, int nv, int nrhs,
                      const void* partial, void* h_out, hipStream_t s, const GivensState* gst,
                      const int32_t* rows) {
  AIM_REQUIRE(nv <= kMaxBasis, AIM_ERR_INVALID_ARG, "Krylov basis too large");
  hipLaunchKernelGGL(gs_update_kernel, dim3(unsigned((n + 127) / 128), nrhs), dim3(128), 0, s,
                     static_cast<const double2*>(V), si, sr, static_cast<double2*>(w), n, nv,
                     static_cast<const double2*>(partial), dot_chunks(n),
                     static_cast<double2*>(h_out), gst, rows);
  AIM_HIP(hipGetLastError());
}

__global__ __launch_bounds__(256) void norm_partial_kernel(const double2* __restrict__ w,
                                                           int64_t n, int nchunk,
                                                           double2* partial,
                                                           const GivensState* __restrict__ gst,
                                                           const int32_t* __restrict__ rows) {
  __shared__ double2 sh[256];
  const int c = blockIdx.x, r = blockIdx.y;
  const int64_t nr = rows ? int64_t(rows[r]) : n;
  if ((gst && gst[r].frozen) || int64_t(c) * kDotChunk >= nr) {  // uniform over the block
    if (threadIdx.x == 0) partial[int64_t(r) * nchunk + c] = make_double2(0.0, 0.0);
    return;
  }
  const double2* wr = w + int64_t(r) * n;
  double2 acc;
  acc.x = 0.0;
  acc.y = 0.0;
  const int64_t b = int64_t(c) * kDotChunk, e = min(nr, b + kDotChunk);
  for (int64_t k = b + threadIdx.x; k < e; k += 256) acc.x += wr[k].x * wr[k].x + wr[k].y * wr[k].y;
  const double2 s = block_sum2(acc, sh);
  if (threadIdx.x == 0) partial[int64_t(r) * nchunk + c] = s;
}

__global__ void norm_finish_kernel(const double2* partial, int nchunk, int nrhs, double* out) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= nrhs) return;
  double s = 0.0;
  for (int c = 0; c < nchunk; ++c) s += partial[int64_t(r) * nchunk + c].x;
  out[r] = sqrt(s);
}

void launch_norms(const void* w, int64_t n, int nrhs, void* partial, double* out, hipStream_t s,
                  const GivensState* gst) {
  const int nchunk = int((n + kDotChunk - 1) / kDotChunk);
  hipLaunchKernelGGL(norm_partial_kernel, dim3(nchunk, nrhs), dim3(256), 0, s,
                     static_cast<const double2*>(w), n, nchunk, static_cast<double2*>(partial), gst,
                     nullptr);
  AIM_HIP(hipGetLastError());
  hipLaunchKernelGGL(norm_finish_kernel, dim3((nrhs + 127) / 128), dim3(128), 0, s,
                     static_cast<const double2*>(partial), nchunk, nrhs, out);
  AIM_HIP(hipGetLastError());
}

__global__ void scale_inv_kernel(const double2* w, const double* nrm, double2* out, int64_t n,
                                 int64_t out_stride, const GivensState* __restrict__ gst,
                                 const int32_t* __restrict__ rows) {
  const int r = blockIdx.y;
  if (gst && gst[r].frozen) return;
  const int64_t nr = rows ? int64_t(rows[r]) : n;
  const double nv = nrm[r];
  const double sc = nv > 0.0 ? 1.0 / nv : 0.0;
  for (int64_t k = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; k < nr;
       k += int64_t(gridDim.x) * blockDim.x) {
    double2 v = w[int64_t(r) * n + k];
    v.x *= sc;
    v.y *= sc;
    out[int64_t(r) * out_stride + k] = v;
  }
}

// out[r] = w[r] / ||w[r]|| with the norm summed from norm_partial_kernel's
// partials by every workgroup (chunks in order, as norm_finish_kernel sums
// them: the same value to the bit); workgroup 0 of each system stores it in
// nrm_out for the Givens step.  No separate finishing launch.
__global__ void scale_norm_kernel(const double2* w, const double2* __restrict__ part, int nchunk,
                                  double* __restrict__ nrm_out, double2* out, int64_t n,
                                  int64_t out_stride, const GivensState* __restrict__ gst,
                                  const int32_t* __restrict__ rows) {
  __shared__ double nrm_s;
  const int r = blockIdx.y;
  if (gst && gst[r].frozen) return;  // uniform over the block
  const int64_t nr = rows ? int64_t(rows[r]) : n;
  if (threadIdx.x == 0) {
    const double2* pp = part + int64_t(r) * nchunk;
    double sum = 0.0;
    for (int c0 = 0; c0 < nchunk; c0 += 8) {
      double v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) v[u] = c0 + u < nchunk ? pp[c0 + u].x : 0.0;
#pragma unroll
      for (int u = 0; u < 8; ++u)
        if (c0 + u < nchunk) sum += v[u];
    }
    nrm_s = sqrt(sum);
    if (blockIdx.x == 0) nrm_out[r] = nrm_s;
  }
  __syncthreads();
  const double nv = nrm_s;
  const double sc = nv > 0.0 ? 1.0 / nv : 0.0;
  for (int64_t k = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; k < nr;
       k += int64_t(gridDim.x) * blockDim.x) {
    double2 v = w[int64_t(r) * n + k];
    v.x *= sc;
    v.y *= sc;
    out[int64_t(r) * out_stride + k] = v;
  }
}

void launch_norm_partials(const void* w, int64_t n, int nrhs, void* partial, hipStream_t s,
                          const GivensState* gst, const int32_t* rows) {
  hipLaunchKernelGGL(norm_partial_kernel, dim3(dot_chunks(n), nrhs), dim3(256), 0, s,
                     static_cast<const double2*>(w), n, dot_chunks(n),
                     static_cast<double2*>(partial), gst, rows);
  AIM_HIP(hipGetLastError());
}

void launch_scale_norm(const void* w, const void* partial, double* nrm_out, void* out, int64_t n,
                       int nrhs, int64_t out_stride, hipStream_t s, const GivensState* gst,
                       const int32_t* rows) {
  hipLaunchKernelGGL(scale_norm_kernel, dim3(grid_for(n, 1024), nrhs), dim3(256), 0, s,
                     static_cast<const double2*>(w), static_cast<const double2*>(partial),
                     dot_chunks(n), nrm_out, static_cast<double2*>(out), n, out_stride, gst, rows);
  AIM_HIP(hipGetLastError());
}

void launch_scale_inv(const void* w, const double* nrm, void* out, int64_t n, int nrhs,
                      int64_t out_stride, hipStream_t s, const GivensState* gst,
                      const int32_t* rows) {
  hipLaunchKernelGGL(scale_inv_kernel, dim3(grid_for(n, 1024), nrhs), dim3(256), 0, s,
                     static_cast<const double2*>(w), nrm, static_cast<double2*>(out), n,
                     out_stride, gst, rows);
  AIM_HIP(hipGetLastError());
}

// One Arnoldi step of restarted GMRES, on the device, thread r = system r
// (the host loop it replaces read h, h2 and the norms back every step).
// Column j of the Hessenberg matrix is the two Gram-Schmidt passes'
// coefficients summed, with the new basis norm below the diagonal; the
// earlier Givens rotations are applied to it, a new rotation zeroes its
// subdiagonal entry, and the rotated right-hand side g gives the residual
// estimate |g_{j+1}| / scale_r.  A system that is frozen does nothing; it
// freezes when the estimate meets tol, max_iter is reached, the norm is zero
// (lucky breakdown), the rotation denominator is zero, or the norm is not
// finite (flagged).  H is stored column by column, ldH = (mcap + 1) per
// column, mcap columns per system.
__device__ __forceinline__ double2 zmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 zconj(double2 a) { return make_double2(a.x, -a.y); }
__device__ __forceinline__ double2 zadd(double2 a, double2 b) {
  return make_double2(a.x + b.x, a.y + b.y);
}

constexpr int kGivensMax = 256;  // restart lengths up to this (aim_solve allows 200)

__global__ __launch_bounds__(64) void givens_step_kernel(
    const double2* __restrict__ h, const double2* __restrict__ h2, const double* __restrict__ nrm,
    int nrhs, int j, int mcap, double2* __restrict__ H, double2* __restrict__ cs,
    double2* __restrict__ sn, double2* __restrict__ g, GivensState* __restrict__ st,
    const double* __restrict__ scale, double tol, int max_iter) {
  // the column and the earlier rotations are staged in LDS by all lanes; one
  // lane runs the (sequential) rotation chain there; all lanes write back
  __shared__ double2 col[kGivensMax + 1], c[kGivensMax], sv[kGivensMax];
  __shared__ int done;
  const int r = blockIdx.x, t = threadIdx.x;
  GivensState& q = st[r];
  if (q.frozen) return;  // uniform over the block
  double2* colg = H + (int64_t(r) * mcap + j) * (mcap + 1);
  double2* cg = cs + int64_t(r) * mcap;
  double2* sg = sn + int64_t(r) * mcap;
  double2* gr = g + int64_t(r) * (mcap + 1);
  const double hn = nrm[r];
  for (int i = t; i <= j; i += 64) col[i] = zadd(h[r * (j + 1) + i], h2[r * (j + 1) + i]);
  for (int i = t; i < j; i += 64) {
    c[i] = cg[i];
    sv[i] = sg[i];
  }
  __syncthreads();
  if (t == 0) {
    done = 0;
    if (!isfinite(hn)) {
      q.nonfinite = 1;
      q.frozen = 1;
      done = 1;
    } else {
      col[j + 1] = make_double2(hn, 0.0);
      for (int i = 0; i < j; ++i) {
        const double2 ci = col[i], cn = col[i + 1];
        const double2 tt = zadd(zmul(c[i], ci), zmul(sv[i], cn));
        const double2 ns = zmul(zconj(sv[i]), ci);
        col[i + 1] = zadd(make_double2(-ns.x, -ns.y), zmul(zconj(c[i]), cn));
        col[i] = tt;
      }
      const double2 a = col[j], bb = col[j + 1];
      const double den = sqrt((a.x * a.x + a.y * a.y) + (bb.x * bb.x + bb.y * bb.y));
      if (den == 0.0) {
        q.frozen = 1;
        done = 1;
      } else {
        const double aa = hypot(a.x, a.y);
        double2 cj, sj;
        if (aa == 0.0) {
          cj = make_double2(0.0, 0.0);
          sj = make_double2(1.0, 0.0);
        } else {
          cj = make_double2(aa / den, 0.0);
          const double2 ph = make_double2(a.x / aa, a.y / aa);
          const double2 tt = zmul(ph, zconj(bb));
          sj = make_double2(tt.x / den, tt.y / den);
        }
        c[j] = cj;
        sv[j] = sj;
        col[j] = zadd(zmul(cj, a), zmul(sj, bb));
        col[j + 1] = make_double2(0.0, 0.0);
        const double2 gj = gr[j];
        const double2 ng = zmul(zconj(sj), gj);
        const double2 g1 = make_double2(-ng.x, -ng.y);
        gr[j + 1] = g1;
        gr[j] = zmul(cj, gj);
        q.len = j + 1;
        q.iters += 1;
        const double est = hypot(g1.x, g1.y) / scale[r];
        if (est <= tol || hn == 0.0 || q.iters >= max_iter) q.frozen = 1;
      }
    }
  }
  __syncthreads();
  if (done) return;
  for (int i = t; i <= j + 1; i += 64) colg[i] = col[i];
  if (t == 0) {
    cg[j] = c[j];
    sg[j] = sv[j];
  }
}

void launch_givens_step(const void* h, const void* h2, const double* nrm, int nrhs, int j,
                        int mcap, void* H, void* cs, void* sn, void* g, GivensState* st,
                        const double* scale, double tol, int max_iter, hipStream_t s) {
  if (mcap > kGivensMax) throw Error(AIM_ERR_INVALID_ARG, "restart length too large");
  hipLaunchKernelGGL(givens_step_kernel, dim3(unsigned(nrhs)), dim3(64), 0, s,
                     static_cast<const double2*>(h), static_cast<const double2*>(h2), nrm, nrhs, j,
                     mcap, static_cast<double2*>(H), static_cast<double2*>(cs),
                     static_cast<double2*>(sn), static_cast<double2*>(g), st, scale, tol,
                     max_iter);
  AIM_HIP(hipGetLastError());
}

void launch_combine(const void* Z, int64_t si, int64_t sr, const void* y, int64_t ldy, int nv,
                    void* x, int64_t n, int nrhs, const GivensState* gst, hipStream_t s,
                    const int32_t* rows) {
  hipLaunchKernelGGL(basis_axpy_kernel<false>, dim3(unsigned((n + 127) / 128), nrhs), dim3(128),
                     0, s, static_cast<const double2*>(Z), si, sr, static_cast<double2*>(x), n, nv,
                     static_cast<const double2*>(y), ldy, gst, rows);
  AIM_HIP(hipGetLastError());
}

__global__ void residual_kernel(const double2* b, double2* r, int64_t cnt) {
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < cnt;
       i += int64_t(gridDim.x) * blockDim.x) {
    double2 v;
    v.x = b[i].x - r[i].x;
    v.y = b[i].y - r[i].y;
    r[i] = v;
  }
}
void launch_residual(const void* b, void* r, int64_t cnt, hipStream_t s) {
  hipLaunchKernelGGL(residual_kernel, dim3(grid_for(cnt)), dim3(256), 0, s,
                     static_cast<const double2*>(b), static_cast<double2*>(r), cnt);
  AIM_HIP(hipGetLastError());
}

__global__ void axpy_kernel(double2* x, const double2* d, int64_t cnt) {
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < cnt;
       i += int64_t(gridDim.x) * blockDim.x) {
    x[i].x += d[i].x;
    x[i].y += d[i].y;
  }
}
void launch_axpy_inplace(void* x, const void* d, int64_t cnt, hipStream_t s) {
  hipLaunchKernelGGL(axpy_kernel, dim3(grid_for(cnt)), dim3(256), 0, s, static_cast<double2*>(x),
                     static_cast<const double2*>(d), cnt);
  AIM_HIP(hipGetLastError());
}

__global__ void diag_pc_kernel(const double2* v, const double* dinv, double2* z, int64_t n) {
  const int r = blockIdx.y;
  for (int64_t k = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; k < n;
       k += int64_t(gridDim.x) * blockDim.x) {
    double2 a = v[int64_t(r) * n + k];
    a.x *= dinv[k];
    a.y *= dinv[k];
    z[int64_t(r) * n + k] = a;
  }
}
void launch_diag_pc(const void* v, const double* dinv, void* z, int64_t n, int nrhs,
                    hipStream_t s) {
  hipLaunchKernelGGL(diag_pc_kernel, dim3(grid_for(n, 1024), nrhs), dim3(256), 0, s,
                     static_cast<const double2*>(v), dinv, static_cast<double2*>(z), n);
  AIM_HIP(hipGetLastError());
}

// z[perm[o + a]] = sum_b Binv[a][b] v[perm[o + b]] per cluster (block of 64)
__global__ __launch_bounds__(64) void block_pc_kernel(const double2* __restrict__ v,
                                                      double2* __restrict__ z,
                                                      const int32_t* __restrict__ cl_ptr,
                                                      const int32_t* __restrict__ perm,
                                                      const int64_t* __restrict__ cl_blk,
                                                      const double* __restrict__ inv, int64_t n) {
  __shared__ double2 sv[64];
  const int c = blockIdx.x, r = blockIdx.y, a = threadIdx.x;
  const int o = cl_ptr[c], m = cl_ptr[c + 1] - o;
  const double2* vr = v + int64_t(r) * n;
  if (a < m) sv[a] = vr[perm[o + a]];
  __syncthreads();
  if (a < m) {
    const double* row = inv + cl_blk[c] + int64_t(a) * m;
    double2 acc;
    acc.x = 0.0;
    acc.y = 0.0;
    for (int b = 0; b < m; ++b) {
      acc.x += row[b] * sv[b].x;
      acc.y += row[b] * sv[b].y;
    }
    z[int64_t(r) * n + perm[o + a]] = acc;
  }
}

// complex block inverses: vector r uses the set of wavenumber rhs_freq[r],
// stored freq_stride complex values after the previous one
__global__ __launch_bounds__(64) void block_pc_complex_kernel(
    const double2* __restrict__ v, double2* __restrict__ z, const int32_t* __restrict__ cl_ptr,
    const int32_t* __restrict__ perm, const int64_t* __restrict__ cl_blk,
    const double2* __restrict__ inv, int64_t freq_stride, const int32_t* __restrict__ rhs_freq,
    int64_t n) {
  __shared__ double2 sv[64];
  const int c = blockIdx.x, r = blockIdx.y, a = threadIdx.x;
  const int o = cl_ptr[c], m = cl_ptr[c + 1] - o;
  const double2* vr = v + int64_t(r) * n;
  if (a < m) sv[a] = vr[perm[o + a]];
  __syncthreads();
  if (a < m) {
    const double2* row = inv + int64_t(rhs_freq[r]) * freq_stride + cl_blk[c] + int64_t(a) * m;
    double ar = 0.0, ai = 0.0;
    for (int b = 0; b < m; ++b) {
      const double2 w = row[b], x = sv[b];
      ar += w.x * x.x - w.y * x.y;
      ai += w.x * x.y + w.y * x.x;
    }
    z[int64_t(r) * n + perm[o + a]] = make_double2(ar, ai);
  }
}

void launch_block_pc_complex(const void* v, void* z, const int32_t* cl_ptr,
                             const int32_t* cl_perm, const int64_t* cl_blk, const void* cl_inv,
                             int64_t freq_stride, const int32_t* rhs_freq, int ncl, int max_cl,
                             int64_t n, int nrhs, hipStream_t s) {
  AIM_REQUIRE(max_cl <= 64, AIM_ERR_STATE, "cluster larger than 64");
  hipLaunchKernelGGL(block_pc_complex_kernel, dim3(ncl, nrhs), dim3(64), 0, s,
                     static_cast<const double2*>(v), static_cast<double2*>(z), cl_ptr, cl_perm,
                     cl_blk, static_cast<const double2*>(cl_inv), freq_stride, rhs_freq, n);
  AIM_HIP(hipGetLastError());
}

void launch_block_pc(const void* v, void* z, const int32_t* cl_ptr, const int32_t* cl_perm,
                     const int64_t* cl_blk, const double* cl_inv, int ncl, int max_cl, int64_t n,
                     int nrhs, hipStream_t s) {
  AIM_REQUIRE(max_cl <= 64, AIM_ERR_STATE, "cluster larger than 64");
  hipLaunchKernelGGL(block_pc_kernel, dim3(ncl, nrhs), dim3(64), 0, s,
                     static_cast<const double2*>(v), static_cast<double2*>(z), cl_ptr, cl_perm,
                     cl_blk, cl_inv, n);
  AIM_HIP(hipGetLastError());
}

__global__ void gather_rows_kernel(const double2* src, double2* dst, const int32_t* idx, int64_t n,
                                   int scatter) {
  const int r = blockIdx.y;
  const int64_t sr = scatter ? r : idx[r];
  const int64_t dr = scatter ? idx[r] : r;
  for (int64_t k = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; k < n;
       k += int64_t(gridDim.x) * blockDim.x)
    dst[dr * n + k] = src[sr * n + k];
}

void launch_gather_rows(const void* src, void* dst, const int32_t* idx, int64_t n, int nrhs,
                        bool scatter, hipStream_t s) {
  hipLaunchKernelGGL(gather_rows_kernel, dim3(grid_for(n, 1024), nrhs), dim3(256), 0, s,
                     static_cast<const double2*>(src), static_cast<double2*>(dst), idx, n,
                     scatter ? 1 : 0);
  AIM_HIP(hipGetLastError());
}

}  // namespace aim

// ===========================================================================
// learned-preconditioner glue (complex64 grids and meshes)
// ===========================================================================
namespace aim {

__global__ void scale_cast_c64_kernel(const double2* v, const double* s, float2* out, int64_t n) {
  const int r = blockIdx.y;
  const double sc = s ? s[r] : 1.0;
  for (int64_t k = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; k < n;
       k += int64_t(gridDim.x) * blockDim.x) {
    const double2 a = v[int64_t(r) * n + k];
    float2 o;
    o.x = float(a.x * sc);
    o.y = float(a.y * sc);
    out[int64_t(r) * n + k] = o;
  }
}

// out[r] = 1 / ||v[r]|| (0 if the norm is 0), from partial sums of squares
__global__ void inv_norm_finish_kernel(const double2* partial, int nchunk, int nrhs, double mul,
                                       double* out) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= nrhs) return;
  double s = 0.0;
  for (int c = 0; c < nchunk; ++c) s += partial[int64_t(r) * nchunk + c].x;
  out[r] = s > 0.0 ? mul / sqrt(s) : 0.0;
}

__global__ __launch_bounds__(256) void sumsq_c64_kernel(const float2* __restrict__ w, int64_t n,
                                                        int nchunk, double2* partial) {
  __shared__ double2 sh[256];
  const int c = blockIdx.x, r = blockIdx.y;
  const float2* wr = w + int64_t(r) * n;
  double acc = 0.0;
  const int64_t b = int64_t(c) * 4096, e = min(n, b + 4096);
  for (int64_t k = b + threadIdx.x; k < e; k += 256)
    acc += double(wr[k].x) * wr[k].x + double(wr[k].y) * wr[k].y;
  sh[threadIdx.x].x = acc;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) sh[threadIdx.x].x += sh[threadIdx.x + o].x;
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[int64_t(r) * nchunk + c] = make_double2(sh[0].x, 0.0);
}

// s[r] = mul / ||x[r]|| for complex64 vectors
void launch_inv_norms_c64(const void* x, int64_t n, int nrhs, double mul, void* partial, double* s,
                          hipStream_t st) {
  const int nchunk = int((n + 4095) / 4096);
  hipLaunchKernelGGL(sumsq_c64_kernel, dim3(nchunk, nrhs), dim3(256), 0, st,
                     static_cast<const float2*>(x), n, nchunk, static_cast<double2*>(partial));
  AIM_HIP(hipGetLastError());
  hipLaunchKernelGGL(inv_norm_finish_kernel, dim3((nrhs + 127) / 128), dim3(128), 0, st,
                     static_cast<const double2*>(partial), nchunk, nrhs, mul, s);
  AIM_HIP(hipGetLastError());
}

__global__ __launch_bounds__(256) void sumsq_c128_kernel(const double2* __restrict__ w, int64_t n,
                                                         int nchunk, double2* partial) {
  __shared__ double sh[256];
  const int c = blockIdx.x, r = blockIdx.y;
  const double2* wr = w + int64_t(r) * n;
  double acc = 0.0;
  const int64_t b = int64_t(c) * 4096, e = min(n, b + 4096);
  for (int64_t k = b + threadIdx.x; k < e; k += 256) acc += wr[k].x * wr[k].x + wr[k].y * wr[k].y;
  sh[threadIdx.x] = acc;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[int64_t(r) * nchunk + c] = make_double2(sh[0], 0.0);
}

// s[r] = mul / ||v[r]|| for complex128 vectors
void launch_inv_norms_c128(const void* v, int64_t n, int nrhs, double mul, void* partial,
                           double* s, hipStream_t st) {
  const int nchunk = int((n + 4095) / 4096);
  hipLaunchKernelGGL(sumsq_c128_kernel, dim3(nchunk, nrhs), dim3(256), 0, st,
                     static_cast<const double2*>(v), n, nchunk, static_cast<double2*>(partial));
  AIM_HIP(hipGetLastError());
  hipLaunchKernelGGL(inv_norm_finish_kernel, dim3((nrhs + 127) / 128), dim3(128), 0, st,
                     static_cast<const double2*>(partial), nchunk, nrhs, mul, s);
  AIM_HIP(hipGetLastError());
}

void launch_scale_cast_c64(const void* v, const double* s, void* out, int64_t n, int nrhs,
                           hipStream_t st) {
  hipLaunchKernelGGL(scale_cast_c64_kernel, dim3(grid_for(n, 1024), nrhs), dim3(256), 0, st,
                     static_cast<const double2*>(v), s, static_cast<float2*>(out), n);
  AIM_HIP(hipGetLastError());
}

__global__ void scale_c64_kernel(float2* x, const double* s, int64_t n) {
  const int r = blockIdx.y;
  const float sc = float(s[r]);
  for (int64_t k = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; k < n;
       k += int64_t(gridDim.x) * blockDim.x) {
    float2 a = x[int64_t(r) * n + k];
    a.x *= sc;
    a.y *= sc;
    x[int64_t(r) * n + k] = a;
  }
}

void launch_scale_c64(void* x, const double* s, int64_t n, int nrhs, hipStream_t st) {
  hipLaunchKernelGGL(scale_c64_kernel, dim3(grid_for(n, 1024), nrhs), dim3(256), 0, st,
                     static_cast<float2*>(x), s, n);
  AIM_HIP(hipGetLastError());
}

// z[r][i] += tau * c[r][i] / (area[i] * sv[r]) with sv = 1/||v||; z holds the
// base preconditioner applied to v on entry
__global__ void unet_combine_kernel(const float2* c, const double* area, double tau,
                                    const double* sv, double2* z, int64_t n) {
  const int r = blockIdx.y;
  const double sc = sv[r] > 0.0 ? tau / sv[r] : 0.0;
  for (int64_t k = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; k < n;
       k += int64_t(gridDim.x) * blockDim.x) {
    const float2 b = c[int64_t(r) * n + k];
    const double f = sc / area[k];
    double2 o = z[int64_t(r) * n + k];
    o.x += f * b.x;
    o.y += f * b.y;
    z[int64_t(r) * n + k] = o;
  }
}

void launch_unet_combine(const void* c, const double* area, double tau, const double* sv, void* z,
                         int64_t n, int nrhs, hipStream_t st) {
  hipLaunchKernelGGL(unet_combine_kernel, dim3(grid_for(n, 1024), nrhs), dim3(256), 0, st,
                     static_cast<const float2*>(c), area, tau, sv, static_cast<double2*>(z), n);
  AIM_HIP(hipGetLastError());
}

// w[r][i] = (e[r][i] - w[r][i]) * ir[r]: on entry w holds the base
// preconditioner applied to the residual, so the result is the part of the
// normalised error the base preconditioner misses (complex128)
__global__ void unet_resid_target_kernel(const double2* e, const double* ir, double2* w,
                                         int64_t n) {
  const int r = blockIdx.y;
  const double s = ir[r];
  for (int64_t k = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; k < n;
       k += int64_t(gridDim.x) * blockDim.x) {
    const double2 b = e[int64_t(r) * n + k];
    double2 o = w[int64_t(r) * n + k];
    o.x = (b.x - o.x) * s;
    o.y = (b.y - o.y) * s;
    w[int64_t(r) * n + k] = o;
  }
}

void launch_unet_resid_target(const void* e, const double* ir, void* w, int64_t n, int nrhs,
                              hipStream_t st) {
  hipLaunchKernelGGL(unet_resid_target_kernel, dim3(grid_for(n, 1024), nrhs), dim3(256), 0, st,
                     static_cast<const double2*>(e), ir, static_cast<double2*>(w), n);
  AIM_HIP(hipGetLastError());
}

// mesh loss: mean over n (x nb) of |c/area - t|^2 with t = w / tau; gradient
// d = 2 (c/area - t) / (area cnt) in complex64; per-block partial losses
__global__ __launch_bounds__(256) void mesh_mse_kernel(const float2* c, const double2* w,
                                                       const double* area, double inv_tau,
                                                       int64_t n, double inv_cnt, float2* d,
                                                       double* part) {
  __shared__ double sh[256];
  double acc = 0.0;
  for (int64_t k = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; k < n;
       k += int64_t(gridDim.x) * blockDim.x) {
    const double ia = 1.0 / area[k];
    const double dx = c[k].x * ia - w[k].x * inv_tau, dy = c[k].y * ia - w[k].y * inv_tau;
    acc += (dx * dx + dy * dy) * inv_cnt;
    float2 o;
    o.x = float(2.0 * dx * ia * inv_cnt);
    o.y = float(2.0 * dy * ia * inv_cnt);
    d[k] = o;
  }
  sh[threadIdx.x] = acc;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

void launch_mesh_mse(const void* c, const void* w, const double* area, double inv_tau, int64_t n,
                     double inv_cnt, void* d, double* part, int nparts, hipStream_t st) {
  hipLaunchKernelGGL(mesh_mse_kernel, dim3(nparts), dim3(256), 0, st,
                     static_cast<const float2*>(c), static_cast<const double2*>(w), area, inv_tau,
                     n, inv_cnt, static_cast<float2*>(d), part);
  AIM_HIP(hipGetLastError());
}

// out = tau c / area (complex64), one vector
__global__ void area_scale_c64_kernel(const float2* c, const double* area, double tau, float2* out,
                                      int64_t n) {
  for (int64_t k = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; k < n;
       k += int64_t(gridDim.x) * blockDim.x) {
    const double f = tau / area[k];
    out[k] = make_float2(float(f * c[k].x), float(f * c[k].y));
  }
}

void launch_area_scale_c64(const void* c, const double* area, double tau, void* out, int64_t n,
                           hipStream_t st) {
  hipLaunchKernelGGL(area_scale_c64_kernel, dim3(grid_for(n, 1024)), dim3(256), 0, st,
                     static_cast<const float2*>(c), area, tau, static_cast<float2*>(out), n);
  AIM_HIP(hipGetLastError());
}

// residual loss of one sample: rho = s - Az; partial sums of wgt |rho|^2 per
// block; out = conj(rho) (complex64), the input of the adjoint product
__global__ __launch_bounds__(256) void resid_loss_kernel(const float2* az, const double2* sv,
                                                         double wgt, int64_t n, float2* out,
                                                         double* part) {
  __shared__ double sh[256];
  double acc = 0.0;
  for (int64_t k = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; k < n;
       k += int64_t(gridDim.x) * blockDim.x) {
    const double rx = sv[k].x - az[k].x, ry = sv[k].y - az[k].y;
    acc += (rx * rx + ry * ry) * wgt;
    out[k] = make_float2(float(rx), float(-ry));
  }
  sh[threadIdx.x] = acc;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

void launch_resid_loss(const void* az, const void* sv, double wgt, int64_t n, void* out,
                       double* part, int nparts, hipStream_t st) {
  hipLaunchKernelGGL(resid_loss_kernel, dim3(nparts), dim3(256), 0, st,
                     static_cast<const float2*>(az), static_cast<const double2*>(sv), wgt, n,
                     static_cast<float2*>(out), part);
  AIM_HIP(hipGetLastError());
}

// d = coef conj(y) / area (complex64): with y = A conj(rho) this is
// coef A^H rho / area, A being complex symmetric
__global__ void resid_grad_kernel(const float2* y, const double* area, double coef, float2* d,
                                  int64_t n) {
  for (int64_t k = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; k < n;
       k += int64_t(gridDim.x) * blockDim.x) {
    const double f = coef / area[k];
    d[k] = make_float2(float(f * y[k].x), float(-f * y[k].y));
  }
}

void launch_resid_grad(const void* y, const double* area, double coef, void* d, int64_t n,
                       hipStream_t st) {
  hipLaunchKernelGGL(resid_grad_kernel, dim3(grid_for(n, 1024)), dim3(256), 0, st,
                     static_cast<const float2*>(y), area, coef, static_cast<float2*>(d), n);
  AIM_HIP(hipGetLastError());
}

// y[r][i] += k_{f_r}^2 D_i x[r][i]
template <typename T>
__global__ void lin_term_kernel(const double* __restrict__ D, const double* __restrict__ k,
                                const int32_t* __restrict__ rhs_freq, const cx<T>* __restrict__ x,
                                cx<T>* __restrict__ y, int64_t n) {
  const int r = blockIdx.y;
  const double kr = k[rhs_freq[r]];
  const T k2 = T(kr * kr);
  const int64_t off = int64_t(r) * n;
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
       i += int64_t(gridDim.x) * blockDim.x) {
    const T d = k2 * T(D[i]);
    const cx<T> xv = x[off + i];
    cx<T> yv = y[off + i];
    yv.x += d * xv.x;
    yv.y += d * xv.y;
    y[off + i] = yv;
  }
}

template <typename T>
void launch_lin_term(const double* D, const double* k, const int32_t* rhs_freq, const void* x,
                     void* y, int64_t n, int nrhs, hipStream_t s) {
  hipLaunchKernelGGL(lin_term_kernel<T>, dim3(grid_for(n, 1024), unsigned(nrhs)), dim3(256), 0, s,
                     D, k, rhs_freq, static_cast<const cx<T>*>(x), static_cast<cx<T>*>(y), n);
  AIM_HIP(hipGetLastError());
}
template void launch_lin_term<double>(const double*, const double*, const int32_t*, const void*,
                                      void*, int64_t, int, hipStream_t);
template void launch_lin_term<float>(const double*, const double*, const int32_t*, const void*,
                                     void*, int64_t, int, hipStream_t);

// zero n 8-byte words (a kernel, so that captured graphs hold no memset node)
__global__ void zero_words_kernel(uint2* p, int64_t n) {
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
       i += int64_t(gridDim.x) * blockDim.x)
    p[i] = make_uint2(0u, 0u);
}

void launch_zero_words(void* p, int64_t n, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(zero_words_kernel, dim3(grid_for(n, 1024)), dim3(256), 0, st,
                     static_cast<uint2*>(p), n);
  AIM_HIP(hipGetLastError());
}

// ---------------------------------------------------------------------------
// double-layer operator (Sec. III-B, eq. KAIMx): the far product
// W sum_a H_grad,a P diag(n_a) x with the odd channel kernels
// H_grad,a(u, v) = (u_a - v_a) F(|u - v|), F radial: the channel sources
// n_a x here, their projections and forward transforms, then one z pass
// (zcross_kernel, DOT) that sums the three spectral products into one grid,
// transformed back.
// ---------------------------------------------------------------------------
__global__ void dlp_sources_kernel(const double2* __restrict__ x, const double* __restrict__ nrm,
                                   double2* __restrict__ xs, int64_t n, int nrhs) {
  const int r = blockIdx.y;
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
       i += int64_t(gridDim.x) * blockDim.x) {
    const double2 v = x[int64_t(r) * n + i];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const double w = nrm[3 * i + a];
      xs[(int64_t(a) * nrhs + r) * n + i] = make_double2(w * v.x, w * v.y);
    }
  }
}

void launch_dlp_sources(const void* x, const double* nrm, void* xs, int64_t n, int nrhs,
                        hipStream_t s) {
  hipLaunchKernelGGL(dlp_sources_kernel, dim3(grid_for(n, 1024), nrhs), dim3(256), 0, s,
                     static_cast<const double2*>(x), nrm, static_cast<double2*>(xs), n, nrhs);
  AIM_HIP(hipGetLastError());
}

// ---------------------------------------------------------------------------
// Fixed device scratch for the matvec variant that allocates nothing: the
// projection grid and the convolution workspace of one call.  The array is
// part of the code object, so each device that loads the library holds its
// own copy until the process ends; host code reaches it only through the
// address hipGetSymbolAddress returns for the current device (the array's
// name in host code is a host-side stand-in, not a device address).
// ---------------------------------------------------------------------------
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

void* static_scratch() {
  constexpr int kMaxDevices = 64;
  static std::mutex mu;
  static void* addr[kMaxDevices] = {};
  int dev = 0;
  AIM_HIP(hipGetDevice(&dev));
  AIM_REQUIRE(dev >= 0 && dev < kMaxDevices, AIM_ERR_DEVICE, "device index out of range");
  std::lock_guard<std::mutex> lock(mu);
  if (!addr[dev]) {
    void* ptr = nullptr;
    AIM_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    AIM_REQUIRE(ptr != nullptr, AIM_ERR_DEVICE, "no device address for the static scratch");
    addr[dev] = ptr;
  }
  return addr[dev];
}

// n complex values of modulus <= 1 from a hash of the index (timing input:
// the clock under load depends on the data, and zeros flatter the kernels)
template <typename T>
__global__ void pattern_kernel(cx<T>* p, int64_t n) {
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
       i += int64_t(gridDim.x) * blockDim.x) {
    uint64_t h = uint64_t(i) * 0x9E3779B97F4A7C15ull;
    h ^= h >> 29;
    h *= 0xBF58476D1CE4E5B9ull;
    h ^= h >> 32;
    const T re = T(int32_t(uint32_t(h))) * T(3.3e-10);
    const T im = T(int32_t(uint32_t(h >> 32))) * T(3.3e-10);
    p[i] = mkc<T>(re, im);
  }
}

void launch_pattern(void* p, int64_t n, bool dbl, hipStream_t st) {
  if (n <= 0) return;
  if (dbl)
    hipLaunchKernelGGL(pattern_kernel<double>, dim3(grid_for(n, 1024)), dim3(256), 0, st,
                       static_cast<double2*>(p), n);
  else
    hipLaunchKernelGGL(pattern_kernel<float>, dim3(grid_for(n, 1024)), dim3(256), 0, st,
                       static_cast<float2*>(p), n);
  AIM_HIP(hipGetLastError());
}

// e = xs - e for a logged iterate (in place): the error of the iterate
// against the converged solution
__global__ void pair_error_kernel(const double2* xs, double2* e, int64_t n) {
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
       i += int64_t(gridDim.x) * blockDim.x) {
    double2 a = e[i];
    a.x = xs[i].x - a.x;
    a.y = xs[i].y - a.y;
    e[i] = a;
  }
}

void launch_pair_error(const void* xs, void* e, int64_t n, hipStream_t st) {
  hipLaunchKernelGGL(pair_error_kernel, dim3(grid_for(n, 1024)), dim3(256), 0, st,
                     static_cast<const double2*>(xs), static_cast<double2*>(e), n);
  AIM_HIP(hipGetLastError());
}

}  // namespace aim
