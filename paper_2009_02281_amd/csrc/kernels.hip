// Device kernels of the AIMx matvec and of the batched Krylov solver, for
// gfx950 (CDNA4: 64-lane wavefronts, 160 KB LDS per CU).
//
// Matvec (eq. LAIMx): y = P^T IFFT( H_hat * FFT( pad(P x) ) ) + C x
//   project        brick-tiled scatter of quadrature-point sources onto the
//                  grid; each thread owns one grid node of an LDS-staged brick
//                  and walks that brick's sorted source list, so the sum order
//                  is fixed and no atomics are used;
//   fft_row/col    LDS-staged Stockham passes (radix 8 with one radix-2/4
//                  stage), pruned: forward passes read only the non-zero half
//                  of each padded line, inverse passes write only the half that
//                  is kept; column passes move whole 128-byte row segments so
//                  the strided y/z lines are read and written coalesced;
//                  the z pass multiplies by the kernel spectrum between its
//                  forward and inverse transforms without leaving LDS;
//   interp_near    gather of the stencil potentials per quadrature point plus
//                  the real CSR near-field correction, one pass over y.
#include <hip/hip_runtime.h>

#include <cmath>
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

template <typename T, int R, bool INV>
struct Dft;

template <typename T, bool INV>
struct Dft<T, 2, INV> {
  static __device__ __forceinline__ void run(cx<T>* v) {
    const cx<T> a = v[0];
    v[0] = cadd(a, v[1]);
    v[1] = csub(a, v[1]);
  }
};

template <typename T, bool INV>
struct Dft<T, 4, INV> {
  static __device__ __forceinline__ void run(cx<T>* v) {
    const cx<T> t0 = cadd(v[0], v[2]), t1 = csub(v[0], v[2]);
    const cx<T> t2 = cadd(v[1], v[3]), t3 = rot90<T, INV>(csub(v[1], v[3]));
    v[0] = cadd(t0, t2);
    v[2] = csub(t0, t2);
    v[1] = cadd(t1, t3);
    v[3] = csub(t1, t3);
  }
};

template <typename T, bool INV>
struct Dft<T, 8, INV> {
  static __device__ __forceinline__ void run(cx<T>* v) {
    cx<T> e[4] = {v[0], v[2], v[4], v[6]};
    cx<T> o[4] = {v[1], v[3], v[5], v[7]};
    Dft<T, 4, INV>::run(e);
    Dft<T, 4, INV>::run(o);
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

// One Stockham stage on L points held in LDS (element e at s[e * es]).
// Butterfly j reads j + r L/R, twiddles by W_{Ns R}^{r (j mod Ns)}, runs the
// R-point DFT and writes (j div Ns) Ns R + (j mod Ns) + r Ns; Ns is the
// product of the radices of the previous stages.
template <typename T, int L, int R, int NT, bool INV>
__device__ __forceinline__ void stockham_stage(cx<T>* s, int es, int t, int lgNs,
                                               const cx<T>* tw) {
  constexpr int NB = L / (R * NT);
  static_assert(NB >= 1, "too many threads per line for this radix");
  constexpr int lgL = ilog2(L), lgR = ilog2(R);
  const int Ns = 1 << lgNs;
  const int twsh = lgL - lgNs - lgR;  // log2(L / (Ns R))
  cx<T> v[NB][R];
#pragma unroll
  for (int i = 0; i < NB; ++i) {
    const int j = t + i * NT;
    const int k = j & (Ns - 1);
#pragma unroll
    for (int r = 0; r < R; ++r) {
      cx<T> a = s[(j + r * (L / R)) * es];
      if (r > 0) {
        cx<T> w = tw[(r * k) << twsh];
        if (INV) w.y = -w.y;
        a = cmul(a, w);
      }
      v[i][r] = a;
    }
    Dft<T, R, INV>::run(v[i]);
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < NB; ++i) {
    const int j = t + i * NT;
    const int k = j & (Ns - 1);
    const int d = ((j >> lgNs) << (lgNs + lgR)) + k;
#pragma unroll
    for (int r = 0; r < R; ++r) s[(d + r * Ns) * es] = v[i][r];
  }
  __syncthreads();
}

// Full length-L transform in LDS: one radix-2 or radix-4 stage if log2 L is
// not a multiple of 3, then radix-8 stages.
template <typename T, int L, int NT, bool INV>
__device__ __forceinline__ void fft_lds(cx<T>* s, int es, int t, const cx<T>* tw) {
  constexpr int P = ilog2(L);
  int lg = 0;
  if constexpr (P % 3 == 1) {
    stockham_stage<T, L, 2, NT, INV>(s, es, t, lg, tw);
    lg = 1;
  } else if constexpr (P % 3 == 2) {
    stockham_stage<T, L, 4, NT, INV>(s, es, t, lg, tw);
    lg = 2;
  }
#pragma unroll
  for (int q = 0; q < P / 3; ++q) {
    stockham_stage<T, L, 8, NT, INV>(s, es, t, lg, tw);
    lg += 3;
  }
}

// ---------------------------------------------------------------------------
// FFT pass kernels
// ---------------------------------------------------------------------------
struct ColArgs {
  int64_t nlines;        // total lines = nli * nlo
  int lg_nli;            // log2 of lines along the contiguous dimension
  int64_t in_es, in_os;  // element and outer strides of the input (elements)
  int64_t out_es, out_os;
  int64_t in_bs, out_bs;  // per right-hand-side strides
  int Lin, Lout;          // leading elements read / written per line
  // spectral multiply (fused z pass): line (li, lo) = (kx, ky), element = kz
  const void* spec;
  int64_t spec_fs;        // per-frequency stride of the folded spectrum
  const int32_t* rhs_freq;
  int Mx, Nx, My, Ny, Mz, Nz;
};

struct RowArgs {
  int64_t nlines;
  int64_t in_ls, out_ls;
  int64_t in_bs, out_bs;
  int Lin, Lout;
};

// MODE 0: forward, 1: inverse, 2: forward * spectrum then inverse.
template <typename T, int L, int TL, int NT, int MODE>
__global__ __launch_bounds__(TL* NT) void fft_col_kernel(const cx<T>* in, cx<T>* out,
                                                         const cx<T>* __restrict__ twg, ColArgs a) {
  __shared__ cx<T> s[L * TL];
  __shared__ cx<T> tw[L];
  constexpr int NTH = TL * NT;
  const int tid = threadIdx.x;
  const int rhs = blockIdx.y;
  const int64_t line0 = int64_t(blockIdx.x) * TL;
  in += rhs * a.in_bs;
  out += rhs * a.out_bs;
  const int64_t nli_mask = (int64_t(1) << a.lg_nli) - 1;
  for (int m = tid; m < L; m += NTH) tw[m] = twg[m];
  for (int idx = tid; idx < L * TL; idx += NTH) {
    const int l = idx & (TL - 1), e = idx / TL;
    const int64_t line = line0 + l;
    cx<T> v = mkc<T>(T(0), T(0));
    if (e < a.Lin && line < a.nlines)
      v = in[(line >> a.lg_nli) * a.in_os + e * a.in_es + (line & nli_mask)];
    s[e * TL + l] = v;
  }
  __syncthreads();
  const int l = tid & (TL - 1), t = tid / TL;
  if constexpr (MODE == 1) {
    fft_lds<T, L, NT, true>(s + l, TL, t, tw);
  } else {
    fft_lds<T, L, NT, false>(s + l, TL, t, tw);
  }
  if constexpr (MODE == 2) {
    const int64_t line = line0 + l;
    if (line < a.nlines) {
      const int kx = int(line & nli_mask), ky = int(line >> a.lg_nli);
      const int fx = kx <= a.Nx ? kx : a.Mx - kx;
      const int fy = ky <= a.Ny ? ky : a.My - ky;
      const cx<T>* sp = static_cast<const cx<T>*>(a.spec) + int64_t(a.rhs_freq[rhs]) * a.spec_fs;
      for (int e = t; e < L; e += NT) {
        const int fz = e <= a.Nz ? e : a.Mz - e;
        const cx<T> hv = sp[(int64_t(fz) * (a.Ny + 1) + fy) * (a.Nx + 1) + fx];
        s[e * TL + l] = cmul(s[e * TL + l], hv);
      }
    }
    __syncthreads();
    fft_lds<T, L, NT, true>(s + l, TL, t, tw);
  }
  for (int idx = tid; idx < a.Lout * TL; idx += NTH) {
    const int ll = idx & (TL - 1), e = idx / TL;
    const int64_t line = line0 + ll;
    if (line < a.nlines)
      out[(line >> a.lg_nli) * a.out_os + e * a.out_es + (line & nli_mask)] = s[e * TL + ll];
  }
}

template <typename T, int L, int TL, int NT, bool INV>
__global__ __launch_bounds__(TL* NT) void fft_row_kernel(const cx<T>* in, cx<T>* out,
                                                         const cx<T>* __restrict__ twg, RowArgs a) {
  constexpr int LP = L + 1;  // padded pitch staggers lines across LDS banks
  __shared__ cx<T> s[TL * LP];
  __shared__ cx<T> tw[L];
  constexpr int NTH = TL * NT;
  const int tid = threadIdx.x;
  const int rhs = blockIdx.y;
  const int64_t line0 = int64_t(blockIdx.x) * TL;
  in += rhs * a.in_bs;
  out += rhs * a.out_bs;
  for (int m = tid; m < L; m += NTH) tw[m] = twg[m];
  for (int idx = tid; idx < L * TL; idx += NTH) {
    const int l = idx / L, e = idx & (L - 1);
    const int64_t line = line0 + l;
    cx<T> v = mkc<T>(T(0), T(0));
    if (e < a.Lin && line < a.nlines) v = in[line * a.in_ls + e];
    s[l * LP + e] = v;
  }
  __syncthreads();
  const int l = tid / NT, t = tid & (NT - 1);
  fft_lds<T, L, NT, INV>(s + l * LP, 1, t, tw);
  const int lg_out = __builtin_ctz(unsigned(a.Lout));  // Lout is a power of two
  for (int idx = tid; idx < a.Lout * TL; idx += NTH) {
    const int ll = idx >> lg_out, e = idx & (a.Lout - 1);
    const int64_t line = line0 + ll;
    if (line < a.nlines) out[line * a.out_ls + e] = s[ll * LP + e];
  }
}

// launch configuration: 256 threads, LDS <= 64 KB of line data
template <typename T>
struct ColCfg {
  static constexpr int kTLmin = sizeof(T) == 8 ? 8 : 16;  // 128-byte row segments
};

template <typename T, int L>
struct PassCfg {
  static constexpr int COL_NT = (L / 8) < (256 / ColCfg<T>::kTLmin) ? (L / 8) : (256 / ColCfg<T>::kTLmin);
  static constexpr int COL_TL = 256 / COL_NT;
  static constexpr int ROW_NT = (L / 8) < 64 ? (L / 8) : 64;
  static constexpr int ROW_TL = 256 / ROW_NT;
};

template <typename T, int L>
void col_pass_L(int mode, const void* in, void* out, const void* tw, const ColArgs& a, int nrhs,
                hipStream_t s) {
  using C = PassCfg<T, L>;
  dim3 grid(unsigned((a.nlines + C::COL_TL - 1) / C::COL_TL), unsigned(nrhs));
  const cx<T>* i = static_cast<const cx<T>*>(in);
  cx<T>* o = static_cast<cx<T>*>(out);
  const cx<T>* w = static_cast<const cx<T>*>(tw);
  if (mode == 0)
    hipLaunchKernelGGL((fft_col_kernel<T, L, C::COL_TL, C::COL_NT, 0>), grid, dim3(256), 0, s, i, o, w, a);
  else if (mode == 1)
    hipLaunchKernelGGL((fft_col_kernel<T, L, C::COL_TL, C::COL_NT, 1>), grid, dim3(256), 0, s, i, o, w, a);
  else
    hipLaunchKernelGGL((fft_col_kernel<T, L, C::COL_TL, C::COL_NT, 2>), grid, dim3(256), 0, s, i, o, w, a);
}

template <typename T, int L>
void row_pass_L(bool inv, const void* in, void* out, const void* tw, const RowArgs& a, int nrhs,
                hipStream_t s) {
  using C = PassCfg<T, L>;
  dim3 grid(unsigned((a.nlines + C::ROW_TL - 1) / C::ROW_TL), unsigned(nrhs));
  const cx<T>* i = static_cast<const cx<T>*>(in);
  cx<T>* o = static_cast<cx<T>*>(out);
  const cx<T>* w = static_cast<const cx<T>*>(tw);
  if (inv)
    hipLaunchKernelGGL((fft_row_kernel<T, L, C::ROW_TL, C::ROW_NT, true>), grid, dim3(256), 0, s, i, o, w, a);
  else
    hipLaunchKernelGGL((fft_row_kernel<T, L, C::ROW_TL, C::ROW_NT, false>), grid, dim3(256), 0, s, i, o, w, a);
}

template <typename T>
void col_pass(int L, int mode, const void* in, void* out, const void* tw, const ColArgs& a,
              int nrhs, hipStream_t s) {
  switch (L) {
    case 16: col_pass_L<T, 16>(mode, in, out, tw, a, nrhs, s); break;
    case 32: col_pass_L<T, 32>(mode, in, out, tw, a, nrhs, s); break;
    case 64: col_pass_L<T, 64>(mode, in, out, tw, a, nrhs, s); break;
    case 128: col_pass_L<T, 128>(mode, in, out, tw, a, nrhs, s); break;
    case 256: col_pass_L<T, 256>(mode, in, out, tw, a, nrhs, s); break;
    case 512: col_pass_L<T, 512>(mode, in, out, tw, a, nrhs, s); break;
    default: throw Error(AIM_ERR_GRID, "unsupported FFT length");
  }
  AIM_HIP(hipGetLastError());
}

template <typename T>
void row_pass(int L, bool inv, const void* in, void* out, const void* tw, const RowArgs& a,
              int nrhs, hipStream_t s) {
  switch (L) {
    case 16: row_pass_L<T, 16>(inv, in, out, tw, a, nrhs, s); break;
    case 32: row_pass_L<T, 32>(inv, in, out, tw, a, nrhs, s); break;
    case 64: row_pass_L<T, 64>(inv, in, out, tw, a, nrhs, s); break;
    case 128: row_pass_L<T, 128>(inv, in, out, tw, a, nrhs, s); break;
    case 256: row_pass_L<T, 256>(inv, in, out, tw, a, nrhs, s); break;
    case 512: row_pass_L<T, 512>(inv, in, out, tw, a, nrhs, s); break;
    default: throw Error(AIM_ERR_GRID, "unsupported FFT length");
  }
  AIM_HIP(hipGetLastError());
}

// ---------------------------------------------------------------------------
// convolution phi = H q: pruned forward FFT, spectral multiply, pruned inverse
// work layout per right-hand side (6 Ng complex): B = [Nz][My][Mx] (4 Ng)
// followed by A = [Nz][Ny][Mx] (2 Ng).
// ---------------------------------------------------------------------------
template <typename T>
void launch_convolve(const GridShape& g, const void* q, void* work, void* phi, const void* spec,
                     const int32_t* rhs_freq, int nrhs, const void* const* tw, hipStream_t s) {
  const int Nx = g.N[0], Ny = g.N[1], Nz = g.N[2];
  const int Mx = g.M[0], My = g.M[1], Mz = g.M[2];
  const int64_t Ng = g.Ng;
  cx<T>* B = static_cast<cx<T>*>(work);
  cx<T>* A = B + 4 * Ng;
  // x forward: rows (y, z) of q, Nx -> Mx
  {
    RowArgs a{int64_t(Ny) * Nz, Nx, Mx, Ng, 6 * Ng, Nx, Mx};
    row_pass<T>(Mx, false, q, A, tw[0], a, nrhs, s);
  }
  // y forward: A [Nz][Ny][Mx] -> B [Nz][My][Mx]
  {
    ColArgs a{};
    a.nlines = int64_t(Mx) * Nz;
    a.lg_nli = ilog2(Mx);
    a.in_es = Mx;
    a.in_os = int64_t(Ny) * Mx;
    a.out_es = Mx;
    a.out_os = int64_t(My) * Mx;
    a.in_bs = a.out_bs = 6 * Ng;
    a.Lin = Ny;
    a.Lout = My;
    col_pass<T>(My, 0, A, B, tw[1], a, nrhs, s);
  }
  // z forward * spectrum * z inverse, in place on B, keeping z < Nz
  {
    ColArgs a{};
    a.nlines = int64_t(Mx) * My;
    a.lg_nli = ilog2(Mx);
    a.in_es = a.out_es = int64_t(My) * Mx;
    a.in_os = a.out_os = Mx;
    a.in_bs = a.out_bs = 6 * Ng;
    a.Lin = Nz;
    a.Lout = Nz;
    a.spec = spec;
    a.spec_fs = g.Nfold;
    a.rhs_freq = rhs_freq;
    a.Mx = Mx;
    a.Nx = Nx;
    a.My = My;
    a.Ny = Ny;
    a.Mz = Mz;
    a.Nz = Nz;
    col_pass<T>(Mz, 2, B, B, tw[2], a, nrhs, s);
  }
  // y inverse: B [Nz][My][Mx] -> A [Nz][Ny][Mx]
  {
    ColArgs a{};
    a.nlines = int64_t(Mx) * Nz;
    a.lg_nli = ilog2(Mx);
    a.in_es = Mx;
    a.in_os = int64_t(My) * Mx;
    a.out_es = Mx;
    a.out_os = int64_t(Ny) * Mx;
    a.in_bs = a.out_bs = 6 * Ng;
    a.Lin = My;
    a.Lout = Ny;
    col_pass<T>(My, 1, B, A, tw[1], a, nrhs, s);
  }
  // x inverse: rows of A (Mx) -> phi (Nx)
  {
    RowArgs a{int64_t(Ny) * Nz, Mx, Nx, 6 * Ng, Ng, Mx, Nx};
    row_pass<T>(Mx, true, A, phi, tw[0], a, nrhs, s);
  }
}

template void launch_convolve<double>(const GridShape&, const void*, void*, void*, const void*,
                                      const int32_t*, int, const void* const*, hipStream_t);
template void launch_convolve<float>(const GridShape&, const void*, void*, void*, const void*,
                                     const int32_t*, int, const void* const*, hipStream_t);

// ---------------------------------------------------------------------------
// kernel spectrum: circulant embedding of G on the padded grid, full 3-D FFT,
// folded to its (Nx+1)(Ny+1)(Nz+1) distinct entries (the embedding is even in
// every axis) and scaled by 1/(Mx My Mz)
// ---------------------------------------------------------------------------
__global__ void green_sample_kernel(double2* c, int Nx, int Ny, int Nz, double k, double h) {
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
      if (d2 == 0.0) {
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
                                     int Ny, int Nz, double scale) {
  const int Fx = Nx + 1, Fy = Ny + 1, Fz = Nz + 1;
  const int64_t total = int64_t(Fx) * Fy * Fz;
  const int Mx = 2 * Nx, My = 2 * Ny;
  for (int64_t idx = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; idx < total;
       idx += int64_t(gridDim.x) * blockDim.x) {
    const int fx = int(idx % Fx), fy = int((idx / Fx) % Fy), fz = int(idx / (int64_t(Fx) * Fy));
    double2 v = full[(int64_t(fz) * My + fy) * Mx + fx];
    v.x *= scale;
    v.y *= scale;
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
                     void* spec32, const void* const* tw64, hipStream_t s) {
  const int Nx = g.N[0], Ny = g.N[1], Nz = g.N[2];
  const int Mx = g.M[0], My = g.M[1], Mz = g.M[2];
  double2* F = static_cast<double2*>(full_work);
  hipLaunchKernelGGL(green_sample_kernel, dim3(4096), dim3(256), 0, s, F, Nx, Ny, Nz, k, h);
  AIM_HIP(hipGetLastError());
  const int64_t Np = int64_t(Mx) * My * Mz;
  {
    RowArgs a{int64_t(My) * Mz, Mx, Mx, 0, 0, Mx, Mx};
    row_pass<double>(Mx, false, F, F, tw64[0], a, 1, s);
  }
  {
    ColArgs a{};
    a.nlines = int64_t(Mx) * Mz;
    a.lg_nli = ilog2(Mx);
    a.in_es = a.out_es = Mx;
    a.in_os = a.out_os = int64_t(My) * Mx;
    a.Lin = a.Lout = My;
    col_pass<double>(My, 0, F, F, tw64[1], a, 1, s);
  }
  {
    ColArgs a{};
    a.nlines = int64_t(Mx) * My;
    a.lg_nli = ilog2(Mx);
    a.in_es = a.out_es = int64_t(My) * Mx;
    a.in_os = a.out_os = Mx;
    a.Lin = a.Lout = Mz;
    col_pass<double>(Mz, 0, F, F, tw64[2], a, 1, s);
  }
  hipLaunchKernelGGL(fold_spectrum_kernel, dim3(2048), dim3(256), 0, s, F,
                     static_cast<double2*>(spec64), static_cast<float2*>(spec32), Nx, Ny, Nz,
                     1.0 / double(Np));
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
// projection q = P x (brick-tiled, node-owner gather from an LDS source list)
// ---------------------------------------------------------------------------
template <typename T, int ORD>
struct QpEntry {
  int sx, sy, sz;
  T wx[ORD + 1], wy[ORD + 1], wz[ORD + 1];
  cx<T> amp;  // (A/3) x_j
};

template <typename T, int ORD>
__device__ __forceinline__ void lagrange_dev(T u, T* out) {
#pragma unroll
  for (int a = 0; a <= ORD; ++a) {
    T w = T(1);
#pragma unroll
    for (int b = 0; b <= ORD; ++b)
      if (b != a) w = w * (u - T(b)) / T(a - b);
    out[a] = w;
  }
}

template <typename T, int ORD, int BX, int BY, int BZ>
__global__ __launch_bounds__(BX* BY* BZ) void project_kernel(
    const cx<T>* __restrict__ x, cx<T>* __restrict__ q, const int32_t* __restrict__ packed,
    const T* __restrict__ local, const T* __restrict__ weight, const int32_t* __restrict__ bptr,
    const int32_t* __restrict__ blist, int64_t nq, int64_t n, int Nx, int Ny, int Nz, int nbx,
    int nby, int64_t Ng) {
  constexpr int NTH = BX * BY * BZ;
  __shared__ QpEntry<T, ORD> ent[NTH];
  const int tid = threadIdx.x;
  const int b = blockIdx.x;
  const int rhs = blockIdx.y;
  const int bx = b % nbx, by = (b / nbx) % nby, bz = b / (nbx * nby);
  const int nx = bx * BX + (tid % BX);
  const int ny = by * BY + ((tid / BX) % BY);
  const int nz = bz * BZ + (tid / (BX * BY));
  x += rhs * n;
  q += rhs * Ng;
  cx<T> acc = mkc<T>(T(0), T(0));
  const int beg = bptr[b], end = bptr[b + 1];
  for (int c0 = beg; c0 < end; c0 += NTH) {
    const int cnt = min(NTH, end - c0);
    if (tid < cnt) {
      const int p = blist[c0 + tid];
      const int pk = packed[p];
      QpEntry<T, ORD> e;
      e.sx = pk & 1023;
      e.sy = (pk >> 10) & 1023;
      e.sz = (pk >> 20) & 1023;
      lagrange_dev<T, ORD>(local[p], e.wx);
      lagrange_dev<T, ORD>(local[nq + p], e.wy);
      lagrange_dev<T, ORD>(local[2 * nq + p], e.wz);
      e.amp = cscale(x[p / 3], weight[p]);
      ent[tid] = e;
    }
    __syncthreads();
    for (int i = 0; i < cnt; ++i) {
      const int dx = nx - ent[i].sx, dy = ny - ent[i].sy, dz = nz - ent[i].sz;
      if (unsigned(dx) <= unsigned(ORD) && unsigned(dy) <= unsigned(ORD) &&
          unsigned(dz) <= unsigned(ORD)) {
        const T w = ent[i].wx[dx] * ent[i].wy[dy] * ent[i].wz[dz];
        acc.x += w * ent[i].amp.x;
        acc.y += w * ent[i].amp.y;
      }
    }
    __syncthreads();
  }
  if (nx < Nx && ny < Ny && nz < Nz) q[(int64_t(nz) * Ny + ny) * Nx + nx] = acc;
}

template <typename T>
void launch_project(const GridShape& g, int order, const QpDevice& qp, const int32_t* brick_ptr,
                    const int32_t* brick_qp, const int bricks[3], const int nbrick[3],
                    const void* x, int64_t n, void* q, int nrhs, hipStream_t s) {
  AIM_REQUIRE(bricks[0] == 8 && bricks[1] == 4 && bricks[2] == 4, AIM_ERR_STATE,
              "projection bricks must be 8x4x4");
  dim3 grid(unsigned(nbrick[0] * nbrick[1] * nbrick[2]), unsigned(nrhs));
  const cx<T>* xi = static_cast<const cx<T>*>(x);
  cx<T>* qo = static_cast<cx<T>*>(q);
  const T* loc = static_cast<const T*>(qp.local);
  const T* w = static_cast<const T*>(qp.weight);
  if (order == 2)
    hipLaunchKernelGGL((project_kernel<T, 2, 8, 4, 4>), grid, dim3(128), 0, s, xi, qo,
                       qp.packed_start, loc, w, brick_ptr, brick_qp, qp.nq, n, g.N[0], g.N[1],
                       g.N[2], nbrick[0], nbrick[1], g.Ng);
  else
    hipLaunchKernelGGL((project_kernel<T, 3, 8, 4, 4>), grid, dim3(128), 0, s, xi, qo,
                       qp.packed_start, loc, w, brick_ptr, brick_qp, qp.nq, n, g.N[0], g.N[1],
                       g.N[2], nbrick[0], nbrick[1], g.Ng);
  AIM_HIP(hipGetLastError());
}

template void launch_project<double>(const GridShape&, int, const QpDevice&, const int32_t*,
                                     const int32_t*, const int*, const int*, const void*, int64_t,
                                     void*, int, hipStream_t);
template void launch_project<float>(const GridShape&, int, const QpDevice&, const int32_t*,
                                    const int32_t*, const int*, const int*, const void*, int64_t,
                                    void*, int, hipStream_t);

// ---------------------------------------------------------------------------
// interpolation y = P^T phi and near correction y += C x (one thread per row)
// ---------------------------------------------------------------------------
template <typename T, int ORD, bool INTERP, bool NEARC>
__global__ __launch_bounds__(256) void interp_near_kernel(
    const cx<T>* __restrict__ phi, const cx<T>* __restrict__ x, cx<T>* __restrict__ y,
    const int32_t* __restrict__ packed, const T* __restrict__ local, const T* __restrict__ weight,
    const int32_t* __restrict__ rowptr, const int32_t* __restrict__ col,
    const T* __restrict__ val, int64_t n, int64_t nq, int Nx, int Ny, int64_t Ng) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  const int rhs = blockIdx.y;
  if (i >= n) return;
  cx<T> acc = mkc<T>(T(0), T(0));
  if constexpr (INTERP) {
    const cx<T>* ph = phi + rhs * Ng;
#pragma unroll
    for (int qq = 0; qq < 3; ++qq) {
      const int64_t p = 3 * i + qq;
      const int pk = packed[p];
      const int sx = pk & 1023, sy = (pk >> 10) & 1023, sz = (pk >> 20) & 1023;
      T wx[ORD + 1], wy[ORD + 1], wz[ORD + 1];
      lagrange_dev<T, ORD>(local[p], wx);
      lagrange_dev<T, ORD>(local[nq + p], wy);
      lagrange_dev<T, ORD>(local[2 * nq + p], wz);
      const cx<T>* base = ph + (int64_t(sz) * Ny + sy) * Nx + sx;
      cx<T> sq = mkc<T>(T(0), T(0));
#pragma unroll
      for (int c = 0; c <= ORD; ++c) {
#pragma unroll
        for (int b = 0; b <= ORD; ++b) {
          const cx<T>* rowp = base + (int64_t(c) * Ny + b) * Nx;
          cx<T> sr = mkc<T>(T(0), T(0));
#pragma unroll
          for (int a = 0; a <= ORD; ++a) {
            const cx<T> v = rowp[a];
            sr.x += wx[a] * v.x;
            sr.y += wx[a] * v.y;
          }
          const T wyz = wy[b] * wz[c];
          sq.x += wyz * sr.x;
          sq.y += wyz * sr.y;
        }
      }
      const T w = weight[p];
      acc.x += w * sq.x;
      acc.y += w * sq.y;
    }
  }
  if constexpr (NEARC) {
    const cx<T>* xr = x + rhs * n;
    for (int k = rowptr[i]; k < rowptr[i + 1]; ++k) {
      const T v = val[k];
      const cx<T> xv = xr[col[k]];
      acc.x += v * xv.x;
      acc.y += v * xv.y;
    }
  }
  y[rhs * n + i] = acc;
}

template <typename T>
void launch_interp_near(const GridShape& g, int order, const QpDevice& qp, const CsrDevice& csr,
                        const void* phi, const void* x, void* y, int nrhs, bool do_interp,
                        bool do_near, hipStream_t s) {
  const int64_t n = csr.n;
  dim3 grid(unsigned((n + 255) / 256), unsigned(nrhs));
  const cx<T>* ph = static_cast<const cx<T>*>(phi);
  const cx<T>* xi = static_cast<const cx<T>*>(x);
  cx<T>* yo = static_cast<cx<T>*>(y);
  const T* loc = static_cast<const T*>(qp.local);
  const T* w = static_cast<const T*>(qp.weight);
  const T* v = static_cast<const T*>(csr.val);
#define AIM_IN_LAUNCH(ORD, I, NR)                                                               \
  hipLaunchKernelGGL((interp_near_kernel<T, ORD, I, NR>), grid, dim3(256), 0, s, ph, xi, yo,    \
                     qp.packed_start, loc, w, csr.rowptr, csr.col, v, n, qp.nq, g.N[0], g.N[1], \
                     g.Ng)
  if (order == 2) {
    if (do_interp && do_near) AIM_IN_LAUNCH(2, true, true);
    else if (do_interp) AIM_IN_LAUNCH(2, true, false);
    else AIM_IN_LAUNCH(2, false, true);
  } else {
    if (do_interp && do_near) AIM_IN_LAUNCH(3, true, true);
    else if (do_interp) AIM_IN_LAUNCH(3, true, false);
    else AIM_IN_LAUNCH(3, false, true);
  }
#undef AIM_IN_LAUNCH
  AIM_HIP(hipGetLastError());
}

template void launch_interp_near<double>(const GridShape&, int, const QpDevice&, const CsrDevice&,
                                         const void*, const void*, void*, int, bool, bool,
                                         hipStream_t);
template void launch_interp_near<float>(const GridShape&, int, const QpDevice&, const CsrDevice&,
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
                                                        double2* partial) {
  __shared__ double2 sh[256];
  const int c = blockIdx.x, i = blockIdx.y, r = blockIdx.z;
  const double2* vi = V + (int64_t(i) * si + int64_t(r) * sr) * n;
  const double2* wr = w + int64_t(r) * n;
  double2 acc;
  acc.x = 0.0;
  acc.y = 0.0;
  const int64_t b = int64_t(c) * kDotChunk, e = min(n, b + kDotChunk);
  for (int64_t k = b + threadIdx.x; k < e; k += 256) {
    const double2 a = vi[k], x = wr[k];
    acc.x += a.x * x.x + a.y * x.y;
    acc.y += a.x * x.y - a.y * x.x;
  }
  const double2 s = block_sum2(acc, sh);
  if (threadIdx.x == 0) partial[(int64_t(r) * nv + i) * nchunk + c] = s;
}

__global__ void reduce_partials_kernel(const double2* partial, int nchunk, int total,
                                       double2* out) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= total) return;
  double2 s;
  s.x = 0.0;
  s.y = 0.0;
  for (int c = 0; c < nchunk; ++c) {
    s.x += partial[int64_t(idx) * nchunk + c].x;
    s.y += partial[int64_t(idx) * nchunk + c].y;
  }
  out[idx] = s;
}

void launch_block_dot(const void* V, int64_t si, int64_t sr, const void* w, int64_t n, int nv,
                      int nrhs, void* partial, void* out, hipStream_t s) {
  const int nchunk = int((n + kDotChunk - 1) / kDotChunk);
  hipLaunchKernelGGL(block_dot_kernel, dim3(nchunk, nv, nrhs), dim3(256), 0, s,
                     static_cast<const double2*>(V), si, sr, static_cast<const double2*>(w), n, nv,
                     nchunk, static_cast<double2*>(partial));
  AIM_HIP(hipGetLastError());
  const int total = nv * nrhs;
  hipLaunchKernelGGL(reduce_partials_kernel, dim3((total + 127) / 128), dim3(128), 0, s,
                     static_cast<const double2*>(partial), nchunk, total,
                     static_cast<double2*>(out));
  AIM_HIP(hipGetLastError());
}

// w[r] -= sum_{i < nv} h[r][i] V[r][i]
__global__ __launch_bounds__(256) void block_update_kernel(const double2* __restrict__ V,
                                                           int64_t si, int64_t sr,
                                                           double2* __restrict__ w,
                                                           int64_t n, int nv,
                                                           const double2* __restrict__ h,
                                                           int64_t ldh) {
  const int r = blockIdx.y;
  const double2* hr = h + int64_t(r) * ldh;
  for (int64_t k = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; k < n;
       k += int64_t(gridDim.x) * blockDim.x) {
    double2 acc = w[int64_t(r) * n + k];
    for (int i = 0; i < nv; ++i) {
      const double2 a = V[(int64_t(i) * si + int64_t(r) * sr) * n + k];
      const double2 c = hr[i];
      acc.x -= c.x * a.x - c.y * a.y;
      acc.y -= c.x * a.y + c.y * a.x;
    }
    w[int64_t(r) * n + k] = acc;
  }
}

void launch_block_update(const void* V, int64_t si, int64_t sr, void* w, int64_t n, int nv,
                         int nrhs, const void* h, int64_t ldh, hipStream_t s) {
  hipLaunchKernelGGL(block_update_kernel, dim3(grid_for(n, 256 * 4), nrhs), dim3(256), 0, s,
                     static_cast<const double2*>(V), si, sr, static_cast<double2*>(w), n, nv,
                     static_cast<const double2*>(h), ldh);
  AIM_HIP(hipGetLastError());
}

__global__ __launch_bounds__(256) void norm_partial_kernel(const double2* __restrict__ w,
                                                           int64_t n, int nchunk,
                                                           double2* partial) {
  __shared__ double2 sh[256];
  const int c = blockIdx.x, r = blockIdx.y;
  const double2* wr = w + int64_t(r) * n;
  double2 acc;
  acc.x = 0.0;
  acc.y = 0.0;
  const int64_t b = int64_t(c) * kDotChunk, e = min(n, b + kDotChunk);
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

void launch_norms(const void* w, int64_t n, int nrhs, void* partial, double* out, hipStream_t s) {
  const int nchunk = int((n + kDotChunk - 1) / kDotChunk);
  hipLaunchKernelGGL(norm_partial_kernel, dim3(nchunk, nrhs), dim3(256), 0, s,
                     static_cast<const double2*>(w), n, nchunk, static_cast<double2*>(partial));
  AIM_HIP(hipGetLastError());
  hipLaunchKernelGGL(norm_finish_kernel, dim3((nrhs + 127) / 128), dim3(128), 0, s,
                     static_cast<const double2*>(partial), nchunk, nrhs, out);
  AIM_HIP(hipGetLastError());
}

__global__ void scale_inv_kernel(const double2* w, const double* nrm, double2* out, int64_t n,
                                 int64_t out_stride) {
  const int r = blockIdx.y;
  const double nv = nrm[r];
  const double sc = nv > 0.0 ? 1.0 / nv : 0.0;
  for (int64_t k = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; k < n;
       k += int64_t(gridDim.x) * blockDim.x) {
    double2 v = w[int64_t(r) * n + k];
    v.x *= sc;
    v.y *= sc;
    out[int64_t(r) * out_stride + k] = v;
  }
}

void launch_scale_inv(const void* w, const double* nrm, void* out, int64_t n, int nrhs,
                      int64_t out_stride, hipStream_t s) {
  hipLaunchKernelGGL(scale_inv_kernel, dim3(grid_for(n, 1024), nrhs), dim3(256), 0, s,
                     static_cast<const double2*>(w), nrm, static_cast<double2*>(out), n,
                     out_stride);
  AIM_HIP(hipGetLastError());
}

__global__ void combine_kernel(const double2* __restrict__ Z, int64_t si, int64_t sr,
                               const double2* __restrict__ y, int64_t ldy, int nv,
                               double2* __restrict__ x, int64_t n) {
  const int r = blockIdx.y;
  const double2* yr = y + int64_t(r) * ldy;
  for (int64_t k = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; k < n;
       k += int64_t(gridDim.x) * blockDim.x) {
    double2 acc = x[int64_t(r) * n + k];
    for (int i = 0; i < nv; ++i) {
      const double2 a = Z[(int64_t(i) * si + int64_t(r) * sr) * n + k];
      const double2 c = yr[i];
      acc.x += c.x * a.x - c.y * a.y;
      acc.y += c.x * a.y + c.y * a.x;
    }
    x[int64_t(r) * n + k] = acc;
  }
}

void launch_combine(const void* Z, int64_t si, int64_t sr, const void* y, int64_t ldy, int nv,
                    void* x, int64_t n, int nrhs, hipStream_t s) {
  hipLaunchKernelGGL(combine_kernel, dim3(grid_for(n, 1024), nrhs), dim3(256), 0, s,
                     static_cast<const double2*>(Z), si, sr, static_cast<const double2*>(y), ldy,
                     nv, static_cast<double2*>(x), n);
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
