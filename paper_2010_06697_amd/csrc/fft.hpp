// fft.hpp -- mixed-radix (2, 3, 4, 8) self-sorting Stockham FFT on lines held
// in LDS, cooperatively by all threads of a workgroup.
//
// A transform of length N = prod R_s runs one stage per radix. At a stage with
// radix R, after Ns = R_1 ... R_{s-1}, butterfly j (0 <= j < N/R) reads
// x[j + r N/R], multiplies element r by w^{(j mod Ns) r N/(Ns R)} with
// w = exp(-2 pi i / N), takes the length-R DFT and writes element r to
// (j - j mod Ns) R + (j mod Ns) + r Ns of the other buffer (the Stockham
// autosort formulation, so no bit reversal is needed). Forward transforms use
// exp(-2 pi i m k / N), inverse ones exp(+...), both unnormalised.
#pragma once

#include "common.hpp"

namespace admm {

template <typename C> __device__ __forceinline__ C cadd(C a, C b) { return C{a.x + b.x, a.y + b.y}; }
template <typename C> __device__ __forceinline__ C csub(C a, C b) { return C{a.x - b.x, a.y - b.y}; }
template <typename C> __device__ __forceinline__ C cmul(C a, C b) {
  return C{a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
// a * conj(b)
template <typename C> __device__ __forceinline__ C cmulc(C a, C b) {
  return C{a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y};
}
// multiply by -i (forward) or +i (inverse)
template <bool INV, typename C> __device__ __forceinline__ C rot90(C a) {
  return INV ? C{-a.y, a.x} : C{a.y, -a.x};
}

template <bool INV, typename C> __device__ __forceinline__ void dft2(C *v) {
  C a = v[0], b = v[1];
  v[0] = cadd(a, b);
  v[1] = csub(a, b);
}

template <bool INV, typename C> __device__ __forceinline__ void dft3(C *v) {
  using T = decltype(v[0].x);
  const T h = (T)0.86602540378443864676372317075294;  // sqrt(3)/2
  C a = v[0], b = v[1], c = v[2];
  C t1 = cadd(b, c);
  C t2 = C{a.x - (T)0.5 * t1.x, a.y - (T)0.5 * t1.y};
  C d = csub(b, c);
  C t3 = rot90<INV>(C{h * d.x, h * d.y});
  v[0] = cadd(a, t1);
  v[1] = cadd(t2, t3);
  v[2] = csub(t2, t3);
}

template <bool INV, typename C> __device__ __forceinline__ void dft4(C *v) {
  C t0 = cadd(v[0], v[2]), t1 = csub(v[0], v[2]);
  C t2 = cadd(v[1], v[3]), t3 = rot90<INV>(csub(v[1], v[3]));
  v[0] = cadd(t0, t2);
  v[2] = csub(t0, t2);
  v[1] = cadd(t1, t3);
  v[3] = csub(t1, t3);
}

template <bool INV, typename C> __device__ __forceinline__ void dft8(C *v) {
  using T = decltype(v[0].x);
  const T c = (T)0.70710678118654752440084436210485;  // sqrt(2)/2
  C e[4] = {v[0], v[2], v[4], v[6]};
  C o[4] = {v[1], v[3], v[5], v[7]};
  dft4<INV>(e);
  dft4<INV>(o);
  // o_k *= w8^k, w8 = exp(-+ 2 pi i / 8)
  C o1 = o[1], o3 = o[3];
  if (!INV) {
    o[1] = C{c * (o1.x + o1.y), c * (o1.y - o1.x)};
    o[3] = C{c * (o3.y - o3.x), -c * (o3.x + o3.y)};
  } else {
    o[1] = C{c * (o1.x - o1.y), c * (o1.x + o1.y)};
    o[3] = C{-c * (o3.x + o3.y), c * (o3.x - o3.y)};
  }
  o[2] = rot90<INV>(o[2]);
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    v[k] = cadd(e[k], o[k]);
    v[k + 4] = csub(e[k], o[k]);
  }
}

// length-16 DFT as 4 x 4 (the register-resident x2 / x3 passes of length
// 256): with n = n1 + 4 n2 and k = 4 k1 + k2,
// X[4 k1 + k2] = sum_n1 w16^(n1 k2) (sum_n2 x[n1 + 4 n2] w4^(n2 k2)) w4^(n1 k1);
// the inner length-4 transforms run on v[n1], v[n1+4], v[n1+8], v[n1+12],
// the outer ones on the twiddled results of each k2
template <bool INV, typename C> __device__ __forceinline__ void dft16(C *v) {
  using T = decltype(v[0].x);
  const T c1 = (T)0.92387953251128675613;  // cos(pi/8)
  const T s1 = (T)0.38268343236508977173;  // sin(pi/8)
  const T h = (T)0.70710678118654752440;   // sqrt(2)/2
  // w16^m = (cos(2 pi m/16), -+ sin(2 pi m/16)) for the m = n1 k2 that occur
  const T wr[10] = {(T)1, c1, h, s1, (T)0, (T)0, -h, (T)0, (T)0, -c1};
  const T wi[10] = {(T)0, s1, h, c1, (T)1, (T)0, h, (T)0, (T)0, -s1};
  C a[4][4];
#pragma unroll
  for (int n1 = 0; n1 < 4; ++n1) {
    C q[4] = {v[n1], v[n1 + 4], v[n1 + 8], v[n1 + 12]};
    dft4<INV>(q);
#pragma unroll
    for (int k2 = 0; k2 < 4; ++k2) {
      const int m = n1 * k2;
      if (m == 0) {
        a[k2][n1] = q[k2];
      } else {
        const C w = C{wr[m], INV ? wi[m] : -wi[m]};
        a[k2][n1] = cmul(q[k2], w);
      }
    }
  }
#pragma unroll
  for (int k2 = 0; k2 < 4; ++k2) {
    dft4<INV>(a[k2]);
#pragma unroll
    for (int k1 = 0; k1 < 4; ++k1) v[4 * k1 + k2] = a[k2][k1];
  }
}

// length-A*B DFT split as n = n1 + A n2, k = k2 + B k1:
// X[k2 + B k1] = sum_n1 w_A^(n1 k1) w_AB^(n1 k2) sum_n2 x[n1 + A n2] w_B^(n2 k2),
// inner length-B transforms over n2, the twiddles, outer length-A ones over
// n1; wc / ws: cos / sin of 2 pi m / (A B) for the m = n1 k2 that occur
template <int A, int B, bool INV, typename C>
__device__ __forceinline__ void dft_split(C *v, const double *wc, const double *ws);

// lengths 12 = 4 x 3 and 24 = 8 x 3 (the register-resident x2 / x3 passes
// of lengths 48 and 96)
template <bool INV, typename C> __device__ __forceinline__ void dft12(C *v) {
  const double h3 = 0.866025403784438646764;  // sqrt(3)/2
  const double wc[7] = {1.0, h3, 0.5, 0.0, -0.5, -h3, -1.0};
  const double ws[7] = {0.0, 0.5, h3, 1.0, h3, 0.5, 0.0};
  dft_split<4, 3, INV>(v, wc, ws);
}
template <bool INV, typename C> __device__ __forceinline__ void dft24(C *v) {
  const double c15 = 0.96592582628906828675, s15 = 0.258819045102520762349;
  const double h3 = 0.866025403784438646764, h2 = 0.707106781186547524401;
  const double wc[15] = {1.0, c15, h3, h2, 0.5, s15, 0.0, -s15, -0.5, -h2, -h3, -c15, -1.0, -c15, -h3};
  const double ws[15] = {0.0, s15, 0.5, h2, h3, c15, 1.0, c15, h3, h2, 0.5, s15, 0.0, -s15, -0.5};
  dft_split<8, 3, INV>(v, wc, ws);
}

template <int R, bool INV, typename C> __device__ __forceinline__ void dftR(C *v) {
  if constexpr (R == 1) (void)v;
  else if constexpr (R == 2) dft2<INV>(v);
  else if constexpr (R == 3) dft3<INV>(v);
  else if constexpr (R == 4) dft4<INV>(v);
  else if constexpr (R == 8) dft8<INV>(v);
  else if constexpr (R == 12) dft12<INV>(v);
  else if constexpr (R == 16) dft16<INV>(v);
  else dft24<INV>(v);
}

template <int A, int B, bool INV, typename C>
__device__ __forceinline__ void dft_split(C *v, const double *wc, const double *ws) {
  using T = decltype(v[0].x);
  C a[B][A];
#pragma unroll
  for (int n1 = 0; n1 < A; ++n1) {
    C q[B];
#pragma unroll
    for (int n2 = 0; n2 < B; ++n2) q[n2] = v[n1 + A * n2];
    dftR<B, INV>(q);
#pragma unroll
    for (int k2 = 0; k2 < B; ++k2) {
      const int m = n1 * k2;
      a[k2][n1] = m == 0 ? q[k2] : cmul(q[k2], C{(T)wc[m], INV ? (T)ws[m] : -(T)ws[m]});
    }
  }
#pragma unroll
  for (int k2 = 0; k2 < B; ++k2) {
    dftR<A, INV>(a[k2]);
#pragma unroll
    for (int k1 = 0; k1 < A; ++k1) v[k2 + B * k1] = a[k2][k1];
  }
}

// One radix-R stage over `nlines` lines. Element k of line l lives at
// buf[l*ls + k*es]. lfast: consecutive threads take consecutive lines (for the
// [k][line] layouts) instead of consecutive butterflies of one line.
template <int R, bool INV, typename C>
__device__ __forceinline__ void fft_stage(const C *__restrict__ src, C *__restrict__ dst, int N,
                                          int Ns, FastDiv fnb, FastDiv fns, int nlines, int ls,
                                          int es, bool lfast, const C *__restrict__ tw, int tid,
                                          int nthr) {
  const int nb = N / R;
  const int total = nb * nlines;
  const int twstep = N / (Ns * R);
  for (int w = tid; w < total; w += nthr) {
    int l, j;
    if (lfast) {
      l = w % nlines;
      j = w / nlines;
    } else {
      l = fdiv(w, fnb);
      j = w - l * nb;
    }
    const C *s = src + l * ls;
    C *d = dst + l * ls;
    // the multiply-high division pays in the x1 transforms (lines along the
    // workgroup, issue bound); in the column layouts it costs registers and
    // occupancy instead
    const int jm = lfast ? j % Ns : j - fdiv(j, fns) * Ns;
    C v[R];
#pragma unroll
    for (int r = 0; r < R; ++r) v[r] = s[(j + r * nb) * es];
    if (Ns > 1) {
#pragma unroll
      for (int r = 1; r < R; ++r) {
        C t = tw[jm * r * twstep];
        v[r] = INV ? cmulc(v[r], t) : cmul(v[r], t);
      }
    }
    dftR<R, INV>(v);
    const int o = (j - jm) * R + jm;
#pragma unroll
    for (int r = 0; r < R; ++r) d[(o + r * Ns) * es] = v[r];
  }
}

// Transforms every line; a and b are two LDS buffers of the same shape, a
// holds the input. Returns the buffer holding the result. Ends with a barrier.
template <bool INV, typename C>
__device__ C *fft_lines(C *a, C *b, const Plan1D &p, const C *__restrict__ twpool, int nlines,
                        int ls, int es, bool lfast, int tid, int nthr) {
  const C *tw = twpool + p.tw;
  int Ns = 1;
  for (int s = 0; s < p.nst; ++s) {
    const int R = p.rad[s];
    switch (R) {
      case 2:
        fft_stage<2, INV>(a, b, p.n, Ns, p.nb[s], p.ns[s], nlines, ls, es, lfast, tw, tid, nthr);
        break;
      case 3:
        fft_stage<3, INV>(a, b, p.n, Ns, p.nb[s], p.ns[s], nlines, ls, es, lfast, tw, tid, nthr);
        break;
      case 4:
        fft_stage<4, INV>(a, b, p.n, Ns, p.nb[s], p.ns[s], nlines, ls, es, lfast, tw, tid, nthr);
        break;
      default:
        fft_stage<8, INV>(a, b, p.n, Ns, p.nb[s], p.ns[s], nlines, ls, es, lfast, tw, tid, nthr);
        break;
    }
    __syncthreads();
    C *t = a;
    a = b;
    b = t;
    Ns *= R;
  }
  return a;
}

}  // namespace admm
