// HIP kernels of the vdW-DF nonlocal-correlation path (Roman-Perez--Soler form, libvdwxc paper
// Sec. 2-3 and appendix), for gfx950.
//
// Data layout in HBM (N1 x N2 x N3 grid, N3 contiguous, H = N3/2 + 1, f = field index alpha):
//   n, sigma, dedn, dedsigma, v : double [N1][N2][N3]
//   A (z-transformed)           : complex [f][kz][x][y]      (y contiguous)
//   B (z,y-transformed)         : complex [f][ky][kz][x]     (x contiguous)
// Each FFT pass transforms the contiguous axis of its input and writes the transformed axis to
// the slowest position, so every global access is a contiguous run (a line, or a tile row of 16
// elements).  The x pass is done in place in B and carries the k-space contraction between its
// forward and inverse transforms.  Real fields are transformed two at a time as the real and
// imaginary part of one complex line.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "fft_lds.h"

namespace vdwxc {

constexpr int kMaxQ = 20;           // largest supported q-mesh (N_alpha)
constexpr double kVacuum = 1e-30;   // n below this is a vacuum point
constexpr double kPi = 3.14159265358979323846;

// PW92 correlation and the vdW-DF q0 constants (appendix of the paper)
constexpr double kA = 0.031091, kAlpha1 = 0.2137;
constexpr double kB1 = 7.5957, kB2 = 3.5876, kB3 = 1.6382, kB4 = 0.49294;
constexpr double kSatA = 5.0;

struct Geometry {
  int n1, n2, n3, h3;      // grid and half-spectrum length of the contiguous axis
  int M;                   // number of q-mesh points / theta fields
  double zab;              // gradient coefficient of q0 (vdW-DF1 or vdW-DF2)
  double bvec[9];          // reciprocal vectors b1, b2, b3 (rows), bohr^-1
  double kmax, inv_dk;     // kernel table range and inverse node spacing
  int nk;                  // kernel table nodes
};

// ---- q0, saturation and the helper splines (per grid point, FP64) ----------------------------

// q0 of the appendix with the saturation h_5, clamped below the first mesh point.  Returns the
// spline interval b (or -1 for a vacuum point), the position t in it, and n*dq0/dn, n*dq0/dsigma.
__device__ __forceinline__ void q0_state(double n, double sigma, double zab, const double* q, int M,
                                         int& b, double& t, double& ndqdn, double& ndqds) {
  if (!(n >= kVacuum)) {
    b = -1;
    t = 0.0;
    ndqdn = ndqds = 0.0;
    return;
  }
  const double kF = cbrt(3.0 * kPi * kPi * n);
  const double rs = cbrt(3.0 / (4.0 * kPi * n));
  const double sq = sqrt(rs);
  const double Q = 2.0 * kA * (kB1 * sq + kB2 * rs + kB3 * rs * sq + kB4 * rs * rs);
  const double dQ = 2.0 * kA * (0.5 * kB1 / sq + kB2 + 1.5 * kB3 * sq + 2.0 * kB4 * rs);
  const double lg = log1p(1.0 / Q);
  const double eps = -2.0 * kA * (1.0 + kAlpha1 * rs) * lg;
  const double deps = -2.0 * kA * kAlpha1 * lg + 2.0 * kA * (1.0 + kAlpha1 * rs) * dQ / (Q * Q + Q);
  const double inv_kn2 = 1.0 / (kF * n * n);
  const double x = kF - (4.0 * kPi / 3.0) * eps - (zab / 36.0) * sigma * inv_kn2;
  const double tt = x / kSatA;
  double q0, hp;
  if (tt >= 2.0) {          // exp(-S) underflows to exactly zero
    q0 = kSatA;
    hp = 0.0;
  } else {
    double S = 1.0 / 12.0, P = 1.0;
#pragma unroll
    for (int m = 11; m >= 1; --m) S = S * tt + 1.0 / m;
    S *= tt;                                 // sum_{m=1..12} t^m / m
#pragma unroll
    for (int m = 0; m < 11; ++m) P = P * tt + 1.0;   // sum_{m=0..11} t^m
    const double e = exp(-S);
    q0 = kSatA * (1.0 - e);
    hp = e * P;
  }
  if (q0 < q[0]) {
    q0 = q[0];
    hp = 0.0;
  }
  if (hp != 0.0) {
    const double dxdn = kF / (3.0 * n) + (4.0 * kPi / 9.0) * (rs / n) * deps
                      + (7.0 * zab / 108.0) * sigma * inv_kn2 / n;
    const double dxds = -(zab / 36.0) * inv_kn2;
    ndqdn = n * hp * dxdn;
    ndqds = n * hp * dxds;
  } else {
    ndqdn = ndqds = 0.0;
  }
  int lo = 0, hi = M - 2;                   // largest b <= M-2 with q[b] <= q0
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (q[mid] <= q0) lo = mid; else hi = mid - 1;
  }
  b = lo;
  t = (q0 - q[b]) / (q[b + 1] - q[b]);
}

// Natural cubic spline through p_a(q_b) = delta_ab with second derivatives mm[a][b]:
//   p_a = (1-t) d_ab + t d_a,b+1 + h^2/6 [((1-t)^3-(1-t)) mm_ab + (t^3-t) mm_a,b+1]
__device__ __forceinline__ double spline_p(int a, int b, double t, double h, const double* mm, int M) {
  const double u = 1.0 - t;
  double p = h * h * (1.0 / 6.0) * ((u * u * u - u) * mm[a * M + b] + (t * t * t - t) * mm[a * M + b + 1]);
  if (a == b) p += u;
  if (a == b + 1) p += t;
  return p;
}
__device__ __forceinline__ double spline_dp(int a, int b, double t, double h, const double* mm, int M) {
  const double u = 1.0 - t;
  double d = h * (1.0 / 6.0) * (-(3.0 * u * u - 1.0) * mm[a * M + b] + (3.0 * t * t - 1.0) * mm[a * M + b + 1]);
  if (a == b) d -= 1.0 / h;
  if (a == b + 1) d += 1.0 / h;
  return d;
}

__device__ __forceinline__ size_t a_index(const Geometry& g, int f, int kz, int x, int y) {
  return ((size_t(f) * g.h3 + kz) * g.n1 + x) * g.n2 + y;
}
__device__ __forceinline__ size_t b_index(const Geometry& g, int f, int ky, int kz, int x) {
  return ((size_t(f) * g.n2 + ky) * g.h3 + kz) * g.n1 + x;
}

// Split the z-spectrum Z = FFT(a + i b) of two real lines into their half spectra at index k:
// X_a = (Z_k + conj Z_{-k})/2, X_b = (Z_k - conj Z_{-k})/(2i).
template <typename T2>
__device__ __forceinline__ void split_pair(T2 zk, T2 zn, T2& xa, T2& xb) {
  using T = decltype(zk.x);
  const T half = T(0.5);
  xa = T2{half * (zk.x + zn.x), half * (zk.y - zn.y)};
  xb = T2{half * (zk.y + zn.y), half * (zn.x - zk.x)};
}

// ---- pass 1: q0 + splines + forward z FFT (theta fields) ------------------------------------
// Block: one x plane, TY consecutive y lines (blockIdx.x = y tile, blockIdx.y = x).

template <typename T, int PPT, int EPT, bool SIGMA_FROM_GRAD>
__global__ void __launch_bounds__(512)
k_theta_zfwd(const double* __restrict__ nden, const double* __restrict__ sig,
             typename Cx<T>::type* __restrict__ A, int* __restrict__ flag,
             const double* __restrict__ qmesh, const double* __restrict__ mm,
             const typename Cx<T>::type* __restrict__ tw, Geometry g, AxisPlan zp, int ty, int lstride) {
  using T2 = typename Cx<T>::type;
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ double s_q[kMaxQ];
  __shared__ double s_mm[kMaxQ * kMaxQ];
  T2* line = reinterpret_cast<T2*>(smem);
  const int tid = threadIdx.x, nthr = blockDim.x;
  const int x = blockIdx.y, y0 = blockIdx.x * ty;
  const int n3 = g.n3, M = g.M;
  const size_t N = size_t(g.n1) * g.n2 * n3;
  for (int i = tid; i < M; i += nthr) s_q[i] = qmesh[i];
  for (int i = tid; i < M * M; i += nthr) s_mm[i] = mm[i];
  __syncthreads();

  const int npts = ty * n3;
  int pb[PPT];
  double pt[PPT], pn[PPT];
  bool bad = false;
#pragma unroll
  for (int c = 0; c < PPT; ++c) {
    const int p = tid + c * nthr;
    pb[c] = -1;
    pt[c] = 0.0;
    pn[c] = 0.0;
    if (p < npts) {
      const int yl = p / n3, z = p - yl * n3, y = y0 + yl;
      if (y < g.n2) {
        const size_t idx = (size_t(x) * g.n2 + y) * n3 + z;
        const double nv = nden[idx];
        double sv;
        if (SIGMA_FROM_GRAD) {
          const double gx = sig[idx], gy = sig[N + idx], gz = sig[2 * N + idx];
          sv = gx * gx + gy * gy + gz * gz;
        } else {
          sv = sig[idx];
        }
        bad |= !(nv == nv) || !(sv == sv);
        double d1, d2;
        q0_state(nv, sv, g.zab, s_q, M, pb[c], pt[c], d1, d2);
        pn[c] = nv;
      }
    }
  }
  if (bad) *flag = 1;

  const int npairs = (M + 1) >> 1;
  for (int pr = 0; pr < npairs; ++pr) {
    const int fa = 2 * pr, fb = 2 * pr + 1;
#pragma unroll
    for (int c = 0; c < PPT; ++c) {
      const int p = tid + c * nthr;
      if (p < npts) {
        const int yl = p / n3, z = p - yl * n3;
        double ta = 0.0, tb = 0.0;
        const int b = pb[c];
        if (b >= 0) {
          const double h = s_q[b + 1] - s_q[b];
          ta = pn[c] * spline_p(fa, b, pt[c], h, s_mm, M);
          if (fb < M) tb = pn[c] * spline_p(fb, b, pt[c], h, s_mm, M);
        }
        line[yl * lstride + z] = T2{T(ta), T(tb)};
      }
    }
    __syncthreads();
    lds_fft<EPT, -1>(line, zp, ty, lstride, tw, tid, nthr);
    const int nout = ty * g.h3;
    for (int e = tid; e < nout; e += nthr) {
      const int yl = e % ty, kz = e / ty, y = y0 + yl;
      if (y < g.n2) {
        const T2 zk = line[yl * lstride + kz];
        const T2 zn = line[yl * lstride + (kz == 0 ? 0 : n3 - kz)];
        T2 xa, xb;
        split_pair(zk, zn, xa, xb);
        A[a_index(g, fa, kz, x, y)] = xa;
        if (fb < M) A[a_index(g, fb, kz, x, y)] = xb;
      }
    }
    __syncthreads();
  }
}

// ---- pass 1 for plain real fields (spectral gradient / divergence inputs) --------------------
// MODE 0: nf fields read from src[f*N + idx].  MODE 1: the three fields 2*S*g_c (divergence
// input), S = dE/dsigma (src) and g the gradient (aux, [3][N]).

template <typename T, int EPT, int MODE>
__global__ void __launch_bounds__(512)
k_real_zfwd(const double* __restrict__ src, const double* __restrict__ aux, int nf,
            typename Cx<T>::type* __restrict__ A, const typename Cx<T>::type* __restrict__ tw,
            Geometry g, AxisPlan zp, int ty, int lstride) {
  using T2 = typename Cx<T>::type;
  extern __shared__ __align__(16) unsigned char smem[];
  T2* line = reinterpret_cast<T2*>(smem);
  const int tid = threadIdx.x, nthr = blockDim.x;
  const int x = blockIdx.y, y0 = blockIdx.x * ty;
  const int n3 = g.n3;
  const size_t N = size_t(g.n1) * g.n2 * n3;
  const int npts = ty * n3;
  for (int fa = 0; fa < nf; fa += 2) {
    const int fb = fa + 1;
    for (int p = tid; p < npts; p += nthr) {
      const int yl = p / n3, z = p - yl * n3, y = y0 + yl;
      double va = 0.0, vb = 0.0;
      if (y < g.n2) {
        const size_t idx = (size_t(x) * g.n2 + y) * n3 + z;
        if (MODE == 0) {
          va = src[size_t(fa) * N + idx];
          if (fb < nf) vb = src[size_t(fb) * N + idx];
        } else {
          const double s2 = 2.0 * src[idx];
          va = s2 * aux[size_t(fa) * N + idx];
          if (fb < nf) vb = s2 * aux[size_t(fb) * N + idx];
        }
      }
      line[yl * lstride + z] = T2{T(va), T(vb)};
    }
    __syncthreads();
    lds_fft<EPT, -1>(line, zp, ty, lstride, tw, tid, nthr);
    const int nout = ty * g.h3;
    for (int e = tid; e < nout; e += nthr) {
      const int yl = e % ty, kz = e / ty, y = y0 + yl;
      if (y < g.n2) {
        const T2 zk = line[yl * lstride + kz];
        const T2 zn = line[yl * lstride + (kz == 0 ? 0 : n3 - kz)];
        T2 xa, xb;
        split_pair(zk, zn, xa, xb);
        A[a_index(g, fa, kz, x, y)] = xa;
        if (fb < nf) A[a_index(g, fb, kz, x, y)] = xb;
      }
    }
    __syncthreads();
  }
}

// ---- pass 2 / 4: y FFT with rotation A[f][kz][x][y] <-> B[f][ky][kz][x] ----------------------
// Block: TX consecutive x of one (f, kz) (blockIdx.x = x tile, .y = kz, .z = f).

template <typename T, int EPT, int DIR>
__global__ void __launch_bounds__(512)
k_ypass(const typename Cx<T>::type* __restrict__ src, typename Cx<T>::type* __restrict__ dst,
        const typename Cx<T>::type* __restrict__ tw, Geometry g, AxisPlan yp, int tx, int lstride) {
  using T2 = typename Cx<T>::type;
  extern __shared__ __align__(16) unsigned char smem[];
  T2* line = reinterpret_cast<T2*>(smem);
  const int tid = threadIdx.x, nthr = blockDim.x;
  const int x0 = blockIdx.x * tx, kz = blockIdx.y, f = blockIdx.z;
  const int n2 = g.n2, tot = tx * n2;
  if (DIR < 0) {
    const size_t base = a_index(g, f, kz, x0, 0);
    for (int e = tid; e < tot; e += nthr) {
      const int xl = e / n2, y = e - xl * n2;
      line[xl * lstride + y] = (x0 + xl < g.n1) ? src[base + e] : T2{T(0), T(0)};
    }
  } else {
    for (int e = tid; e < tot; e += nthr) {
      const int xl = e % tx, ky = e / tx;
      line[xl * lstride + ky] = (x0 + xl < g.n1) ? src[b_index(g, f, ky, kz, x0 + xl)] : T2{T(0), T(0)};
    }
  }
  __syncthreads();
  lds_fft<EPT, DIR>(line, yp, tx, lstride, tw, tid, nthr);
  if (DIR < 0) {
    for (int e = tid; e < tot; e += nthr) {
      const int xl = e % tx, ky = e / tx;
      if (x0 + xl < g.n1) dst[b_index(g, f, ky, kz, x0 + xl)] = line[xl * lstride + ky];
    }
  } else {
    const size_t base = a_index(g, f, kz, x0, 0);
    for (int e = tid; e < tot; e += nthr) {
      const int xl = e / n2, y = e - xl * n2;
      if (x0 + xl < g.n1) dst[base + e] = line[xl * lstride + y];
    }
  }
}

// signed frequency of index m on an axis of length n, and whether it is the Nyquist index
__device__ __forceinline__ int signed_freq(int m, int n) { return m <= n / 2 ? m : m - n; }
__device__ __forceinline__ bool is_nyquist(int m, int n) { return (n % 2 == 0) && (m == n / 2); }

// |G|^2 with the Nyquist components added in quadrature to the rest (even in G)
__device__ __forceinline__ double gnorm2(const Geometry& g, int kx, int ky, int kz) {
  double reg[3] = {0.0, 0.0, 0.0}, nyq[3] = {0.0, 0.0, 0.0};
  const int m[3] = {kx, ky, kz};
  const int n[3] = {g.n1, g.n2, g.n3};
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    const double f = double(signed_freq(m[i], n[i]));
    double* acc = is_nyquist(m[i], n[i]) ? nyq : reg;
#pragma unroll
    for (int c = 0; c < 3; ++c) acc[c] += f * g.bvec[3 * i + c];
  }
  return reg[0] * reg[0] + reg[1] * reg[1] + reg[2] * reg[2] + nyq[0] * nyq[0] + nyq[1] * nyq[1] + nyq[2] * nyq[2];
}

// ---- pass 3: x FFT, k-space contraction, inverse x FFT (in place in B) -----------------------
// Block: the M field lines of one (ky, kz) column (blockIdx.x = ky, .y = kz).
// Per k: phi_ab = (1-w) T_j,ab + w T_j+1,ab with |G| = (j + w) dk; F_a = sum_b phi_ab theta_b;
// energy weight 2 for kz strictly inside the half spectrum, 1 on its edges.

template <typename T, int EPT>
__global__ void __launch_bounds__(512)
k_xcontract(typename Cx<T>::type* __restrict__ B, const T* __restrict__ table,
            double* __restrict__ partials, const typename Cx<T>::type* __restrict__ tw,
            Geometry g, AxisPlan xp) {
  using T2 = typename Cx<T>::type;
  extern __shared__ __align__(16) unsigned char smem[];
  T2* line = reinterpret_cast<T2*>(smem);
  const int tid = threadIdx.x, nthr = blockDim.x;
  const int ky = blockIdx.x, kz = blockIdx.y, M = g.M, n1 = g.n1;
  for (int e = tid; e < M * n1; e += nthr) {
    const int f = e / n1, x = e - f * n1;
    line[e] = B[b_index(g, f, ky, kz, x)];
  }
  __syncthreads();
  const int G = (nthr * EPT) / n1;   // lines per batched transform
  for (int l0 = 0; l0 < M; l0 += G) lds_fft<EPT, -1>(line + l0 * n1, xp, min(G, M - l0), n1, tw, tid, nthr);

  const double wz = (kz == 0 || is_nyquist(kz, g.n3)) ? 1.0 : 2.0;
  const int MM = M * M;
  double esum = 0.0;
  for (int kx = tid; kx < n1; kx += nthr) {
    const double kn = sqrt(gnorm2(g, kx, ky, kz));
    T2 th[kMaxQ];
#pragma unroll
    for (int b = 0; b < kMaxQ; ++b) th[b] = b < M ? line[b * n1 + kx] : T2{T(0), T(0)};
    const bool inside = kn < g.kmax;
    const double s = kn * g.inv_dk;
    int j = inside ? int(floor(s)) : 0;
    if (j > g.nk - 2) j = g.nk - 2;
    const T w = T(inside ? s - j : 0.0);
    const T w0 = inside ? T(1) - w : T(0);
    const T w1 = inside ? w : T(0);
    const T* t0 = table + size_t(j) * MM;
    const T* t1 = t0 + MM;
    double e = 0.0;
#pragma unroll
    for (int a = 0; a < kMaxQ; ++a) {
      if (a < M) {
        T2 F = T2{T(0), T(0)};
#pragma unroll
        for (int b = 0; b < kMaxQ; ++b) {
          if (b < M) {
            const T phi = w0 * t0[a * M + b] + w1 * t1[a * M + b];
            F.x += phi * th[b].x;
            F.y += phi * th[b].y;
          }
        }
        e += double(th[a].x) * double(F.x) + double(th[a].y) * double(F.y);
        line[a * n1 + kx] = F;
      }
    }
    esum += wz * e;
  }
  __syncthreads();
  for (int l0 = 0; l0 < M; l0 += G) lds_fft<EPT, +1>(line + l0 * n1, xp, min(G, M - l0), n1, tw, tid, nthr);
  for (int e = tid; e < M * n1; e += nthr) {
    const int f = e / n1, x = e - f * n1;
    B[b_index(g, f, ky, kz, x)] = line[e];
  }
  // block sum of the energy, fixed order: wave shuffles, then the waves in order
  for (int off = 32; off > 0; off >>= 1) esum += __shfl_xor(esum, off, 64);
  __syncthreads();
  double* red = reinterpret_cast<double*>(smem);
  if ((tid & 63) == 0) red[tid >> 6] = esum;
  __syncthreads();
  if (tid == 0) {
    double s = 0.0;
    for (int w = 0; w < (nthr + 63) / 64; ++w) s += red[w];
    partials[size_t(kz) * g.n2 + ky] = s;
  }
}

// ---- pass 3 for the spectral gradient (1 -> 3 fields) and divergence (3 -> 1) ----------------
// D_c f = IFFT(i G_c FFT f) with every frequency touching a Nyquist index set to zero.

template <typename T, int EPT, int NIN, int NOUT>
__global__ void __launch_bounds__(512)
k_xspectral(typename Cx<T>::type* __restrict__ B, const typename Cx<T>::type* __restrict__ tw,
            Geometry g, AxisPlan xp) {
  using T2 = typename Cx<T>::type;
  extern __shared__ __align__(16) unsigned char smem[];
  T2* line = reinterpret_cast<T2*>(smem);
  const int tid = threadIdx.x, nthr = blockDim.x;
  const int ky = blockIdx.x, kz = blockIdx.y, n1 = g.n1;
  for (int e = tid; e < NIN * n1; e += nthr) {
    const int f = e / n1, x = e - f * n1;
    line[e] = B[b_index(g, f, ky, kz, x)];
  }
  __syncthreads();
  const int G = (nthr * EPT) / n1;
  for (int l0 = 0; l0 < NIN; l0 += G) lds_fft<EPT, -1>(line + l0 * n1, xp, min(G, NIN - l0), n1, tw, tid, nthr);
  const bool nyq_yz = is_nyquist(ky, g.n2) || is_nyquist(kz, g.n3);
  const double fy = signed_freq(ky, g.n2), fz = signed_freq(kz, g.n3);
  for (int kx = tid; kx < n1; kx += nthr) {
    const bool zero = nyq_yz || is_nyquist(kx, n1);
    const double fx = signed_freq(kx, n1);
    double G[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) G[c] = fx * g.bvec[c] + fy * g.bvec[3 + c] + fz * g.bvec[6 + c];
    T2 in[NIN];
#pragma unroll
    for (int f = 0; f < NIN; ++f) in[f] = line[f * n1 + kx];
    if (NIN == 1) {
#pragma unroll
      for (int c = 0; c < NOUT; ++c) {   // i G_c X
        const T gc = zero ? T(0) : T(G[c]);
        line[c * n1 + kx] = T2{-gc * in[0].y, gc * in[0].x};
      }
    } else {
      T2 acc = T2{T(0), T(0)};
#pragma unroll
      for (int c = 0; c < NIN; ++c) {    // sum_c i G_c X_c
        const T gc = zero ? T(0) : T(G[c]);
        acc.x -= gc * in[c].y;
        acc.y += gc * in[c].x;
      }
      line[kx] = acc;
    }
  }
  __syncthreads();
  for (int l0 = 0; l0 < NOUT; l0 += G) lds_fft<EPT, +1>(line + l0 * n1, xp, min(G, NOUT - l0), n1, tw, tid, nthr);
  for (int e = tid; e < NOUT * n1; e += nthr) {
    const int f = e / n1, x = e - f * n1;
    B[b_index(g, f, ky, kz, x)] = line[e];
  }
}

// Rebuild the full complex z-line Z = X_a + i X_b of a field pair from their half spectra (the
// imaginary parts of the k = 0 and Nyquist terms are dropped, as a complex-to-real transform does).
template <typename T2>
__device__ __forceinline__ void load_pair_line(const T2* __restrict__ A, const Geometry& g, int fa, int fb,
                                               int x, int y0, int ty, T2* line, int lstride, int tid, int nthr) {
  using T = decltype(line[0].x);
  const int n3 = g.n3, tot = ty * g.h3;
  for (int e = tid; e < tot; e += nthr) {
    const int yl = e % ty, kz = e / ty, y = y0 + yl;
    T2 xa = T2{T(0), T(0)}, xb = T2{T(0), T(0)};
    if (y < g.n2) {
      xa = A[a_index(g, fa, kz, x, y)];
      if (fb >= 0) xb = A[a_index(g, fb, kz, x, y)];
    }
    const bool edge = (kz == 0) || is_nyquist(kz, n3);
    if (edge) {
      xa.y = T(0);
      xb.y = T(0);
    }
    line[yl * lstride + kz] = T2{xa.x - xb.y, xa.y + xb.x};
    if (!edge) line[yl * lstride + (n3 - kz)] = T2{xa.x + xb.y, xb.x - xa.y};
  }
}

// ---- pass 5: inverse z FFT + assembly of dE/dn, dE/dsigma (eqs. dedn, dedsigma) -------------

template <typename T, int PPT, int EPT, bool SIGMA_FROM_GRAD>
__global__ void __launch_bounds__(512)
k_zinv_assemble(const typename Cx<T>::type* __restrict__ A, const double* __restrict__ nden,
                const double* __restrict__ sig, double* __restrict__ dedn, double* __restrict__ dedsig,
                const double* __restrict__ qmesh, const double* __restrict__ mm,
                const typename Cx<T>::type* __restrict__ tw, Geometry g, AxisPlan zp, int ty, int lstride) {
  using T2 = typename Cx<T>::type;
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ double s_q[kMaxQ];
  __shared__ double s_mm[kMaxQ * kMaxQ];
  T2* line = reinterpret_cast<T2*>(smem);
  const int tid = threadIdx.x, nthr = blockDim.x;
  const int x = blockIdx.y, y0 = blockIdx.x * ty;
  const int n3 = g.n3, M = g.M;
  const size_t N = size_t(g.n1) * g.n2 * n3;
  for (int i = tid; i < M; i += nthr) s_q[i] = qmesh[i];
  for (int i = tid; i < M * M; i += nthr) s_mm[i] = mm[i];
  __syncthreads();

  const int npts = ty * n3;
  int pb[PPT];
  double pt[PPT], pdn[PPT], pds[PPT], acc_n[PPT], acc_s[PPT];
#pragma unroll
  for (int c = 0; c < PPT; ++c) {
    const int p = tid + c * nthr;
    pb[c] = -1;
    pt[c] = pdn[c] = pds[c] = 0.0;
    acc_n[c] = acc_s[c] = 0.0;
    if (p < npts) {
      const int yl = p / n3, z = p - yl * n3, y = y0 + yl;
      if (y < g.n2) {
        const size_t idx = (size_t(x) * g.n2 + y) * n3 + z;
        const double nv = nden[idx];
        double sv;
        if (SIGMA_FROM_GRAD) {
          const double gx = sig[idx], gy = sig[N + idx], gz = sig[2 * N + idx];
          sv = gx * gx + gy * gy + gz * gz;
        } else {
          sv = sig[idx];
        }
        q0_state(nv, sv, g.zab, s_q, M, pb[c], pt[c], pdn[c], pds[c]);
      }
    }
  }

  const int npairs = (M + 1) >> 1;
  for (int pr = 0; pr < npairs; ++pr) {
    const int fa = 2 * pr, fb = 2 * pr + 1 < M ? 2 * pr + 1 : -1;
    load_pair_line(A, g, fa, fb, x, y0, ty, line, lstride, tid, nthr);
    __syncthreads();
    lds_fft<EPT, +1>(line, zp, ty, lstride, tw, tid, nthr);
#pragma unroll
    for (int c = 0; c < PPT; ++c) {
      const int p = tid + c * nthr;
      const int b = pb[c];
      if (p < npts && b >= 0) {
        const int yl = p / n3, z = p - yl * n3;
        const T2 F = line[yl * lstride + z];
        const double h = s_q[b + 1] - s_q[b];
        const double pa = spline_p(fa, b, pt[c], h, s_mm, M);
        const double dpa = spline_dp(fa, b, pt[c], h, s_mm, M);
        acc_n[c] += double(F.x) * (pa + pdn[c] * dpa);
        acc_s[c] += double(F.x) * (pds[c] * dpa);
        if (fb >= 0) {
          const double pbv = spline_p(fb, b, pt[c], h, s_mm, M);
          const double dpb = spline_dp(fb, b, pt[c], h, s_mm, M);
          acc_n[c] += double(F.y) * (pbv + pdn[c] * dpb);
          acc_s[c] += double(F.y) * (pds[c] * dpb);
        }
      }
    }
    __syncthreads();
  }
  const double invN = 1.0 / double(N);
#pragma unroll
  for (int c = 0; c < PPT; ++c) {
    const int p = tid + c * nthr;
    if (p < npts) {
      const int yl = p / n3, z = p - yl * n3, y = y0 + yl;
      if (y < g.n2) {
        const size_t idx = (size_t(x) * g.n2 + y) * n3 + z;
        dedn[idx] = acc_n[c] * invN;
        dedsig[idx] = acc_s[c] * invN;
      }
    }
  }
}

// ---- pass 5 for plain real fields: out[f] = IFFT/N (COMBINE: out[0] -= IFFT/N) -------------

template <typename T, int EPT, bool COMBINE>
__global__ void __launch_bounds__(512)
k_real_zinv(const typename Cx<T>::type* __restrict__ A, int nf, double* __restrict__ out,
            const typename Cx<T>::type* __restrict__ tw, Geometry g, AxisPlan zp, int ty, int lstride) {
  using T2 = typename Cx<T>::type;
  extern __shared__ __align__(16) unsigned char smem[];
  T2* line = reinterpret_cast<T2*>(smem);
  const int tid = threadIdx.x, nthr = blockDim.x;
  const int x = blockIdx.y, y0 = blockIdx.x * ty;
  const int n3 = g.n3;
  const size_t N = size_t(g.n1) * g.n2 * n3;
  const double invN = 1.0 / double(N);
  const int npts = ty * n3;
  for (int fa = 0; fa < nf; fa += 2) {
    const int fb = fa + 1 < nf ? fa + 1 : -1;
    load_pair_line(A, g, fa, fb, x, y0, ty, line, lstride, tid, nthr);
    __syncthreads();
    lds_fft<EPT, +1>(line, zp, ty, lstride, tw, tid, nthr);
    for (int p = tid; p < npts; p += nthr) {
      const int yl = p / n3, z = p - yl * n3, y = y0 + yl;
      if (y < g.n2) {
        const size_t idx = (size_t(x) * g.n2 + y) * n3 + z;
        const T2 v = line[yl * lstride + z];
        if (COMBINE) {
          out[idx] -= double(v.x) * invN;
        } else {
          out[size_t(fa) * N + idx] = double(v.x) * invN;
          if (fb >= 0) out[size_t(fb) * N + idx] = double(v.y) * invN;
        }
      }
    }
    __syncthreads();
  }
}

// ---- energy: fixed-order sum of the per-column partials --------------------------------------

__global__ void __launch_bounds__(512)
k_energy_reduce(const double* __restrict__ partials, int nparts, double scale,
                const int* __restrict__ flag, double* __restrict__ out) {
  __shared__ double red[16];
  const int tid = threadIdx.x;
  double s = 0.0;
  for (int i = tid; i < nparts; i += blockDim.x) s += partials[i];
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
  if ((tid & 63) == 0) red[tid >> 6] = s;
  __syncthreads();
  if (tid == 0) {
    double tot = 0.0;
    for (int w = 0; w < (int(blockDim.x) + 63) / 64; ++w) tot += red[w];
    out[0] = (*flag != 0) ? __builtin_nan("") : tot * scale;
  }
}

__global__ void k_clear_flag(int* flag) {
  if (threadIdx.x == 0) *flag = 0;
}

}  // namespace vdwxc
