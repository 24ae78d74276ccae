// HIP kernels of the vdW-DF nonlocal-correlation path (Roman-Perez--Soler form, libvdwxc paper
// Sec. 2-3 and appendix), for gfx950.
//
// Data layout in HBM (N1 x N2 x N3 grid, N3 contiguous, H = N3/2 + 1, f = field index alpha):
//   n, sigma, dedn, dedsigma, v : double [N1][N2][N3]
//   A (z-transformed)           : complex [f][x][kz][y]      (y contiguous)
//   B (z,y-transformed)         : complex [f][kz][ky][x]     (x contiguous)
// Each FFT pass transforms the contiguous axis of its input and writes the transformed axis out
// of the contiguous position, so every global access is a contiguous run (a line, or a tile row
// of 16 elements).  The x pass is done in place in B and carries the k-space contraction between its
// forward and inverse transforms.  Real fields are transformed two at a time as the real and
// imaginary part of one complex line.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

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
  double bn2[3];           // |b_i|^2 (used when the cell is orthogonal)
  int xpair;               // |G| even in kx, bitwise, with N1 even: paired table reads (contraction)
};

// four values of the path's precision in one aligned load: a kernel-table entry, or the spline
// state of a grid point
template <typename T>
struct alignas(4 * sizeof(T)) Quad {
  T x, y, z, w;
};

// Non-temporal loads and stores, for data a pass touches once: they do not displace what the
// caches should keep (the kernel table of the contraction).  ld<NT> / st<NT> pick them or plain
// accesses at compile time.
typedef double nt_double2 __attribute__((ext_vector_type(2)));
typedef float nt_float2 __attribute__((ext_vector_type(2)));
typedef double nt_double4 __attribute__((ext_vector_type(4)));
typedef float nt_float4 __attribute__((ext_vector_type(4)));
__device__ __forceinline__ double2 nt_load(const double2* p) {
  const nt_double2 v = __builtin_nontemporal_load(reinterpret_cast<const nt_double2*>(p));
  return double2{v.x, v.y};
}
__device__ __forceinline__ float2 nt_load(const float2* p) {
  const nt_float2 v = __builtin_nontemporal_load(reinterpret_cast<const nt_float2*>(p));
  return float2{v.x, v.y};
}
__device__ __forceinline__ Quad<double> nt_load(const Quad<double>* p) {
  const nt_double4 v = __builtin_nontemporal_load(reinterpret_cast<const nt_double4*>(p));
  return Quad<double>{v.x, v.y, v.z, v.w};
}
__device__ __forceinline__ Quad<float> nt_load(const Quad<float>* p) {
  const nt_float4 v = __builtin_nontemporal_load(reinterpret_cast<const nt_float4*>(p));
  return Quad<float>{v.x, v.y, v.z, v.w};
}
__device__ __forceinline__ void nt_store(double2* p, double2 v) {
  __builtin_nontemporal_store(nt_double2{v.x, v.y}, reinterpret_cast<nt_double2*>(p));
}
__device__ __forceinline__ void nt_store(float2* p, float2 v) {
  __builtin_nontemporal_store(nt_float2{v.x, v.y}, reinterpret_cast<nt_float2*>(p));
}
__device__ __forceinline__ void nt_store(Quad<double>* p, Quad<double> v) {
  __builtin_nontemporal_store(nt_double4{v.x, v.y, v.z, v.w}, reinterpret_cast<nt_double4*>(p));
}
__device__ __forceinline__ void nt_store(Quad<float>* p, Quad<float> v) {
  __builtin_nontemporal_store(nt_float4{v.x, v.y, v.z, v.w}, reinterpret_cast<nt_float4*>(p));
}
__device__ __forceinline__ double nt_load(const double* p) { return __builtin_nontemporal_load(p); }
__device__ __forceinline__ void nt_store(double* p, double v) { __builtin_nontemporal_store(v, p); }
__device__ __forceinline__ void nt_store(float* p, float v) { __builtin_nontemporal_store(v, p); }
__device__ __forceinline__ void nt_store(unsigned char* p, unsigned char v) { __builtin_nontemporal_store(v, p); }
template <bool NT, typename V>
__device__ __forceinline__ V ld(const V* p) {
  if constexpr (NT) return nt_load(p);
  else return *p;
}
template <bool NT, typename V>
__device__ __forceinline__ void st(V* p, V v) {
  if constexpr (NT) nt_store(p, v);
  else *p = v;
}
// the contraction pass's column accesses
#ifndef VDWXC_XNT
#define VDWXC_XNT 1
#endif
constexpr bool kNtX = VDWXC_XNT;
// the streaming accesses of the other passes, per site and precision (bit masks of NtSite)
enum NtSite {
  kNtThetaOut = 1,    // theta pass: half spectra and spline state
  kNtYfLoad = 2,      // forward y pass: A lines
  kNtYfStore = 4,     // forward y pass: B rows
  kNtYiLoad = 8,      // inverse y pass: B rows
  kNtYiStore = 16,    // inverse y pass: A lines
  kNtAsmA = 32,       // assembly: half spectra
  kNtAsmState = 64,   // assembly: spline state
  kNtAsmOut = 128,    // assembly: dE/dn, dE/dsigma
  kNtDivZLoad = 256,  // z divergence pass: dE/dsigma and the gradient
  kNtDivZStore = 512, // z divergence pass: its three outputs
  kNtThetaIn = 1024,  // theta pass: density and gradient (or sigma)
  kNtThetaSb = 2048   // theta pass: the spline interval bytes
};
// (at 512^3: FP64 theta, y and contraction 52.2 -> 50.7 ms/step with sites 1-16; FP32 30.4 -> 30.0
// with sites 1-4, z divergence 1.09 -> 0.99 ms FP32 with its sites (FP64: 1.89 -> 1.96, so not
// there).  Non-temporal reads of the assembly's half spectra, and of the FP32 inverse y pass's rows,
// were slower: 7.25 -> 7.45 ms and 5.2 -> 6.6 ms, 4.2 -> 4.6 ms.  The theta pass's inputs and
// interval bytes and the assembly's state and outputs measured equal within the run-to-run spread.)
#ifndef VDWXC_NT64
#define VDWXC_NT64 (kNtThetaOut | kNtYfLoad | kNtYfStore | kNtYiLoad | kNtYiStore)
#endif
#ifndef VDWXC_NT32
#define VDWXC_NT32 (kNtThetaOut | kNtYfLoad | kNtYfStore | kNtDivZLoad | kNtDivZStore)
#endif
template <typename T, int SITE>
constexpr bool nt_site() {
  return (((sizeof(T) == 8) ? VDWXC_NT64 : VDWXC_NT32) & SITE) != 0;
}

// ---- q0, saturation and the helper splines (per grid point, FP64) ----------------------------

// PW92 LDA correlation energy per electron eps_c(r_s) of the paper's appendix (spin-paired) and
// its derivative d eps_c / d r_s
__device__ __forceinline__ void pw92(double rs, double& eps, double& deps) {
  const double sq = sqrt(rs);
  const double Q = 2.0 * kA * (kB1 * sq + kB2 * rs + kB3 * rs * sq + kB4 * rs * rs);
  const double dQ = 2.0 * kA * (0.5 * kB1 / sq + kB2 + 1.5 * kB3 * sq + 2.0 * kB4 * rs);
  const double iQ = 1.0 / Q;
  const double lg = log1p(iQ);
  eps = -2.0 * kA * (1.0 + kAlpha1 * rs) * lg;
  deps = -2.0 * kA * kAlpha1 * lg + 2.0 * kA * (1.0 + kAlpha1 * rs) * dQ * iQ / (Q + 1.0);
}

// r_s = (3 / (4 pi n))^(1/3) through k_F = (3 pi^2 n)^(1/3): k_F r_s = (9 pi / 4)^(1/3)
constexpr double kRsKf = 1.9191582926775130066248;

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
  // k_F r_s = (9 pi / 4)^(1/3), so one cube root and two reciprocals serve all the divisions
  const double kF = cbrt(3.0 * kPi * kPi * n);
  const double inv_n = 1.0 / n, inv_kF = 1.0 / kF;
  const double rs = kRsKf * inv_kF;
  double eps, deps;
  pw92(rs, eps, deps);
  const double inv_kn2 = inv_kF * inv_n * inv_n;
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
    const double dxdn = (1.0 / 3.0) * kF * inv_n + (4.0 * kPi / 9.0) * rs * inv_n * deps
                      + (7.0 * zab / 108.0) * sigma * inv_kn2 * inv_n;
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

// A: [f][x][kz][y].  A z-pass block (one x, a tile of y) then writes and reads rows that lie in one
// H*N2 window of a field instead of N1*N2 apart, which keeps its address translations few
__device__ __forceinline__ size_t a_index(const Geometry& g, int f, int kz, int x, int y) {
  return ((size_t(f) * g.n1 + x) * g.h3 + kz) * g.n2 + y;
}
// B: [f][kz][ky][x].  With ky inside kz, the rows a y-pass block writes (one per ky, for its kz
// and x tile) lie in one N2*N1 window of a field instead of N1*H apart, which keeps the pass's
// address translations few
__device__ __forceinline__ size_t b_index(const Geometry& g, int f, int ky, int kz, int x) {
  return ((size_t(f) * g.h3 + kz) * g.n2 + ky) * g.n1 + x;
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

#ifndef VDWXC_THETA_U
#define VDWXC_THETA_U 2   // density/gradient loads in flight per thread in the theta pass
#endif

// Minimum waves per SIMD requested from the register allocator, per kernel (1: no constraint).
// The theta pass needs <= 128 VGPRs so that two 512-thread blocks share a CU at N3 = 512.
#ifndef VDWXC_WPE_THETA
#define VDWXC_WPE_THETA 4
#endif
#ifndef VDWXC_WPE_Y
#define VDWXC_WPE_Y 1
#endif
#ifndef VDWXC_WPE_ASM
#define VDWXC_WPE_ASM 4   // FP32 assembly: <= 128 VGPRs, two 512-thread blocks per CU
#endif

// ---- strided gathers with several loads in flight -------------------------------------------
// Thread tid handles the elements e = tid, tid + nthr, ... of [0, tot).  Each group of U of them
// is loaded first (get returns the raw loaded values, with no arithmetic that would have to wait
// for them) and consumed after (put), so a thread keeps U independent global loads in flight
// instead of waiting on each in turn.
template <int U, typename Get, typename Put>
__device__ __forceinline__ void gather_strided(int tid, int nthr, int tot, Get get, Put put) {
  using V = decltype(get(0));
#pragma unroll 1
  for (int e0 = tid; e0 < tot; e0 += U * nthr) {
    V r[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int e = e0 + u * nthr;
      if (e < tot) r[u] = get(e);
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int e = e0 + u * nthr;
      if (e < tot) put(e, r[u]);
    }
  }
}

// (q, r) = divmod(e, d) for e = e0, e0 + step, e0 + 2 step, ..., advanced by additions only
struct DivModStep {
  int q, r, dq, dr, d;
  __device__ __forceinline__ DivModStep(int e0, int step, int d_) : d(d_) {
    q = e0 / d;
    r = e0 - q * d;
    dq = step / d;
    dr = step - dq * d;
  }
  __device__ __forceinline__ void next() {
    q += dq;
    r += dr;
    if (r >= d) {
      r -= d;
      ++q;
    }
  }
};

// gather_strided over a 2-D index: get(e, q, r) / put(e, q, r, v) receive (q, r) = divmod(e, d)
template <int U, typename Get, typename Put>
__device__ __forceinline__ void gather_strided_dm(int tid, int nthr, int tot, int d, Get get, Put put) {
  using V = decltype(get(0, 0, 0));
  DivModStep it(tid, nthr, d);
#pragma unroll 1
  for (int e0 = tid; e0 < tot; e0 += U * nthr) {
    V v[U];
    int qq[U], rr[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int e = e0 + u * nthr;
      qq[u] = it.q;
      rr[u] = it.r;
      if (e < tot) v[u] = get(e, it.q, it.r);
      it.next();
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int e = e0 + u * nthr;
      if (e < tot) put(e, qq[u], rr[u], v[u]);
    }
  }
}

// ---- twiddles staged in LDS ----------------------------------------------------------------------
// Every axis (at most kMaxAxis points) keeps its twiddle table exp(-2 pi i t/n) in the first bytes
// of the block's dynamic LDS, so the barrier-separated FFT stages never wait on global memory.
constexpr int kMaxAxis = 2048;

template <typename T2>
__host__ __device__ constexpr size_t tw_lds_bytes(int n) {
  return (size_t(n) * sizeof(T2) + 15) / 16 * 16;
}

template <typename T2>
__device__ __forceinline__ const T2* stage_twiddles(unsigned char* smem_raw, const T2* __restrict__ tw, int n,
                                                    int tid, int nthr) {
  T2* t = reinterpret_cast<T2*>(smem_raw);
  gather_strided<4>(tid, nthr, n, [&](int i) { return tw[i]; }, [&](int i, T2 v) { t[i] = v; });
  return t;   // visible after the kernel's next barrier
}

// ---- XCD-aware block order ---------------------------------------------------------------------
// The dispatcher hands block b to XCD b mod 8, and each XCD has its own L2.  Remapping the linear
// block id so that consecutive logical tiles land on the same XCD lets the two blocks that write
// the halves of one cache line merge them in one L2.
__device__ __forceinline__ int xcd_logical_block(int b, int nb) {
  const int per = nb >> 3;
  if (b >= (per << 3)) return b;
  return (b & 7) * per + (b >> 3);
}

// logical (tile, x) of a z-pass block; grid = (ntiles, n1)
__device__ __forceinline__ void zpass_block(int& tile, int& x) {
  const int nb = gridDim.x * gridDim.y;
  const int L = xcd_logical_block(blockIdx.x + gridDim.x * blockIdx.y, nb);
  tile = L % gridDim.x;
  x = L / gridDim.x;
}

// ---- per-point spline state in LDS --------------------------------------------------------------
// Natural cubic spline on interval b (h = q_{b+1} - q_b, c6 = h^2/6) with second derivatives mm:
//   p_a  = (1-t) d_ab + t d_a,b+1 + c6 [((1-t)^3-(1-t)) mm_ab + (t^3-t) mm_a,b+1]
//   p_a' = (d_a,b+1 - d_ab)/h + (h/6) [-(3(1-t)^2-1) mm_ab + (3t^2-1) mm_a,b+1]
// mmT holds mm transposed ([b][a]) so that the two fields of a pair are adjacent.
template <typename T>
struct SplineLds {
  T* mmT;      // [M][M]
  T* h;        // [M-1]
  T* c6;       // [M-1]
  double* q;   // [M]
};

// carve the shared tables out of LDS (after `off` bytes) and fill them from global memory
template <typename T>
__device__ __forceinline__ SplineLds<T> load_spline_lds(unsigned char* smem, size_t off, const double* qmesh,
                                                        const double* mm, int M, int tid, int nthr) {
  SplineLds<T> S;
  off = (off + 15) & ~size_t(15);   // 16-byte aligned: mmT rows are read two entries at a time
  S.q = reinterpret_cast<double*>(smem + off);
  S.mmT = reinterpret_cast<T*>(smem + off + kMaxQ * sizeof(double));
  S.h = S.mmT + kMaxQ * kMaxQ;
  S.c6 = S.h + kMaxQ;
  for (int i = tid; i < M; i += nthr) S.q[i] = qmesh[i];
  for (int i = tid; i < M * M; i += nthr) {
    const int a = i / M, b = i - a * M;
    S.mmT[b * kMaxQ + a] = T(mm[i]);
  }
  for (int i = tid; i < M - 1; i += nthr) {
    const double hh = qmesh[i + 1] - qmesh[i];
    S.h[i] = T(hh);
    S.c6[i] = T(hh * hh / 6.0);
  }
  return S;
}

// bytes of the spline tables in LDS
template <typename T>
constexpr size_t spline_lds_bytes() {
  return 16 + kMaxQ * sizeof(double) + (kMaxQ * kMaxQ + 2 * kMaxQ) * sizeof(T);   // + alignment
}

// raw inputs of one point: n and either sigma (s[0]) or the three gradient components
struct PointIn {
  double n, s[3];
};

template <bool NT = false>
__device__ __forceinline__ PointIn point_load(const double* __restrict__ nden, const double* __restrict__ sig,
                                              size_t idx, size_t N, bool from_grad) {
  PointIn r;
  r.n = ld<NT>(&nden[idx]);
  r.s[0] = ld<NT>(&sig[idx]);
  r.s[1] = from_grad ? ld<NT>(&sig[N + idx]) : 0.0;
  r.s[2] = from_grad ? ld<NT>(&sig[2 * N + idx]) : 0.0;
  return r;
}

__device__ __forceinline__ double point_sigma(const PointIn& r, bool from_grad) {
  return from_grad ? r.s[0] * r.s[0] + r.s[1] * r.s[1] + r.s[2] * r.s[2] : r.s[0];
}

// ---- pass 1: q0 + splines + forward z FFT (theta fields) ------------------------------------
// Block: one x plane, TY consecutive y lines.  LDS: the TY pair lines, then per point the spline
// interval b (uint8, 255 = vacuum), position t and density n, then the spline tables.  q0 is
// evaluated once per point in FP64; theta_a = n p_a(q0) is formed in the path's precision T.  The
// point's state (t, n dq0/dn, n dq0/dsigma, b) also goes to `state` for the inverse z pass.

template <typename T, int EPT, bool SIGMA_FROM_GRAD>
__global__ void __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(VDWXC_WPE_THETA)))
k_theta_zfwd(const double* __restrict__ nden, const double* __restrict__ sig,
             typename Cx<T>::type* __restrict__ A, Quad<T>* __restrict__ state, int* __restrict__ flag,
             const double* __restrict__ qmesh, const double* __restrict__ mm,
             const typename Cx<T>::type* __restrict__ tw, Geometry g, AxisPlan zp, int ty, int lstride) {
  using T2 = typename Cx<T>::type;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  unsigned char* smem = smem_raw + tw_lds_bytes<T2>(g.n3);
  const T2* twl = stage_twiddles(smem_raw, tw, g.n3, threadIdx.x, blockDim.x);
  const int tid = threadIdx.x, nthr = blockDim.x;
  int tile, x;
  zpass_block(tile, x);
  const int y0 = tile * ty;
  const int n3 = g.n3, M = g.M;
  const size_t N = size_t(g.n1) * g.n2 * n3;
  const int npts = ty * n3;
  T2* line = reinterpret_cast<T2*>(smem);
  size_t off = size_t(ty) * lstride * sizeof(T2);
  T* st_t = reinterpret_cast<T*>(smem + off);
  off += size_t(npts) * sizeof(T);
  T* st_n = reinterpret_cast<T*>(smem + off);
  off += size_t(npts) * sizeof(T);
  unsigned char* st_b = smem + off;
  off += (size_t(npts) + 15) & ~size_t(15);
  const SplineLds<T> S = load_spline_lds<T>(smem, off, qmesh, mm, M, tid, nthr);
  __syncthreads();

  bool bad = false;
  gather_strided_dm<VDWXC_THETA_U>(
      tid, nthr, npts, n3,
      [&](int, int yl, int z) {
        const int y = y0 + yl;
        PointIn r{0.0, {0.0, 0.0, 0.0}};
        if (y < g.n2) r = point_load(nden, sig, (size_t(x) * g.n2 + y) * n3 + z, N, SIGMA_FROM_GRAD);
        return r;
      },
      [&](int p, int yl, int z, const PointIn& r) {
        const int y = y0 + yl;
        int b = -1;
        double t = 0.0;
        if (y < g.n2) {
          const double sv = point_sigma(r, SIGMA_FROM_GRAD);
          bad |= !(r.n == r.n) || !(sv == sv);
          double an, as;
          q0_state(r.n, sv, g.zab, S.q, M, b, t, an, as);
          // the point's spline state for the inverse z pass: (t, n dq0/dn, n dq0/dsigma, b)
          state[(size_t(x) * g.n2 + y) * n3 + z] = Quad<T>{T(t), T(an), T(as), T(b < 0 ? 255 : b)};
        }
        st_b[p] = b < 0 ? 255 : (unsigned char)b;
        st_t[p] = T(t);
        st_n[p] = T(r.n);
      });
  if (bad) *flag = 1;
  __syncthreads();

  const int npairs = (M + 1) >> 1;
#pragma unroll 1
  for (int pr = 0; pr < npairs; ++pr) {
    const int fa = 2 * pr, fb = 2 * pr + 1;
    DivModStep it(tid, nthr, n3);
#pragma unroll 1
    for (int p = tid; p < npts; p += nthr, it.next()) {
      const int yl = it.q, z = it.r;
      const int b = st_b[p];
      T ta = T(0), tb = T(0);
      if (b != 255) {
        // theta_a = n p_a = n [u d_ab + t d_a,b+1 + c6 ((u^3-u) m_b,a + (t^3-t) m_b+1,a)]: the
        // weights once per point, the m entries of fields fa, fa+1 in one read per knot
        const T t = st_t[p], nv = st_n[p], u = T(1) - t;
        const T c = S.c6[b] * nv;
        const T wa = c * (u * u * u - u), wb = c * (t * t * t - t);
        const T2 m0 = *reinterpret_cast<const T2*>(S.mmT + b * kMaxQ + fa);
        const T2 m1 = *reinterpret_cast<const T2*>(S.mmT + (b + 1) * kMaxQ + fa);
        const T nu = nv * u, nt = nv * t;
        ta = wa * m0.x + wb * m1.x + (fa == b ? nu : T(0)) + (fa == b + 1 ? nt : T(0));
        tb = fb < M ? wa * m0.y + wb * m1.y + (fb == b ? nu : T(0)) + (fb == b + 1 ? nt : T(0)) : T(0);
      }
      line[yl * lstride + lidx<>(z)] = T2{ta, tb};
    }
    __syncthreads();
    lds_fft<EPT, -1>(line, zp, ty, lstride, twl, tid, nthr);
    const int nout = ty * g.h3;
    // A[f][x][kz][y0 + yl] = Aa[kz * kzstride + yl] (field fa), Aa[fstride + ...] (field fb)
    T2* Aa = A + a_index(g, fa, 0, x, y0);
    const size_t kzstride = g.n2, fstride = size_t(g.n1) * g.h3 * g.n2;
    DivModStep ot(tid, nthr, ty);
#pragma unroll 1
    for (int e = tid; e < nout; e += nthr, ot.next()) {
      const int yl = ot.r, kz = ot.q, y = y0 + yl;
      if (y < g.n2) {
        const T2 zk = line[yl * lstride + lidx<>(kz)];
        const T2 zn = line[yl * lstride + lidx<>(kz == 0 ? 0 : n3 - kz)];
        T2 xa, xb;
        split_pair(zk, zn, xa, xb);
        T2* dst = Aa + size_t(kz) * kzstride + yl;
        dst[0] = xa;
        if (fb < M) dst[fstride] = xb;
      }
    }
    __syncthreads();
  }
}

// The same pass for N3 = 512, where the transform's thread mapping fixes the points of a thread:
// thread t owns line (y) t / 64 of the tile and the points z = t mod 64 + 64 r, r = 0..7, which
// are exactly the inputs of its first transform stage.  So the points' q0 state stays in the
// thread's registers from q0 to every field pair, and theta_a goes straight into the first stage:
// no per-point state in LDS (the block holds the ty lines, the twiddles and the spline tables,
// half the LDS of the general kernel) and no theta round trip through LDS.  nthr = 64 ty.  WPE:
// the waves per SIMD the registers must allow (the eight points' state in FP64 needs more than
// the 128 registers of four).  PB field pairs go through one transform (PB ty lines in LDS): fewer
// rounds of transform, store and barrier per block.
template <typename T, bool SIGMA_FROM_GRAD, int WPE, int PB>
__global__ void __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(WPE)))
k_theta_zfwd512(const double* __restrict__ nden, const double* __restrict__ sig,
                typename Cx<T>::type* __restrict__ A, Quad<T>* __restrict__ state, unsigned char* __restrict__ sb, int* __restrict__ flag,
                const double* __restrict__ qmesh, const double* __restrict__ mm,
                const typename Cx<T>::type* __restrict__ tw, Geometry g, int ty, int lstride) {
  using T2 = typename Cx<T>::type;
  constexpr int n3 = 512;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  unsigned char* smem = smem_raw + tw_lds_bytes<T2>(n3);
  const T2* twl = stage_twiddles(smem_raw, tw, n3, threadIdx.x, blockDim.x);
  const int tid = threadIdx.x, nthr = blockDim.x;
  int tile, x;
  zpass_block(tile, x);
  const int y0 = tile * ty, M = g.M;
  const size_t N = size_t(g.n1) * g.n2 * n3;
  T2* line = reinterpret_cast<T2*>(smem);
  const SplineLds<T> S = load_spline_lds<T>(smem, size_t(PB) * ty * lstride * sizeof(T2), qmesh, mm, M, tid, nthr);
  // the thread's points
  const int yl = __builtin_amdgcn_readfirstlane(tid >> 6), i = tid & 63, y = y0 + yl;
  const bool live = y < g.n2;
  const size_t pbase = (size_t(x) * g.n2 + y) * n3 + i;
  PointIn in[8];
#pragma unroll
  for (int r = 0; r < 8; ++r) {
    in[r] = PointIn{0.0, {0.0, 0.0, 0.0}};
    if (live) in[r] = point_load<nt_site<T, kNtThetaIn>()>(nden, sig, pbase + 64 * r, N, SIGMA_FROM_GRAD);
  }
  __syncthreads();   // spline tables and twiddles in LDS (the point loads are in flight meanwhile)
  int pb[8];      // spline interval, 255: vacuum (theta = 0)
  T pt[8], pn[8]; // position in the interval, density
  bool bad = false;
#pragma unroll
  for (int r = 0; r < 8; ++r) {
    int b = -1;
    double t = 0.0;
    if (live) {
      const double sv = point_sigma(in[r], SIGMA_FROM_GRAD);
      bad |= !(in[r].n == in[r].n) || !(sv == sv);
      double an, as;
      q0_state(in[r].n, sv, g.zab, S.q, M, b, t, an, as);
      // the point's spline state for the inverse z pass: (t, n dq0/dn, n dq0/dsigma, b)
      st<nt_site<T, kNtThetaOut>()>(&state[pbase + 64 * r], Quad<T>{T(t), T(an), T(as), T(b < 0 ? 255 : b)});
      st<nt_site<T, kNtThetaSb>()>(&sb[pbase + 64 * r], (unsigned char)(b < 0 ? 255 : b));   // the interval alone, for the assembly
    }
    pb[r] = b < 0 ? 255 : b;
    pt[r] = T(t);
    pn[r] = T(in[r].n);
  }
  if (bad) *flag = 1;

  const int npairs = (M + 1) >> 1;
  const size_t kzstride = g.n2, fstride = size_t(g.n1) * g.h3 * g.n2;
#pragma unroll 1
  for (int pr0 = 0; pr0 < npairs; pr0 += PB) {
    const int nb = min(PB, npairs - pr0);
    // theta_a = n p_a = n [u d_ab + t d_a,b+1 + c6 ((u^3-u) m_b,a + (t^3-t) m_b+1,a)] of fields fa,
    // fa+1 as the real and imaginary part of the first stage's input (line l = yl + q ty holds
    // pair pr0 + q)
    lds_fft512<PB, -1, kLdsPadShift>(
        line, nb * ty, lstride, twl, tid, nthr,
        [&](int l, int r, int) {
          const int fa = 2 * (pr0 + (l - yl) / ty), fb = fa + 1;
          const int b = pb[r];
          T ta = T(0), tb = T(0);
          if (b != 255) {
            const T t = pt[r], nv = pn[r], u = T(1) - t;
            const T c = S.c6[b] * nv;
            const T wa = c * (u * u * u - u), wb = c * (t * t * t - t);
            const T2 m0 = *reinterpret_cast<const T2*>(S.mmT + b * kMaxQ + fa);
            const T2 m1 = *reinterpret_cast<const T2*>(S.mmT + (b + 1) * kMaxQ + fa);
            const T nu = nv * u, nt = nv * t;
            ta = wa * m0.x + wb * m1.x + (fa == b ? nu : T(0)) + (fa == b + 1 ? nt : T(0));
            tb = fb < M ? wa * m0.y + wb * m1.y + (fb == b ? nu : T(0)) + (fb == b + 1 ? nt : T(0)) : T(0);
          }
          return T2{ta, tb};
        },
        LdsLines{});
    // A[f][x][kz][y0 + yl] = Aa[kz * kzstride + yl] (field fa), Aa[fstride + ...] (field fb)
    for (int q = 0; q < nb; ++q) {
      const int fa = 2 * (pr0 + q), fb = fa + 1;
      T2* Aa = A + a_index(g, fa, 0, x, y0);
      const T2* lq = line + size_t(q) * ty * lstride;
      const int nout = ty * g.h3;
      DivModStep ot(tid, nthr, ty);
#pragma unroll 1
      for (int e = tid; e < nout; e += nthr, ot.next()) {
        const int ol = ot.r, kz = ot.q;
        if (y0 + ol < g.n2) {
          const T2 zk = lq[ol * lstride + lidx<>(kz)];
          const T2 zn = lq[ol * lstride + lidx<>(kz == 0 ? 0 : n3 - kz)];
          T2 xa, xb;
          split_pair(zk, zn, xa, xb);
          T2* dst = Aa + size_t(kz) * kzstride + ol;
          st<nt_site<T, kNtThetaOut>()>(dst, xa);
          if (fb < M) st<nt_site<T, kNtThetaOut>()>(dst + fstride, xb);
        }
      }
    }
    __syncthreads();
  }
}

// ---- pass 2 / 4: y FFT with rotation A[f][x][kz][y] <-> B[f][kz][ky][x] ----------------------
// Block: TX consecutive x of one (f, kz) (blockIdx.x = x tile, .y = kz, .z = f).

template <typename T, int EPT, int DIR>
__global__ void __launch_bounds__(1024) __attribute__((amdgpu_waves_per_eu(VDWXC_WPE_Y)))
k_ypass(const typename Cx<T>::type* __restrict__ src, typename Cx<T>::type* __restrict__ dst,
        const typename Cx<T>::type* __restrict__ tw, Geometry g, AxisPlan yp, int tx, int lstride) {
  using T2 = typename Cx<T>::type;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  unsigned char* smem = smem_raw + tw_lds_bytes<T2>(g.n2);
  T2* line = reinterpret_cast<T2*>(smem);
  const int tid = threadIdx.x, nthr = blockDim.x;
  const int nb = gridDim.x * gridDim.y * gridDim.z;
  const int L = xcd_logical_block(blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z), nb);
  const int x0 = (L % gridDim.x) * tx, kz = (L / gridDim.x) % gridDim.y, f = L / (gridDim.x * gridDim.y);
  const int n2 = g.n2, tot = tx * n2;
  // 512-point lines: the first forward stage reads the A lines (y contiguous) straight from global
  // memory, the last inverse stage writes them there
  const bool f512 = n2 == 512 && (nthr & 63) == 0;
  const T2* twl = stage_twiddles(smem_raw, tw, g.n2, tid, nthr);
  const size_t xs = size_t(g.h3) * g.n2;   // x stride of A
  if (DIR < 0 && f512) {
    // the staged twiddles are read from the second stage on, and the transform synchronises its
    // stages within each wave only
    __syncthreads();
    const T2* sbase = src + a_index(g, f, kz, x0, 0);
    lds_fft512<(EPT + 7) / 8, DIR, kLdsPadShift>(
        line, tx, lstride, twl, tid, nthr,
        [&](int xl, int, int y) { return (x0 + xl < g.n1) ? ld<nt_site<T, kNtYfLoad>()>(&sbase[size_t(xl) * xs + y]) : T2{T(0), T(0)}; },
        LdsLines{});
  } else if (DIR < 0) {
    const T2* sbase = src + a_index(g, f, kz, x0, 0);
    gather_strided_dm<8>(
        tid, nthr, tot, n2, [&](int, int xl, int y) { return (x0 + xl < g.n1) ? sbase[size_t(xl) * xs + y] : T2{T(0), T(0)}; },
        [&](int, int xl, int y, T2 v) { line[xl * lstride + lidx<>(y)] = v; });
  } else {
    // B[f][kz][ky][x0 + xl] = sbase[size_t(ky) * ystride + xl]
    const T2* sbase = src + b_index(g, f, 0, kz, x0);
    const int ystride = g.n1;
    gather_strided_dm<8>(
        tid, nthr, tot, tx,
        [&](int, int ky, int xl) { return (x0 + xl < g.n1) ? ld<nt_site<T, kNtYiLoad>()>(&sbase[size_t(ky) * ystride + xl]) : T2{T(0), T(0)}; },
        [&](int, int ky, int xl, T2 v) { line[xl * lstride + lidx<>(ky)] = v; });
  }
  if (DIR > 0 && f512) {
    __syncthreads();
    T2* dbase = dst + a_index(g, f, kz, x0, 0);
    lds_fft512<(EPT + 7) / 8, DIR, kLdsPadShift, false>(line, tx, lstride, twl, tid, nthr, LdsLines{},
                                                       [&](int xl, int, int y, T2 v) {
                                                         if (x0 + xl < g.n1) st<nt_site<T, kNtYiStore>()>(&dbase[size_t(xl) * xs + y], v);
                                                       });
    return;
  }
  if (!(DIR < 0 && f512)) {
    __syncthreads();
    lds_fft<EPT, DIR>(line, yp, tx, lstride, twl, tid, nthr);
  }
  if (DIR < 0) {
    T2* dbase = dst + b_index(g, f, 0, kz, x0);
    const int ystride = g.n1;
    DivModStep it(tid, nthr, tx);
    for (int e = tid; e < tot; e += nthr, it.next()) {
      const int xl = it.r, ky = it.q;
      if (x0 + xl < g.n1) st<nt_site<T, kNtYfStore>()>(&dbase[size_t(ky) * ystride + xl], line[xl * lstride + lidx<>(ky)]);
    }
  } else {
    T2* dbase = dst + a_index(g, f, kz, x0, 0);
    DivModStep it(tid, nthr, n2);
    for (int e = tid; e < tot; e += nthr, it.next()) {
      const int xl = it.q, y = it.r;
      if (x0 + xl < g.n1) dbase[size_t(xl) * xs + y] = line[xl * lstride + lidx<>(y)];
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
// Block: the M field lines of one (ky, kz) column (blockIdx.x = ky, .y = kz).  With ky fastest,
// the blocks resident at one time read and write one contiguous window of each field (the lines
// of consecutive ky are adjacent in B) instead of lines a whole plane apart.
// Per k: phi_ab = (1-w) T_j,ab + w T_j+1,ab with |G| = (j + w) dk (Sec. 3 step 3a);
// F_a = sum_b phi_ab theta_b (step 3b); energy sum_a Re theta_a* F_a (step 3c), weight 2 for kz
// strictly inside the half spectrum, 1 on its edges.  phi is symmetric, so each unordered pair
// (a <= b) is interpolated once and feeds F_a and F_b.  The table holds, per two consecutive
// pairs g and node j (j contiguous), T_j and T_j+1 - T_j of both pairs: one 16-byte read (FP32)
// per two pairs and one FMA per interpolation.  Every lane reads its own nodes; kx and -kx, which
// have the same |G| in orthogonal cells, sit in adjacent lanes and share them.

// q-mesh buckets of the contraction kernel (its MB parameter): the smallest of 8, 10, 12, 16, 20
// that holds M
__host__ __device__ constexpr int q_bucket(int M) { return M <= 8 ? 8 : M <= 10 ? 10 : M <= 12 ? 12 : M <= 16 ? 16 : 20; }

// Order of the unordered pairs (a <= b) in the table and the contraction.  The pairs of a bucket
// MB come first: segment s holds the pairs whose larger index lies in [bucket s-1, bucket s), so
// a mesh of M <= MB points reads and contracts only the first MB(MB+1)/2.  Within a segment the
// pairs are scheduled greedily so that each one updates the accumulators F_a, F_b that have
// waited longest since their last update: consecutive FMAs into one accumulator would form a
// dependency chain (in plain row order every pair of a column updates F_b).
constexpr int kNumPairs = kMaxQ * (kMaxQ + 1) / 2;
static_assert(kNumPairs % 2 == 0, "pairs are stored two per table entry");
struct PairList {
  int row[kNumPairs], col[kNumPairs];
  int pos[kMaxQ][kMaxQ];   // place of pair (a, b), either order
  constexpr PairList() : row(), col(), pos() {
    bool used[kMaxQ][kMaxQ] = {};
    int last[kMaxQ] = {};
    for (int a = 0; a < kMaxQ; ++a) last[a] = -kNumPairs;
    const int ends[5] = {8, 10, 12, 16, 20};
    int p = 0, lo = 0;
    for (int s = 0; s < 5; ++s) {
      const int hi = ends[s];
      const int count = hi * (hi + 1) / 2 - lo * (lo + 1) / 2;
      for (int k = 0; k < count; ++k) {
        int ba = -1, bb = -1, best = -1;
        for (int b = lo; b < hi; ++b)
          for (int a = 0; a <= b; ++a) {
            if (used[a][b]) continue;
            const int da = p - last[a], db = p - last[b];
            const int score = da < db ? da : db;
            if (score > best) {
              best = score;
              ba = a;
              bb = b;
            }
          }
        used[ba][bb] = true;
        row[p] = ba;
        col[p] = bb;
        pos[ba][bb] = pos[bb][ba] = p;
        last[ba] = last[bb] = p;
        ++p;
      }
      lo = hi;
    }
  }
};
constexpr PairList kPairs{};
static_assert(kPairs.pos[0][0] < 36 && kPairs.pos[7][7] < 36 && kPairs.pos[0][8] >= 36, "bucket prefix order");

// table entries per load chunk of the contraction: FP64 3 (96 bytes of one node), FP32 2 (the
// register-capped FP32 kernel spills less with the smaller double buffer)
#ifndef VDWXC_XCHUNK64
#define VDWXC_XCHUNK64 3
#endif
#ifndef VDWXC_XCHUNK32
#define VDWXC_XCHUNK32 2
#endif
template <typename T>
__host__ __device__ constexpr int x_chunk() { return sizeof(T) == 8 ? VDWXC_XCHUNK64 : VDWXC_XCHUNK32; }
#ifndef VDWXC_XRING_HALF
#define VDWXC_XRING_HALF 3   // chunks of the paired contraction's load ring
#endif


// raw buffer resource, dword 3 on gfx9: no format conversion, plain byte addressing
constexpr int kBufferWord3 = 0x00020000;

__device__ __forceinline__ void buffer_load_quad(__amdgpu_buffer_rsrc_t r, int voff, int soff, Quad<float>& q) {
  const auto raw = __builtin_amdgcn_raw_buffer_load_b128(r, voff, soff, 0);
  __builtin_memcpy(&q, &raw, sizeof(q));
}
__device__ __forceinline__ void buffer_load_quad(__amdgpu_buffer_rsrc_t r, int voff, int soff, Quad<double>& q) {
  const auto lo = __builtin_amdgcn_raw_buffer_load_b128(r, voff, soff, 0);
  const auto hi = __builtin_amdgcn_raw_buffer_load_b128(r, voff + 16, soff, 0);
  __builtin_memcpy(&q.x, &lo, 16);
  __builtin_memcpy(&q.z, &hi, 16);
}

// one half (T_j, D_j of one pair) of a table entry
__device__ __forceinline__ void buffer_load_half(__amdgpu_buffer_rsrc_t r, int voff, int soff, float2& h) {
  const auto raw = __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0);
  __builtin_memcpy(&h, &raw, sizeof(h));
}
__device__ __forceinline__ void buffer_load_half(__amdgpu_buffer_rsrc_t r, int voff, int soff, double2& h) {
  const auto raw = __builtin_amdgcn_raw_buffer_load_b128(r, voff, soff, 0);
  __builtin_memcpy(&h, &raw, sizeof(h));
}

// x of lane (lane & ~3) + P[lane & 3] (DPP quad permutation CTRL), all four lanes active
template <int CTRL>
__device__ __forceinline__ float quad_perm(float x) {
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(x), CTRL, 0xF, 0xF, false));
}
template <int CTRL>
__device__ __forceinline__ double quad_perm(double x) {
  const long long b = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_mov_dpp(int(b), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_mov_dpp(int(b >> 32), CTRL, 0xF, 0xF, false);
  return __longlong_as_double((long long)(unsigned)lo | ((long long)hi << 32));
}
constexpr int kDppEvenOfPair = 0xA0;   // quad_perm [0, 0, 2, 2]
constexpr int kDppOddOfPair = 0xF5;    // quad_perm [1, 1, 3, 3]

// body(std::integral_constant<int, i>) for i = 0 .. N-1, unrolled at compile time
template <int N, typename Body>
__device__ __forceinline__ void static_for(Body&& body) {
  if constexpr (N > 0) {
    static_for<N - 1>(body);
    body(std::integral_constant<int, N - 1>{});
  }
}

// PS: LDS layout of the lines (kNoPad or kSwizzle: no padding).  Without padding and with the
// twiddles read from global memory, the 20 FP32 lines of a 512-point axis take exactly 80 KB, so
// two blocks can share a CU; WPE = 4 caps the registers at 128 so that two 512-thread blocks also
// fit the register file (the launch picks it for such blocks).
// MB: the q-mesh bucket, M <= MB (one of q_bucket's values).  The per-thread field arrays, the
// pair list and the table chunks the kernel reads are those of an MB-point mesh: the pairs (a, b)
// with b < MB are the first MB(MB+1)/2 (pair_index order), so a shorter mesh contracts and loads
// in proportion to MB(MB+1)/2.
template <typename T, int EPT, int PS, int WPE, int MB>
__global__ void __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(WPE)))
k_xcontract(typename Cx<T>::type* __restrict__ B, const Quad<T>* __restrict__ table4,
            double* __restrict__ partials, const typename Cx<T>::type* __restrict__ tw,
            Geometry g, AxisPlan xp) {
  using T2 = typename Cx<T>::type;
  extern __shared__ __align__(16) unsigned char smem[];
  const T2* twl = tw;                       // twiddles from global memory (L1/L2 resident)
  T2* line = reinterpret_cast<T2*>(smem);   // all M field lines of the column
  const int tid = threadIdx.x, nthr = blockDim.x;
  const int ky = blockIdx.x, kz = blockIdx.y, M = g.M, n1 = g.n1;
  const int ls = lds_span<PS>(n1);
  // field f of this column: cb[f * fstride + x]
  T2* cb = B + b_index(g, 0, ky, kz, 0);
  const size_t fstride = size_t(g.n2) * g.h3 * n1;
  const int G = (nthr * EPT) / n1;   // lines per batched transform
  // 512-point columns: the first forward stage reads the field lines straight from global memory
  // (13.4 -> 11.9 ms FP32, 21.3 -> 20.3 ms FP64 at 512^3)
  const bool f512 = n1 == 512 && (nthr & 63) == 0 && M <= G;
  if (f512) {
    lds_fft512<(EPT + 7) / 8, -1, PS>(line, M, ls, twl, tid, nthr,
                                      [&](int f, int, int x) { return ld<kNtX>(&cb[size_t(f) * fstride + x]); },
                                      LdsLines{});
  } else {
    gather_strided_dm<16>(
        tid, nthr, M * n1, n1, [&](int, int f, int x) { return cb[size_t(f) * fstride + x]; },
        [&](int, int f, int x, T2 v) { line[f * ls + lidx<PS>(x)] = v; });
    __syncthreads();
    for (int l0 = 0; l0 < M; l0 += G) lds_fft<EPT, -1, PS>(line + l0 * ls, xp, min(G, M - l0), ls, twl, tid, nthr);
  }

  // one k-point per slot, slots strided over the block's threads
  constexpr int NPT = 1;
  const int nslots = n1;
  double e = 0.0;
#pragma unroll 1
  for (int slot = tid; slot < nslots; slot += nthr) {
    int kx[NPT];
    bool valid[NPT];
    {
      // kx and -kx in adjacent lanes (same |G| in orthogonal cells, so the same table nodes):
      // even n1: slots 0, 1 -> 0, n1/2; slot 2m, 2m+1 -> m, n1-m.  odd n1: 0 -> 0; 2m-1, 2m -> m, n1-m.
      int x;
      if ((n1 & 1) == 0) {
        const int m = slot >> 1;
        x = slot == 0 ? 0 : slot == 1 ? n1 / 2 : ((slot & 1) ? n1 - m : m);
      } else {
        const int m = (slot + 1) >> 1;
        x = slot == 0 ? 0 : ((slot & 1) ? m : n1 - m);
      }
      kx[0] = x;
      valid[0] = true;
    }
    T2 th[NPT][MB], F[NPT][MB];
#pragma unroll
    for (int q = 0; q < NPT; ++q)
#pragma unroll
      for (int a = 0; a < MB; ++a) {
        th[q][a] = (a < M && valid[q]) ? line[a * ls + lidx<PS>(kx[q])] : T2{T(0), T(0)};
        F[q][a] = T2{T(0), T(0)};
      }
    const double kn = sqrt(gnorm2(g, kx[0], ky, kz));
    // phi = 0 for |G| >= k_max: there the thetas are taken as zero, so F = 0 and no energy
    const bool inside = kn < g.kmax;
    if (!inside) {
#pragma unroll
      for (int a = 0; a < MB; ++a) th[0][a] = T2{T(0), T(0)};
    }
    const double sc = kn * g.inv_dk;
    int j = inside ? int(floor(sc)) : 0;
    if (j > g.nk - 2) j = g.nk - 2;
    const T w = T(inside ? sc - j : 0.0);
    // Table entry (group g, node j) = T_j and T_j+1 - T_j of pair 2g, then of pair 2g+1, so
    // phi = T_j + w (T_j+1 - T_j) is one FMA.  The entries are stored chunk-major,
    // [g / kXChunk][j][g % kXChunk]: the kXChunk entries a lane reads for one chunk are adjacent,
    // so a chunk's loads share cache lines.  Buffer loads: the lane's node offset in one VGPR
    // (plus the entry's place in the chunk as an immediate), the chunk's offset in an SGPR,
    // advanced through one running offset that is laundered after every chunk (otherwise all
    // chunk offsets are formed up front and stay live).  Each pair is read and interpolated once
    // (phi is symmetric) and feeds F_a += phi theta_b and F_b += phi theta_a.  The next chunk's
    // loads are issued before the current chunk's arithmetic.
    // Paired reads (FP64 with g.xpair): the lanes of a kx, -kx pair have the same node j and
    // weight w, so the even lane reads and interpolates pair 2g, the odd lane pair 2g+1, and the
    // two phis are swapped between them by DPP: half the table bytes per k-point (the
    // contraction's loads are bound by the vector memory pipeline).  The wave holding kx = 0 and
    // N1/2 (slots 0 and 1, whose |G| differ) reads whole entries.  (FP32 keeps whole-entry reads:
    // its register-capped kernel spills with the paired path.)
    constexpr int kXChunk = x_chunk<T>();
    constexpr int kPairsMB = MB * (MB + 1) / 2;
    constexpr int kGroups = (kPairsMB + 1) / 2;
    constexpr int kChunks = (kGroups + kXChunk - 1) / kXChunk;
    constexpr int kQ = int(sizeof(Quad<T>));
    const int joff = j * (kXChunk * kQ);
    const int cstride = g.nk * (kXChunk * kQ);
    const __amdgpu_buffer_rsrc_t trs =
        __builtin_amdgcn_make_buffer_rsrc(const_cast<Quad<T>*>(table4), short(0), cstride * kChunks, kBufferWord3);
    constexpr bool kPairable = sizeof(T) == 8;
    auto contract = [&](auto half_tag) {
      constexpr bool HALF = decltype(half_tag)::value;
      using Buf = std::conditional_t<HALF, T2, Quad<T>>;
      const int voff = HALF ? joff + (tid & 1) * (kQ / 2) : joff;
      int tcur = 0;
      auto load_chunk = [&](Buf* dst, int cc) {
        asm volatile("" : "+s"(tcur));
#pragma unroll
        for (int i = 0; i < kXChunk; ++i)
          if (cc * kXChunk + i < kGroups) {
            if constexpr (HALF) buffer_load_half(trs, voff + i * kQ, tcur, dst[i]);
            else buffer_load_quad(trs, voff + i * kQ, tcur, dst[i]);
          }
        tcur += cstride;
      };
      // a ring of R chunks: chunk c + R - 1 is loaded while chunk c is contracted (the paired
      // path's entries are half as large, so it keeps twice the loads in flight in the same
      // registers)
      constexpr int R = HALF ? VDWXC_XRING_HALF : 2;
      Buf buf[R][kXChunk];
#pragma unroll
      for (int c = 0; c < R - 1; ++c)
        if (c < kChunks) load_chunk(buf[c], c);
#pragma unroll
      for (int c = 0; c < kChunks; ++c) {
        if (c + R - 1 < kChunks) load_chunk(buf[(c + R - 1) % R], c + R - 1);
#pragma unroll
        for (int i = 0; i < kXChunk; ++i) {
          const int grp = c * kXChunk + i;
          if (grp < kGroups) {
            const int a0 = kPairs.row[2 * grp], b0 = kPairs.col[2 * grp];
            const int a1 = kPairs.row[2 * grp + 1], b1 = kPairs.col[2 * grp + 1];
            T phi0, phi1;
            if constexpr (HALF) {
              const T2& hv = buf[c % R][i];
              const T own = hv.x + w * hv.y;
              phi0 = quad_perm<kDppEvenOfPair>(own);
              phi1 = quad_perm<kDppOddOfPair>(own);
            } else {
              const Quad<T>& v = buf[c % R][i];
              phi0 = v.x + w * v.y;
              phi1 = v.z + w * v.w;
            }
#pragma unroll
            for (int q = 0; q < NPT; ++q) {
              F[q][a0].x += phi0 * th[q][b0].x;
              F[q][a0].y += phi0 * th[q][b0].y;
              if (a0 != b0) {
                F[q][b0].x += phi0 * th[q][a0].x;
                F[q][b0].y += phi0 * th[q][a0].y;
              }
              if (2 * grp + 1 < kPairsMB) {   // an odd pair count leaves the last entry half used
                F[q][a1].x += phi1 * th[q][b1].x;
                F[q][a1].y += phi1 * th[q][b1].y;
                if (a1 != b1) {
                  F[q][b1].x += phi1 * th[q][a1].x;
                  F[q][b1].y += phi1 * th[q][a1].y;
                }
              }
            }
          }
        }
        // pin the accumulators here, so this chunk's arithmetic is not moved below the next
        // chunk's loads (which would keep every loaded entry live at once)
#pragma unroll
        for (int q = 0; q < NPT; ++q)
#pragma unroll
          for (int a = 0; a < MB; ++a) asm volatile("" : "+v"(F[q][a].x), "+v"(F[q][a].y));
      }
    };
    if (kPairable && g.xpair != 0 && __builtin_amdgcn_readfirstlane(slot) != 0) contract(std::true_type{});
    else contract(std::false_type{});
#pragma unroll
    for (int q = 0; q < NPT; ++q) {
      if (valid[q]) {
#pragma unroll
        for (int a = 0; a < MB; ++a) {
          if (a < M) {
            e += double(th[q][a].x) * double(F[q][a].x) + double(th[q][a].y) * double(F[q][a].y);
            line[a * ls + lidx<PS>(kx[q])] = F[q][a];
          }
        }
      }
    }
  }
  __syncthreads();
  if (f512) {
    // 512-point columns: the last inverse stage stores straight to global memory (no LDS round
    // trip and barrier; it also frees registers: 18.4 -> 17.4 ms FP64, 11.1 -> 9.7 ms FP32 at 512^3)
    lds_fft512<(EPT + 7) / 8, +1, PS, false>(line, M, ls, twl, tid, nthr, LdsLines{},
                                             [&](int f, int, int x, T2 v) { st<kNtX>(&cb[size_t(f) * fstride + x], v); });
  } else {
    for (int l0 = 0; l0 < M; l0 += G) lds_fft<EPT, +1, PS>(line + l0 * ls, xp, min(G, M - l0), ls, twl, tid, nthr);
    DivModStep it(tid, nthr, n1);
    for (int e2 = tid; e2 < M * n1; e2 += nthr, it.next()) cb[size_t(it.q) * fstride + it.r] = line[it.q * ls + lidx<PS>(it.r)];
  }

  // block sum of the energy, fixed order: wave shuffles, then the waves in order
  const double wz = (kz == 0 || is_nyquist(kz, g.n3)) ? 1.0 : 2.0;
  double esum = wz * e;
  for (int off = 32; off > 0; off >>= 1) esum += __shfl_xor(esum, off, 64);
  __syncthreads();
  double* red = reinterpret_cast<double*>(smem);
  if ((tid & 63) == 0) red[tid >> 6] = esum;
  __syncthreads();
  if (tid == 0) {
    double sum = 0.0;
    for (int wv = 0; wv < (nthr + 63) / 64; ++wv) sum += red[wv];
    partials[size_t(kz) * g.n2 + ky] = sum;
  }
}

// Rebuild the full complex z-line Z = X_a + i X_b of a field pair from their half spectra (the
// imaginary parts of the k = 0 and Nyquist terms are dropped, as a complex-to-real transform does).
template <typename T2>
__device__ __forceinline__ void store_pair_values(T2 xa, T2 xb, int kz, int yl, int n3, T2* line, int lstride) {
  using T = decltype(line[0].x);
  const bool edge = (kz == 0) || is_nyquist(kz, n3);
  if (edge) {
    xa.y = T(0);
    xb.y = T(0);
  }
  line[yl * lstride + lidx<>(kz)] = T2{xa.x - xb.y, xa.y + xb.x};
  if (!edge) line[yl * lstride + lidx<>(n3 - kz)] = T2{xa.x + xb.y, xb.x - xa.y};
}

// The half spectra of one field pair for a z-pass tile, held in registers so that the next pair's
// loads are in flight while the current pair is transformed.  PF >= ceil(ty*h3 / nthr).
template <typename T2, int PF>
struct PairPrefetch {
  T2 a[PF], b[PF];
  __device__ __forceinline__ void issue(const T2* __restrict__ A, const Geometry& g, int fa, int fb, int x, int y0,
                                        int ty, int tid, int nthr) {
    using T = decltype(a[0].x);
    const int tot = ty * g.h3;
    DivModStep it(tid, nthr, ty);
#pragma unroll
    for (int c = 0; c < PF; ++c, it.next()) {
      const int e = tid + c * nthr;
      a[c] = b[c] = T2{T(0), T(0)};
      if (e < tot) {
        const int yl = it.r, kz = it.q, y = y0 + yl;
        if (y < g.n2) {
          a[c] = ld<nt_site<T, kNtAsmA>()>(&A[a_index(g, fa, kz, x, y)]);
          if (fb >= 0) b[c] = ld<nt_site<T, kNtAsmA>()>(&A[a_index(g, fb, kz, x, y)]);
        }
      }
    }
  }
  __device__ __forceinline__ void store(const Geometry& g, int ty, T2* line, int lstride, int tid, int nthr) const {
    const int tot = ty * g.h3;
    DivModStep it(tid, nthr, ty);
#pragma unroll
    for (int c = 0; c < PF; ++c, it.next()) {
      const int e = tid + c * nthr;
      if (e < tot) store_pair_values(a[c], b[c], it.q, it.r, g.n3, line, lstride);
    }
  }
};

// Clear an evaluation's NaN flags (a fill kernel rather than a memset, so that it can sit in a
// captured graph).  One block.
__global__ void k_clear_flags(int* __restrict__ flag) {
  if (threadIdx.x < 2) flag[threadIdx.x] = 0;
}

// ---- energy: fixed-order sum of the per-column partials (one block) ----------------------------
// Eight independent loads in flight per thread, then a fixed reduction tree: the same inputs give
// the same bits.  flag[0] is raised by the theta pass on a NaN input; it is moved to flag[1] (the
// evaluation's result, read by the host) and cleared here, so the next evaluation starts from
// zero.  `red` holds one double per wave; the block is synchronised on return.
__device__ __forceinline__ void energy_reduce_block(const double* __restrict__ partials, int nparts, double scale,
                                                    int* __restrict__ flag, double* __restrict__ out, double* red,
                                                    int tid, int nthr) {
  double acc[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  for (int i0 = tid; i0 < nparts; i0 += 8 * nthr) {
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int i = i0 + u * nthr;
      if (i < nparts) acc[u] += partials[i];
    }
  }
  double s = ((acc[0] + acc[1]) + (acc[2] + acc[3])) + ((acc[4] + acc[5]) + (acc[6] + acc[7]));
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
  if ((tid & 63) == 0) red[tid >> 6] = s;
  __syncthreads();
  if (tid == 0) {
    double tot = 0.0;
    for (int w = 0; w < (nthr + 63) / 64; ++w) tot += red[w];
    const int bad = flag[0];
    out[0] = bad != 0 ? __builtin_nan("") : tot * scale;
    flag[1] = bad;
    flag[0] = 0;
  }
  __syncthreads();
}

// ---- semilocal completion: the LDA correlation (appendix, PW92) -----------------------------
// E_c^LDA = (Omega/N) sum_p n_p eps_c(r_s(n_p)) and v_c^LDA = d(n eps_c)/dn = eps_c - (r_s/3)
// d eps_c/d r_s per point, in FP64: a streaming pass of 8 bytes read and 8 written per point.
// Each thread takes kLdaUnroll points a step (their loads issued together), sums n eps_c in a fixed
// order and the block adds its threads' sums in a fixed tree into partials[block]; k_lda_energy
// adds the blocks' sums in one block.  Equal inputs give equal bits.  A NaN density yields NaN at
// its point and in the energy; points below the vacuum threshold give zero.
constexpr int kLdaThreads = 256, kLdaUnroll = 4, kLdaBlocks = 2048;

__device__ __forceinline__ double block_sum_fixed(double s, double* red, int tid) {
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
  if ((tid & 63) == 0) red[tid >> 6] = s;
  __syncthreads();
  double tot = 0.0;
  if (tid == 0)
    for (int w = 0; w < kLdaThreads / 64; ++w) tot += red[w];
  return tot;   // valid in thread 0
}

__global__ void __launch_bounds__(kLdaThreads) k_lda_pw92(const double* __restrict__ n, double* __restrict__ v,
                                                         double* __restrict__ partials, long long npts) {
  __shared__ double red[kLdaThreads / 64];
  const int tid = threadIdx.x;
  const long long step = (long long)gridDim.x * kLdaThreads * kLdaUnroll;
  double acc = 0.0;
  for (long long p0 = (long long)blockIdx.x * kLdaThreads * kLdaUnroll + tid; p0 < npts; p0 += step) {
    double x[kLdaUnroll];
#pragma unroll
    for (int u = 0; u < kLdaUnroll; ++u) {
      const long long p = p0 + (long long)u * kLdaThreads;
      x[u] = p < npts ? n[p] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < kLdaUnroll; ++u) {
      const long long p = p0 + (long long)u * kLdaThreads;
      double vp = 0.0, e = 0.0;
      if (x[u] >= kVacuum) {
        const double rs = kRsKf / cbrt(3.0 * kPi * kPi * x[u]);
        double eps, deps;
        pw92(rs, eps, deps);
        vp = eps - (rs / 3.0) * deps;
        e = x[u] * eps;
      } else if (x[u] != x[u]) {
        vp = e = x[u];
      }
      if (p < npts) v[p] = vp;
      acc += e;
    }
  }
  const double tot = block_sum_fixed(acc, red, tid);
  if (tid == 0) partials[blockIdx.x] = tot;
}

__global__ void __launch_bounds__(kLdaThreads) k_lda_energy(const double* __restrict__ partials, int nparts,
                                                           double scale, double* __restrict__ energy) {
  __shared__ double red[kLdaThreads / 64];
  const int tid = threadIdx.x;
  double acc = 0.0;
  for (int i = tid; i < nparts; i += kLdaThreads) acc += partials[i];
  const double tot = block_sum_fixed(acc, red, tid);
  if (tid == 0) energy[0] = tot * scale;
}

// ---- spin polarisation (the variant Sec. 7 announces) -----------------------------------------
// The paper prints only the spin-paired q0.  Spin-polarised q0 here: the gradient-corrected LDA
// exchange of the appendix spin-scaled, E_x[n_up, n_dn] = (E_x[2 n_up] + E_x[2 n_dn]) / 2, plus the
// spin-resolved PW92 correlation eps_c(r_s, zeta):
//   q0 = sum_s [ (n_s/n) k_s - (Z_ab/36) sigma_ss / (n n_s k_s) ] - (4 pi/3) eps_c(r_s, zeta)
// with k_s = (6 pi^2 n_s)^(1/3), n = n_up + n_dn, zeta = (n_up - n_dn)/n; a spin density below the
// vacuum threshold (or negative) counts as zero.  theta_a = n p_a(q0) as spin-paired.
//
// The spin-paired pipeline runs unchanged on (n, sigma_eff): sigma_eff is the sigma for which the
// spin-paired q0 formula gives the spin-polarised q0 (the gradient term is linear in sigma, so it
// is one division).  q0 then carries the same saturation, clamp and spline state, and from the
// pipeline's dE/dn|sigma_eff = P + n h' dx_u/dn D and dE/dsigma_eff = n h' dx_u/dsigma D
// (P = sum F p, D = sum F p', h' the saturation slope, x_u the spin-paired unsaturated q0):
//   dE/dn_s       = dE/dn + (dE/dsigma_eff / dx_u/dsigma) (dx/dn_s - dx_u/dn)
//   dE/dsigma_ss  = (dE/dsigma_eff / dx_u/dsigma) dx/dsigma_ss
// exactly (dx_u/dsigma = -Z_ab/(36 k_F n^2) is never zero).

// Perdew-Wang 1992 fits of eps_c(r_s, 1) and of -alpha_c(r_s) (the spin stiffness), in the form of
// the appendix's eps_c(r_s, 0); f''(0) of the spin interpolation f(zeta)
constexpr double kFerro[6] = {0.015545, 0.20548, 14.1189, 6.1977, 3.3662, 0.62517};
constexpr double kStiff[6] = {0.016887, 0.11125, 10.357, 3.6231, 0.88026, 0.49671};
constexpr double kFzz0 = 1.709921;

// G(r_s) = -2A (1 + alpha1 r_s) ln[1 + 1/(2A (b1 r_s^1/2 + b2 r_s + b3 r_s^3/2 + b4 r_s^2))], dG/dr_s
__device__ __forceinline__ void pw92_fit(const double (&c)[6], double rs, double sq, double& G, double& dG) {
  const double A = c[0];
  const double Q = 2.0 * A * (c[2] * sq + c[3] * rs + c[4] * rs * sq + c[5] * rs * rs);
  const double dQ = 2.0 * A * (0.5 * c[2] / sq + c[3] + 1.5 * c[4] * sq + 2.0 * c[5] * rs);
  const double lg = log1p(1.0 / Q);
  G = -2.0 * A * (1.0 + c[1] * rs) * lg;
  dG = -2.0 * A * c[1] * lg + 2.0 * A * (1.0 + c[1] * rs) * dQ / (Q * (Q + 1.0));
}

// Unsaturated spin-polarised q0 x and its partials (n_up, n_dn, sigma_uu, sigma_dd) at a point with
// n = nu + nd >= the vacuum threshold (nu, nd already cut at it), and the spin-paired
// quantities the conversion needs: k_F, r_s and eps_c(r_s, 0), d eps_c / d r_s.
struct SpinQ0 {
  double x, dx[4];
  double kF, rs, e0, de0;
};
__device__ __forceinline__ SpinQ0 spin_q0(double nu, double nd, double su, double sd, double zab) {
  SpinQ0 r;
  const double n = nu + nd, inv_n = 1.0 / n;
  double X = 0.0, dxs[2] = {0.0, 0.0}, dss[2] = {0.0, 0.0}, ks[2] = {0.0, 0.0};
  const double ns[2] = {nu, nd}, ss[2] = {su, sd};
#pragma unroll
  for (int c = 0; c < 2; ++c) {
    if (ns[c] > 0.0) {
      const double k = cbrt(6.0 * kPi * kPi * ns[c]);
      ks[c] = k;
      const double inv_nk = 1.0 / (ns[c] * k);
      X += ns[c] * inv_n * k - (zab / 36.0) * ss[c] * inv_n * inv_nk;
      dxs[c] = (4.0 / 3.0) * k * inv_n + (zab / 27.0) * ss[c] * inv_n * inv_nk / ns[c];
      dss[c] = -(zab / 36.0) * inv_n * inv_nk;
    }
  }
  r.kF = cbrt(3.0 * kPi * kPi * n);
  r.rs = kRsKf / r.kF;
  const double sq = sqrt(r.rs);
  pw92(r.rs, r.e0, r.de0);
  double e1, de1, ma, dma;
  pw92_fit(kFerro, r.rs, sq, e1, de1);
  pw92_fit(kStiff, r.rs, sq, ma, dma);
  const double ac = -ma, dac = -dma;
  // a true division: at n_dn = 0 it gives zeta = 1 exactly, where f' holds (1 - zeta)^(1/3) and a
  // rounded 1 - 2^-53 would add cbrt(1e-16) ~ 5e-6 to it
  const double z = (nu - nd) / n;
  // (1 +- zeta)^(1/3) = (2 n_s / n)^(1/3) = k_s / k_F (zero for an empty channel)
  const double inv_kF = 1.0 / r.kF;
  const double cu = ks[0] * inv_kF, cd = ks[1] * inv_kF;
  const double fden = 1.0 / (2.0 * cbrt(2.0) - 2.0);   // 1 / (2^(4/3) - 2)
  const double f = ((1.0 + z) * cu + (1.0 - z) * cd - 2.0) * fden;
  const double df = (4.0 / 3.0) * (cu - cd) * fden;
  const double z3 = z * z * z, z4 = z3 * z;
  const double ec = r.e0 + ac * f / kFzz0 * (1.0 - z4) + (e1 - r.e0) * f * z4;
  const double dec_drs = r.de0 + dac * f / kFzz0 * (1.0 - z4) + (de1 - r.de0) * f * z4;
  const double dec_dz = ac / kFzz0 * (df * (1.0 - z4) - 4.0 * z3 * f) + (e1 - r.e0) * (df * z4 + 4.0 * z3 * f);
  const double c43 = 4.0 * kPi / 3.0;
  r.x = X - c43 * ec;
  const double drs = -r.rs * (1.0 / 3.0) * inv_n;
  r.dx[0] = dxs[0] - X * inv_n - c43 * (dec_drs * drs + dec_dz * (1.0 - z) * inv_n);
  r.dx[1] = dxs[1] - X * inv_n - c43 * (dec_drs * drs - dec_dz * (1.0 + z) * inv_n);
  r.dx[2] = dss[0];
  r.dx[3] = dss[1];
  return r;
}

// the spin densities as the functional takes them: cut at the vacuum threshold (NaN stays NaN)
__device__ __forceinline__ double spin_channel(double v) { return (v >= kVacuum || v != v) ? v : 0.0; }

constexpr int kSpinThreads = 256, kSpinBlocks = 4096;

// sigma_ss at point p: given (FROM_GRAD false), or |grad n_s|^2 from the gradient [3][npts]
template <bool FROM_GRAD>
__device__ __forceinline__ double spin_sigma(const double* __restrict__ s, long long p, long long npts) {
  if constexpr (FROM_GRAD) {
    const double a = s[p], b = s[npts + p], c = s[2 * npts + p];
    return a * a + b * b + c * c;
  } else {
    return s[p];
  }
}

// (n_up, n_dn, sigma_uu, sigma_dd) -> (n, sigma_eff) for the spin-paired pipeline (su, sd: the
// sigmas, or with FROM_GRAD the gradients of n_up, n_dn; suu_out, sdd_out, when given, receive the
// sigmas).  A NaN input gives NaN in both (the pipeline flags it).
template <bool FROM_GRAD>
__global__ void __launch_bounds__(kSpinThreads)
k_spin_in(const double* __restrict__ nu, const double* __restrict__ nd, const double* __restrict__ su,
          const double* __restrict__ sd, double* __restrict__ n_out, double* __restrict__ s_out,
          double* __restrict__ suu_out, double* __restrict__ sdd_out, double zab, long long npts) {
  for (long long p = (long long)blockIdx.x * kSpinThreads + threadIdx.x; p < npts;
       p += (long long)gridDim.x * kSpinThreads) {
    const double a = spin_channel(nu[p]), b = spin_channel(nd[p]);
    const double sa = spin_sigma<FROM_GRAD>(su, p, npts), sb = spin_sigma<FROM_GRAD>(sd, p, npts);
    const double n = a + b;
    double seff = 0.0;
    if (!(a == a) || !(b == b) || !(sa == sa) || !(sb == sb)) {
      seff = __builtin_nan("");
    } else if (n >= kVacuum) {
      const SpinQ0 q = spin_q0(a, b, sa, sb, zab);
      seff = (q.kF - (4.0 * kPi / 3.0) * q.e0 - q.x) * (36.0 / zab) * q.kF * n * n;
    }
    n_out[p] = n;
    s_out[p] = seff;
    if (suu_out) {   // the sigmas formed from the gradients, for k_spin_out
      suu_out[p] = sa;
      sdd_out[p] = sb;
    }
  }
}

// The pipeline's dE/dn|sigma_eff (in dnu) and dE/dsigma_eff (in dsu) -> the four spin partials,
// in place: dnu, dnd (which held n), dsu, dsd (which held sigma_eff).  su, sd as for k_spin_in.
template <bool FROM_GRAD>
__global__ void __launch_bounds__(kSpinThreads)
k_spin_out(const double* __restrict__ nu, const double* __restrict__ nd, const double* __restrict__ su,
           const double* __restrict__ sd, double* __restrict__ dnu, double* __restrict__ dnd,
           double* __restrict__ dsu, double* __restrict__ dsd, double zab, long long npts) {
  for (long long p = (long long)blockIdx.x * kSpinThreads + threadIdx.x; p < npts;
       p += (long long)gridDim.x * kSpinThreads) {
    const double n = dnd[p], seff = dsd[p], den = dnu[p], des = dsu[p];
    double o[4] = {den, den, 0.0, 0.0};
    // des = 0 where q0 is saturated or clamped (h' = 0): there dE/dn_s = dE/dn and no sigma
    // dependence, without forming 0 * (a possibly infinite sigma_eff term)
    if (n >= kVacuum && seff == seff && des != 0.0) {
      const double a = spin_channel(nu[p]), b = spin_channel(nd[p]);
      const SpinQ0 q = spin_q0(a, b, spin_sigma<FROM_GRAD>(su, p, npts), spin_sigma<FROM_GRAD>(sd, p, npts), zab);
      const double inv_n = 1.0 / n, inv_kn2 = inv_n * inv_n / q.kF;
      // the spin-paired x_u's partials at (n, sigma_eff), as the pipeline's q0 pass forms them
      const double dxdn_u = (1.0 / 3.0) * q.kF * inv_n + (4.0 * kPi / 9.0) * q.rs * inv_n * q.de0 +
                            (7.0 * zab / 108.0) * seff * inv_kn2 * inv_n;
      const double dxds_u = -(zab / 36.0) * inv_kn2;
      const double g = des / dxds_u;
      o[0] = den + g * (q.dx[0] - dxdn_u);
      o[1] = den + g * (q.dx[1] - dxdn_u);
      o[2] = g * q.dx[2];
      o[3] = g * q.dx[3];
    } else if (!(n >= kVacuum) && n == n) {
      o[0] = o[1] = 0.0;
    }
    dnu[p] = o[0];
    dnd[p] = o[1];
    dsu[p] = o[2];
    dsd[p] = o[3];
  }
}

// ---- pass 5: inverse z FFT + assembly of dE/dn, dE/dsigma (eqs. dedn, dedsigma) -------------
// dE/dn = sum_a F_a [p_a + n p_a' dq0/dn],  dE/dsigma = sum_a F_a n p_a' dq0/dsigma, with F_a(r)
// from the inverse transforms (1/N applied here).  The per-point spline state (b, t, n dq0/dn,
// n dq0/dsigma), computed in FP64 by the forward theta pass and stored in the path's precision,
// is read once into LDS; the two sums sit in FP64 registers.

template <typename T, int PPT, int EPT, int PB>
__global__ void __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 ? VDWXC_WPE_ASM : 1)))
k_zinv_assemble(const typename Cx<T>::type* __restrict__ A, const Quad<T>* __restrict__ state,
                double* __restrict__ dedn, double* __restrict__ dedsig,
                const double* __restrict__ qmesh, const double* __restrict__ mm,
                const typename Cx<T>::type* __restrict__ tw, Geometry g, AxisPlan zp, int ty, int lstride,
                const double* __restrict__ partials, int nparts, double escale, int* __restrict__ flag,
                double* __restrict__ energy, int sets) {
  using T2 = typename Cx<T>::type;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  unsigned char* smem = smem_raw + tw_lds_bytes<T2>(g.n3);
  const T2* twl = stage_twiddles(smem_raw, tw, g.n3, threadIdx.x, blockDim.x);
  const int tid = threadIdx.x, nthr = blockDim.x;
  // the energy of the evaluation (the contraction pass left its partials), in the first block,
  // with the line area of LDS as scratch before anything else uses it
  if (blockIdx.x == 0 && blockIdx.y == 0)
    energy_reduce_block(partials, nparts, escale, flag, energy, reinterpret_cast<double*>(smem), tid, nthr);
  int tile, x;
  zpass_block(tile, x);
  const int y0 = tile * ty;
  const int n3 = g.n3, M = g.M;
  const size_t N = size_t(g.n1) * g.n2 * n3;
  const int npts = ty * n3;
  T2* line = reinterpret_cast<T2*>(smem);   // `sets` (<= PB) line sets of ty lines, one per pair of a batch
  size_t off = size_t(sets) * ty * lstride * sizeof(T2);
  T* st_t = reinterpret_cast<T*>(smem + off);
  off += size_t(npts) * sizeof(T);
  T* st_an = reinterpret_cast<T*>(smem + off);
  off += size_t(npts) * sizeof(T);
  T* st_as = reinterpret_cast<T*>(smem + off);
  off += size_t(npts) * sizeof(T);
  unsigned char* st_b = smem + off;
  off += (size_t(npts) + 15) & ~size_t(15);
  const SplineLds<T> S = load_spline_lds<T>(smem, off, qmesh, mm, M, tid, nthr);
  __syncthreads();

  // the spline state of each point, as the forward theta pass left it
  gather_strided_dm<4>(
      tid, nthr, npts, n3,
      [&](int, int yl, int z) {
        const int y = y0 + yl;
        Quad<T> q{T(0), T(0), T(0), T(255)};
        if (y < g.n2) q = state[(size_t(x) * g.n2 + y) * n3 + z];
        return q;
      },
      [&](int p, int, int, const Quad<T>& q) {
        st_b[p] = (unsigned char)int(q.w);
        st_t[p] = q.x;
        st_an[p] = q.y;
        st_as[p] = q.z;
      });

  __syncthreads();
  // Per point, with F_a the inverse transforms and m_c,a = p_a''(q_c):
  //   sum_a F_a p_a  = u F_b + t F_b+1 + c6 [(u^3-u) X0 + (t^3-t) X1]
  //   sum_a F_a p_a' = (F_b+1 - F_b)/h + (h/6) [-(3u^2-1) X0 + (3t^2-1) X1]
  // with X0 = sum_a F_a m_b,a, X1 = sum_a F_a m_b+1,a (u = 1-t).  So each field costs one
  // F read and the two m entries of its pair, and the spline weights are formed once per point.
  double X0[PPT], X1[PPT];
  T Fb[PPT], Fb1[PPT];
  int bb[PPT], loff[PPT];   // spline interval (255: none) and LDS line offset of each point
  {
    DivModStep it(tid, nthr, n3);
#pragma unroll
    for (int c = 0; c < PPT; ++c, it.next()) {
      const int p = tid + c * nthr;
      bb[c] = p < npts ? st_b[p] : 255;
      loff[c] = it.q * lstride + lidx<>(it.r);
      X0[c] = X1[c] = 0.0;
      Fb[c] = Fb1[c] = T(0);
    }
  }
  // field pairs in batches of `sets`: one transform of sets * ty lines per batch (fewer, fuller FFT
  // stages), the next batch's half spectra in flight meanwhile
  const int npairs = (M + 1) >> 1;
  PairPrefetch<T2, EPT / 2 + 1> pf[PB];
#pragma unroll
  for (int q = 0; q < PB; ++q)
    if (q < sets && q < npairs) pf[q].issue(A, g, 2 * q, 2 * q + 1 < M ? 2 * q + 1 : -1, x, y0, ty, tid, nthr);
#pragma unroll 1
  for (int pr0 = 0; pr0 < npairs; pr0 += sets) {
    const int nb = min(sets, npairs - pr0);
#pragma unroll
    for (int q = 0; q < PB; ++q)
      if (q < nb) pf[q].store(g, ty, line + q * ty * lstride, lstride, tid, nthr);
    __syncthreads();
#pragma unroll
    for (int q = 0; q < PB; ++q) {
      const int pn = pr0 + sets + q;
      if (q < sets && pn < npairs) pf[q].issue(A, g, 2 * pn, 2 * pn + 1 < M ? 2 * pn + 1 : -1, x, y0, ty, tid, nthr);
    }
    lds_fft<PB * EPT, +1>(line, zp, nb * ty, lstride, twl, tid, nthr);
#pragma unroll
    for (int q = 0; q < PB; ++q) {
      if (q >= nb) break;
      const int fa = 2 * (pr0 + q), fb = fa + 1 < M ? fa + 1 : -1;
      const T2* lq = line + q * ty * lstride;
#pragma unroll
    for (int c = 0; c < PPT; ++c) {
      const int b = bb[c];
      if (b != 255) {
        const T2 F = lq[loff[c]];
        // m entries of fields fa, fa+1 at knots b and b+1 (adjacent in the transposed table)
        const T2 m0 = *reinterpret_cast<const T2*>(S.mmT + b * kMaxQ + fa);
        const T2 m1 = *reinterpret_cast<const T2*>(S.mmT + (b + 1) * kMaxQ + fa);
        const T m0y = fb >= 0 ? m0.y : T(0), m1y = fb >= 0 ? m1.y : T(0);
        X0[c] += double(F.x * m0.x + F.y * m0y);
        X1[c] += double(F.x * m1.x + F.y * m1y);
        if (fa == b) Fb[c] = F.x;
        if (fb == b) Fb[c] = F.y;
        if (fa == b + 1) Fb1[c] = F.x;
        if (fb == b + 1) Fb1[c] = F.y;
      }
    }
    }
    __syncthreads();
  }
  const double invN = 1.0 / double(N);
  DivModStep ot(tid, nthr, n3);
#pragma unroll
  for (int c = 0; c < PPT; ++c, ot.next()) {
    const int p = tid + c * nthr;
    if (p < npts) {
      const int yl = ot.q, z = ot.r, y = y0 + yl;
      if (y < g.n2) {
        double vn = 0.0, vs = 0.0;
        const int b = bb[c];
        if (b != 255) {
          const double t = st_t[p], an = st_an[p], as = st_as[p];
          const double hh = S.h[b], c6 = S.c6[b], u = 1.0 - t;
          const double fb0 = Fb[c], fb1 = Fb1[c];
          const double P = u * fb0 + t * fb1 + c6 * ((u * u * u - u) * X0[c] + (t * t * t - t) * X1[c]);
          const double D = (fb1 - fb0) / hh + hh * (1.0 / 6.0) * (-(3.0 * u * u - 1.0) * X0[c] + (3.0 * t * t - 1.0) * X1[c]);
          vn = P + an * D;
          vs = as * D;
        }
        const size_t idx = (size_t(x) * g.n2 + y) * n3 + z;
        dedn[idx] = vn * invN;
        dedsig[idx] = vs * invN;
      }
    }
  }
}

// The same pass for N3 = 512 (the counterpart of k_theta_zfwd512): thread t owns line (y) t / 64
// of the tile and the points z = t mod 64 + 64 r, which are exactly the outputs of its last
// inverse-transform stage.  Their spline state stays in registers, and the two spline sums of each
// point accumulate straight from that stage (no per-point state in LDS, no read of the transformed
// lines).  Field pairs go through the transform PB at a time; with PREFETCH the next batch's half
// spectra are in flight during the transform (more registers), else they are loaded after it.
// nthr = 64 ty.
template <typename T, int PB, int WPE, bool PREFETCH>
__global__ void __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(WPE)))
k_zinv_assemble512(const typename Cx<T>::type* __restrict__ A, const Quad<T>* __restrict__ state,
                   const unsigned char* __restrict__ sb,
                   double* __restrict__ dedn, double* __restrict__ dedsig, const double* __restrict__ qmesh,
                   const double* __restrict__ mm, const typename Cx<T>::type* __restrict__ tw, Geometry g, int ty,
                   int lstride, const double* __restrict__ partials, int nparts, double escale,
                   int* __restrict__ flag, double* __restrict__ energy) {
  using T2 = typename Cx<T>::type;
  constexpr int n3 = 512;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  unsigned char* smem = smem_raw + tw_lds_bytes<T2>(n3);
  const T2* twl = stage_twiddles(smem_raw, tw, n3, threadIdx.x, blockDim.x);
  const int tid = threadIdx.x, nthr = blockDim.x;
  // the energy of the evaluation (the contraction pass left its partials), in the first block,
  // with the line area of LDS as scratch before anything else uses it
  if (blockIdx.x == 0 && blockIdx.y == 0)
    energy_reduce_block(partials, nparts, escale, flag, energy, reinterpret_cast<double*>(smem), tid, nthr);
  int tile, x;
  zpass_block(tile, x);
  const int y0 = tile * ty, M = g.M;
  const size_t N = size_t(g.n1) * g.n2 * n3;
  T2* line = reinterpret_cast<T2*>(smem);   // PB line sets of ty lines
  const SplineLds<T> S = load_spline_lds<T>(smem, size_t(PB) * ty * lstride * sizeof(T2), qmesh, mm, M, tid, nthr);
  const int yl = __builtin_amdgcn_readfirstlane(tid >> 6), i = tid & 63, y = y0 + yl;
  const bool live = y < g.n2;
  const size_t pbase = (size_t(x) * g.n2 + y) * n3 + i;
  // the spline interval of the thread's points, as the forward theta pass left it in its byte
  // array (the rest of the state, t, n dq0/dn and n dq0/dsigma, is read after the transforms,
  // which keeps it out of the registers the transforms need)
  int pb[8];
#pragma unroll
  for (int r = 0; r < 8; ++r) pb[r] = live ? int(sb[pbase + 64 * r]) : 255;
  // Per point, with F_a the inverse transforms and m_c,a = p_a''(q_c):
  //   sum_a F_a p_a  = u F_b + t F_b+1 + c6 [(u^3-u) X0 + (t^3-t) X1]
  //   sum_a F_a p_a' = (F_b+1 - F_b)/h + (h/6) [-(3u^2-1) X0 + (3t^2-1) X1]
  // with X0 = sum_a F_a m_b,a, X1 = sum_a F_a m_b+1,a (u = 1-t), as in k_zinv_assemble.
  double X0[8], X1[8];
  T Fb[8], Fb1[8];
#pragma unroll
  for (int r = 0; r < 8; ++r) {
    X0[r] = X1[r] = 0.0;
    Fb[r] = Fb1[r] = T(0);
  }
  const int npairs = (M + 1) >> 1;
  PairPrefetch<T2, 5> pf[PB];   // ceil(ty * 257 / (64 ty)) = 5 half-spectrum values per field and thread
#pragma unroll
  for (int q = 0; q < PB; ++q)
    if (q < npairs) pf[q].issue(A, g, 2 * q, 2 * q + 1 < M ? 2 * q + 1 : -1, x, y0, ty, tid, nthr);
#pragma unroll 1
  for (int pr0 = 0; pr0 < npairs; pr0 += PB) {
    const int nb = min(PB, npairs - pr0);
    if (!PREFETCH && pr0 > 0) {
#pragma unroll
      for (int q = 0; q < PB; ++q)
        if (pr0 + q < npairs)
          pf[q].issue(A, g, 2 * (pr0 + q), 2 * (pr0 + q) + 1 < M ? 2 * (pr0 + q) + 1 : -1, x, y0, ty, tid, nthr);
    }
#pragma unroll
    for (int q = 0; q < PB; ++q)
      if (q < nb) pf[q].store(g, ty, line + q * ty * lstride, lstride, tid, nthr);
    __syncthreads();
    if (PREFETCH) {
#pragma unroll
      for (int q = 0; q < PB; ++q) {
        const int pn = pr0 + PB + q;
        if (pn < npairs) pf[q].issue(A, g, 2 * pn, 2 * pn + 1 < M ? 2 * pn + 1 : -1, x, y0, ty, tid, nthr);
      }
    }
    lds_fft512<PB, +1, kLdsPadShift>(
        line, nb * ty, lstride, twl, tid, nthr, LdsLines{}, [&](int l, int r, int, T2 F) {
          const int fa = 2 * (pr0 + (l - yl) / ty), fb = fa + 1 < M ? fa + 1 : -1;
          const int b = pb[r];
          if (b != 255) {
            // m entries of fields fa, fa+1 at knots b and b+1 (adjacent in the transposed table)
            const T2 m0 = *reinterpret_cast<const T2*>(S.mmT + b * kMaxQ + fa);
            const T2 m1 = *reinterpret_cast<const T2*>(S.mmT + (b + 1) * kMaxQ + fa);
            const T m0y = fb >= 0 ? m0.y : T(0), m1y = fb >= 0 ? m1.y : T(0);
            X0[r] += double(F.x * m0.x + F.y * m0y);
            X1[r] += double(F.x * m1.x + F.y * m1y);
            if (fa == b) Fb[r] = F.x;
            if (fb == b) Fb[r] = F.y;
            if (fa == b + 1) Fb1[r] = F.x;
            if (fb == b + 1) Fb1[r] = F.y;
          }
        });
  }
  if (live) {
    const double invN = 1.0 / double(N);
    Quad<T> stv[8];
#pragma unroll
    for (int r = 0; r < 8; ++r) stv[r] = ld<nt_site<T, kNtAsmState>()>(&state[pbase + 64 * r]);
#pragma unroll
    for (int r = 0; r < 8; ++r) {
      double vn = 0.0, vs = 0.0;
      const int b = pb[r];
      if (b != 255) {
        const double t = stv[r].x, an = stv[r].y, as = stv[r].z;
        const double hh = S.h[b], c6 = S.c6[b], u = 1.0 - t;
        const double fb0 = Fb[r], fb1 = Fb1[r];
        const double P = u * fb0 + t * fb1 + c6 * ((u * u * u - u) * X0[r] + (t * t * t - t) * X1[r]);
        const double D = (fb1 - fb0) / hh + hh * (1.0 / 6.0) * (-(3.0 * u * u - 1.0) * X0[r] + (3.0 * t * t - 1.0) * X1[r]);
        vn = P + an * D;
        vs = as * D;
      }
      st<nt_site<T, kNtAsmOut>()>(&dedn[pbase + 64 * r], vn * invN);
      st<nt_site<T, kNtAsmOut>()>(&dedsig[pbase + 64 * r], vs * invN);
    }
  }
}

// ---- spectral divergence, one axis at a time ---------------------------------------------------
// The divergence of h_c = 2 (dE/dsigma) g_c is (1/N) F^-1 [chi(m) sum_c i G_c F h_c] with G the
// wave vector of index m and chi zero wherever an index is a Nyquist index.  With G = sum_i m_i b_i
// (b_i the reciprocal vectors, m_i the signed indices), sum_c G_c h^_c = sum_i m_i H^_i for the
// real-space combinations H_i = sum_c b_i,c h_c, and chi = chi_1 chi_2 chi_3 factors over the axes.
// So the operator splits into one-dimensional ones along each axis of length n:
//   D = (1/n) F^-1 [i m chi(m)] F   (spectral derivative in index units, Nyquist dropped)
//   P = (1/n) F^-1 chi F            (removal of the Nyquist mode (-1)^x: an alternating sum;
//                                    the identity for odd n)
// and div = P_y P_z D_x H_1 + P_x P_z D_y H_2 + P_x P_y D_z H_3.  P_a commutes with D_b (b != a)
// and P_a D_a = D_a, which gives three line passes:
//   z: A = D_z H_3,            B1 = P_z H_1,  B2 = P_z H_2
//   y: A' = P_y A + D_y B2,    B1' = P_y B1
//   x: div = P_x A' + D_x B1'
// This is the same linear operator as the three-dimensional transform, with one derivative FFT
// pair per point and pass instead of forward transforms of three fields and an inverse of one.
// Each pass keeps whole lines of its axis in LDS: "P lines" (two real series as re/im of one
// complex line) get the projection, "D lines" (two real series packed the same way) the derivative
// through one forward and one inverse complex FFT.  The multiplier i m chi / n maps real series to
// real series, so the packed pair comes back as (D a, D b).

// loads in flight per thread in the divergence passes: each block streams its whole tile once,
// and one block per CU slot covers the grid at typical sizes, so the load latency is not hidden
// by other blocks
#ifndef VDWXC_DIV_U
#define VDWXC_DIV_U 8
#endif
constexpr int kDivU = VDWXC_DIV_U;

// np P lines and nd D lines of length plan.n in LDS (stride lstride).  On return the D lines hold
// their derivatives and csum[l] = (1/n) sum_x (-1)^x P_l[x] (zero for odd n); the caller subtracts
// (-1)^x csum[l] from P line l.  Requires nd * n <= nthr * EPT, nthr a multiple of 64, and the
// lines complete (synchronised) on entry; lines and csum are complete on return.
template <int EPT, typename T2>
__device__ __forceinline__ void project_and_derive(T2* pl, int np, T2* dl, int nd, T2* csum, int lstride,
                                                   const AxisPlan& plan, const T2* __restrict__ tw, int tid,
                                                   int nthr) {
  using T = decltype(pl[0].x);
  const int n = plan.n;
  const T invn = T(1) / T(n);
  if ((n & 1) == 0) {
    // one wave per P line: strided alternating partial sums, then a butterfly over the lanes
    const int lane = tid & 63, nwave = nthr >> 6;
    for (int l = tid >> 6; l < np; l += nwave) {
      T sx = T(0), sy = T(0);
      for (int i = lane; i < n; i += 64) {
        const T2 v = pl[l * lstride + lidx<>(i)];
        const T sg = (i & 1) ? T(-1) : T(1);
        sx += sg * v.x;
        sy += sg * v.y;
      }
      for (int off = 32; off > 0; off >>= 1) {
        sx += __shfl_xor(sx, off, 64);
        sy += __shfl_xor(sy, off, 64);
      }
      if (lane == 0) csum[l] = T2{sx * invn, sy * invn};
    }
  } else {
    for (int l = tid; l < np; l += nthr) csum[l] = T2{T(0), T(0)};
  }
  if (nd > 0) {
    lds_fft<EPT, -1>(dl, plan, nd, lstride, tw, tid, nthr);
    DivModStep it(tid, nthr, n);
    for (int e = tid; e < nd * n; e += nthr, it.next()) {
      const int l = it.q, m = it.r;
      const T mu = is_nyquist(m, n) ? T(0) : T(signed_freq(m, n)) * invn;
      T2& v = dl[l * lstride + lidx<>(m)];
      v = T2{-mu * v.y, mu * v.x};
    }
    __syncthreads();
    lds_fft<EPT, +1>(dl, plan, nd, lstride, tw, tid, nthr);
  } else {
    __syncthreads();
  }
}

// z pass.  Block: `ty` y lines of one x plane (the z-pass block order).  in: S = dE/dsigma and the
// three gradient components; out: [A, B1, B2] as three real fields of N points (natural order).
template <typename T, int EPT>
__global__ void __launch_bounds__(512)
k_div_z(const double* __restrict__ S, const double* __restrict__ grad, T* __restrict__ out,
        const typename Cx<T>::type* __restrict__ tw, Geometry g, AxisPlan zp, int ty, int lstride) {
  using T2 = typename Cx<T>::type;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  unsigned char* smem = smem_raw + tw_lds_bytes<T2>(g.n3);
  const T2* twl = stage_twiddles(smem_raw, tw, g.n3, threadIdx.x, blockDim.x);
  const int tid = threadIdx.x, nthr = blockDim.x;
  int tile, x;
  zpass_block(tile, x);
  const int y0 = tile * ty, n3 = g.n3;
  const size_t N = size_t(g.n1) * g.n2 * n3;
  const int nd = (ty + 1) >> 1, npts = ty * n3;
  T2* pl = reinterpret_cast<T2*>(smem);     // line yl: (H_1, H_2)
  T2* dl = pl + size_t(ty) * lstride;        // line j: (H_3 of yl = 2j, 2j+1)
  T2* csum = dl + size_t(nd) * lstride;
  struct In {
    double s, g0, g1, g2;
  };
  gather_strided_dm<kDivU>(
      tid, nthr, npts, n3,
      [&](int, int yl, int z) {
        const int y = y0 + yl;
        In r{0.0, 0.0, 0.0, 0.0};
        if (y < g.n2) {
          const size_t idx = (size_t(x) * g.n2 + y) * n3 + z;
          constexpr bool nt = nt_site<T, kNtDivZLoad>();
          r.s = ld<nt>(&S[idx]);
          r.g0 = ld<nt>(&grad[idx]);
          r.g1 = ld<nt>(&grad[N + idx]);
          r.g2 = ld<nt>(&grad[2 * N + idx]);
        }
        return r;
      },
      [&](int, int yl, int z, const In& r) {
        const double s2 = 2.0 * r.s;
        double H[3];
#pragma unroll
        for (int i = 0; i < 3; ++i) H[i] = s2 * (g.bvec[3 * i] * r.g0 + g.bvec[3 * i + 1] * r.g1 + g.bvec[3 * i + 2] * r.g2);
        pl[yl * lstride + lidx<>(z)] = T2{T(H[0]), T(H[1])};
        T* d = reinterpret_cast<T*>(dl + (yl >> 1) * lstride + lidx<>(z));
        d[yl & 1] = T(H[2]);
        if (!(yl & 1) && yl + 1 == ty) d[1] = T(0);   // odd tile: the last pair has one member
      });
  __syncthreads();
  project_and_derive<EPT>(pl, ty, dl, nd, csum, lstride, zp, twl, tid, nthr);
  DivModStep it(tid, nthr, n3);
  for (int e = tid; e < npts; e += nthr, it.next()) {
    const int yl = it.q, z = it.r, y = y0 + yl;
    if (y < g.n2) {
      const size_t idx = (size_t(x) * g.n2 + y) * n3 + z;
      const T2 p = pl[yl * lstride + lidx<>(z)], c = csum[yl];
      const T2 d = dl[(yl >> 1) * lstride + lidx<>(z)];
      const T sg = (z & 1) ? T(-1) : T(1);
      constexpr bool nt = nt_site<T, kNtDivZStore>();
      st<nt>(&out[idx], (yl & 1) ? d.y : d.x);
      st<nt>(&out[N + idx], p.x - sg * c.x);
      st<nt>(&out[2 * N + idx], p.y - sg * c.y);
    }
  }
}

// y pass.  Block: `tz` consecutive z of one x plane (grid: z tiles x n1, XCD-aware order, so the
// blocks that share the cache lines of a row run on one XCD).  in: [A, B1, B2]; out: [A', B1'].
template <typename T, int EPT>
__global__ void __launch_bounds__(512)
k_div_y(const T* __restrict__ in, T* __restrict__ out, const typename Cx<T>::type* __restrict__ tw, Geometry g,
        AxisPlan yp, int tz, int lstride) {
  using T2 = typename Cx<T>::type;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  unsigned char* smem = smem_raw + tw_lds_bytes<T2>(g.n2);
  const T2* twl = stage_twiddles(smem_raw, tw, g.n2, threadIdx.x, blockDim.x);
  const int tid = threadIdx.x, nthr = blockDim.x;
  const int L = xcd_logical_block(blockIdx.x + gridDim.x * blockIdx.y, gridDim.x * gridDim.y);
  const int z0 = (L % gridDim.x) * tz, x = L / gridDim.x;
  const int n2 = g.n2, n3 = g.n3;
  const size_t N = size_t(g.n1) * n2 * n3;
  const int nd = (tz + 1) >> 1, tot = tz * n2;
  T2* pl = reinterpret_cast<T2*>(smem);     // line zl: (A, B1)
  T2* dl = pl + size_t(tz) * lstride;        // line j: (B2 of zl = 2j, 2j+1)
  T2* csum = dl + size_t(nd) * lstride;
  struct In {
    T a, b1, b2;
  };
  gather_strided_dm<kDivU>(
      tid, nthr, tot, tz,
      [&](int, int y, int zl) {
        In r{T(0), T(0), T(0)};
        if (z0 + zl < n3) {
          const size_t idx = (size_t(x) * n2 + y) * n3 + z0 + zl;
          r.a = in[idx];
          r.b1 = in[N + idx];
          r.b2 = in[2 * N + idx];
        }
        return r;
      },
      [&](int, int y, int zl, const In& r) {
        pl[zl * lstride + lidx<>(y)] = T2{r.a, r.b1};
        T* d = reinterpret_cast<T*>(dl + (zl >> 1) * lstride + lidx<>(y));
        d[zl & 1] = r.b2;
        if (!(zl & 1) && zl + 1 == tz) d[1] = T(0);
      });
  __syncthreads();
  project_and_derive<EPT>(pl, tz, dl, nd, csum, lstride, yp, twl, tid, nthr);
  DivModStep it(tid, nthr, tz);
  for (int e = tid; e < tot; e += nthr, it.next()) {
    const int y = it.q, zl = it.r;
    if (z0 + zl < n3) {
      const size_t idx = (size_t(x) * n2 + y) * n3 + z0 + zl;
      const T2 p = pl[zl * lstride + lidx<>(y)], c = csum[zl];
      const T2 d = dl[(zl >> 1) * lstride + lidx<>(y)];
      const T sg = (y & 1) ? T(-1) : T(1);
      out[idx] = (p.x - sg * c.x) + ((zl & 1) ? d.y : d.x);
      out[N + idx] = p.y - sg * c.y;
    }
  }
}

// x pass.  Block: `tz` consecutive z of one y (grid: z tiles x n2, XCD-aware order).  in: [A', B1'];
// v -= P_x A' + D_x B1'.
template <typename T, int EPT>
__global__ void __launch_bounds__(512)
k_div_x(const T* __restrict__ in, double* __restrict__ v, const typename Cx<T>::type* __restrict__ tw, Geometry g,
        AxisPlan xp, int tz, int lstride) {
  using T2 = typename Cx<T>::type;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  unsigned char* smem = smem_raw + tw_lds_bytes<T2>(g.n1);
  const T2* twl = stage_twiddles(smem_raw, tw, g.n1, threadIdx.x, blockDim.x);
  const int tid = threadIdx.x, nthr = blockDim.x;
  const int L = xcd_logical_block(blockIdx.x + gridDim.x * blockIdx.y, gridDim.x * gridDim.y);
  const int z0 = (L % gridDim.x) * tz, y = L / gridDim.x;
  const int n1 = g.n1, n2 = g.n2, n3 = g.n3;
  const size_t N = size_t(n1) * n2 * n3;
  const int nd = (tz + 1) >> 1, tot = tz * n1;
  T2* pl = reinterpret_cast<T2*>(smem);     // line j: (A' of zl = 2j, 2j+1)
  T2* dl = pl + size_t(nd) * lstride;        // line j: (B1' of zl = 2j, 2j+1)
  T2* csum = dl + size_t(nd) * lstride;
  struct In {
    T a, b;
  };
  gather_strided_dm<kDivU>(
      tid, nthr, tot, tz,
      [&](int, int x, int zl) {
        In r{T(0), T(0)};
        if (z0 + zl < n3) {
          const size_t idx = (size_t(x) * n2 + y) * n3 + z0 + zl;
          r.a = in[idx];
          r.b = in[N + idx];
        }
        return r;
      },
      [&](int, int x, int zl, const In& r) {
        T* p = reinterpret_cast<T*>(pl + (zl >> 1) * lstride + lidx<>(x));
        T* d = reinterpret_cast<T*>(dl + (zl >> 1) * lstride + lidx<>(x));
        p[zl & 1] = r.a;
        d[zl & 1] = r.b;
        if (!(zl & 1) && zl + 1 == tz) p[1] = d[1] = T(0);
      });
  __syncthreads();
  project_and_derive<EPT>(pl, nd, dl, nd, csum, lstride, xp, twl, tid, nthr);
  gather_strided_dm<kDivU>(
      tid, nthr, tot, tz,
      [&](int, int x, int zl) { return z0 + zl < n3 ? v[(size_t(x) * n2 + y) * n3 + z0 + zl] : 0.0; },
      [&](int, int x, int zl, double old) {
        if (z0 + zl < n3) {
          const T2 p = pl[(zl >> 1) * lstride + lidx<>(x)], c = csum[zl >> 1];
          const T2 d = dl[(zl >> 1) * lstride + lidx<>(x)];
          const T sg = (x & 1) ? T(-1) : T(1);
          const T div = (zl & 1) ? (p.y - sg * c.y) + d.y : (p.x - sg * c.x) + d.x;
          v[(size_t(x) * n2 + y) * n3 + z0 + zl] = old - double(div);
        }
      });
}

// ---- spectral gradient, one axis at a time ----------------------------------------------------
// The same factorisation gives the gradient of n (every Nyquist frequency dropped):
// g_c = sum_i b_i,c d_i with d_x = P_y P_z D_x n, d_y = P_x P_z D_y n, d_z = P_x P_y D_z n, in
// three passes:
//   z: a = D_z n,  q = P_z n
//   y: a' = P_y a,  b = D_y q,  q' = P_y q
//   x: d_z = P_x a',  d_y = P_x b,  d_x = D_x q';  g_c = sum_i b_i,c d_i

// z pass.  Block: `ty` y lines of one x plane (the z-pass block order).  in: n; out: [a, q].
template <typename T, int EPT>
__global__ void __launch_bounds__(512)
k_grad_z(const double* __restrict__ nin, T* __restrict__ out, const typename Cx<T>::type* __restrict__ tw,
         Geometry g, AxisPlan zp, int ty, int lstride) {
  using T2 = typename Cx<T>::type;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  unsigned char* smem = smem_raw + tw_lds_bytes<T2>(g.n3);
  const T2* twl = stage_twiddles(smem_raw, tw, g.n3, threadIdx.x, blockDim.x);
  const int tid = threadIdx.x, nthr = blockDim.x;
  int tile, x;
  zpass_block(tile, x);
  const int y0 = tile * ty, n3 = g.n3;
  const size_t N = size_t(g.n1) * g.n2 * n3;
  const int nd = (ty + 1) >> 1, npts = ty * n3;
  T2* pl = reinterpret_cast<T2*>(smem);     // line j: n of yl = 2j, 2j+1 (for the projection)
  T2* dl = pl + size_t(nd) * lstride;        // the same values (for the derivative)
  T2* csum = dl + size_t(nd) * lstride;
  gather_strided_dm<kDivU>(
      tid, nthr, npts, n3,
      [&](int, int yl, int z) {
        const int y = y0 + yl;
        return y < g.n2 ? nin[(size_t(x) * g.n2 + y) * n3 + z] : 0.0;
      },
      [&](int, int yl, int z, double v) {
        T* pp = reinterpret_cast<T*>(pl + (yl >> 1) * lstride + lidx<>(z));
        T* dd = reinterpret_cast<T*>(dl + (yl >> 1) * lstride + lidx<>(z));
        pp[yl & 1] = dd[yl & 1] = T(v);
        if (!(yl & 1) && yl + 1 == ty) pp[1] = dd[1] = T(0);   // odd tile: the last pair has one member
      });
  __syncthreads();
  project_and_derive<EPT>(pl, nd, dl, nd, csum, lstride, zp, twl, tid, nthr);
  DivModStep it(tid, nthr, n3);
  for (int e = tid; e < npts; e += nthr, it.next()) {
    const int yl = it.q, z = it.r, y = y0 + yl;
    if (y < g.n2) {
      const size_t idx = (size_t(x) * g.n2 + y) * n3 + z;
      const T2 pv = pl[(yl >> 1) * lstride + lidx<>(z)], c = csum[yl >> 1];
      const T2 d = dl[(yl >> 1) * lstride + lidx<>(z)];
      const T sg = (z & 1) ? T(-1) : T(1);
      out[idx] = (yl & 1) ? d.y : d.x;
      out[N + idx] = (yl & 1) ? pv.y - sg * c.y : pv.x - sg * c.x;
    }
  }
}

// y pass.  Block: `tz` consecutive z of one x plane (grid: z tiles x n1, XCD-aware order).
// in: [a, q]; out: [a', b, q'].
template <typename T, int EPT>
__global__ void __launch_bounds__(512)
k_grad_y(const T* __restrict__ in, T* __restrict__ out, const typename Cx<T>::type* __restrict__ tw, Geometry g,
         AxisPlan yp, int tz, int lstride) {
  using T2 = typename Cx<T>::type;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  unsigned char* smem = smem_raw + tw_lds_bytes<T2>(g.n2);
  const T2* twl = stage_twiddles(smem_raw, tw, g.n2, threadIdx.x, blockDim.x);
  const int tid = threadIdx.x, nthr = blockDim.x;
  const int L = xcd_logical_block(blockIdx.x + gridDim.x * blockIdx.y, gridDim.x * gridDim.y);
  const int z0 = (L % gridDim.x) * tz, x = L / gridDim.x;
  const int n2 = g.n2, n3 = g.n3;
  const size_t N = size_t(g.n1) * n2 * n3;
  const int nd = (tz + 1) >> 1, tot = tz * n2;
  T2* pl = reinterpret_cast<T2*>(smem);     // line zl: (a, q)
  T2* dl = pl + size_t(tz) * lstride;        // line j: (q of zl = 2j, 2j+1)
  T2* csum = dl + size_t(nd) * lstride;
  struct In {
    T a, q;
  };
  gather_strided_dm<kDivU>(
      tid, nthr, tot, tz,
      [&](int, int y, int zl) {
        In r{T(0), T(0)};
        if (z0 + zl < n3) {
          const size_t idx = (size_t(x) * n2 + y) * n3 + z0 + zl;
          r.a = in[idx];
          r.q = in[N + idx];
        }
        return r;
      },
      [&](int, int y, int zl, const In& r) {
        pl[zl * lstride + lidx<>(y)] = T2{r.a, r.q};
        T* d = reinterpret_cast<T*>(dl + (zl >> 1) * lstride + lidx<>(y));
        d[zl & 1] = r.q;
        if (!(zl & 1) && zl + 1 == tz) d[1] = T(0);
      });
  __syncthreads();
  project_and_derive<EPT>(pl, tz, dl, nd, csum, lstride, yp, twl, tid, nthr);
  DivModStep it(tid, nthr, tz);
  for (int e = tid; e < tot; e += nthr, it.next()) {
    const int y = it.q, zl = it.r;
    if (z0 + zl < n3) {
      const size_t idx = (size_t(x) * n2 + y) * n3 + z0 + zl;
      const T2 p = pl[zl * lstride + lidx<>(y)], c = csum[zl];
      const T2 d = dl[(zl >> 1) * lstride + lidx<>(y)];
      const T sg = (y & 1) ? T(-1) : T(1);
      out[idx] = p.x - sg * c.x;
      out[N + idx] = (zl & 1) ? d.y : d.x;
      out[2 * N + idx] = p.y - sg * c.y;
    }
  }
}

// x pass.  Block: `tz` consecutive z of one y (grid: z tiles x n2, XCD-aware order).
// in: [a', b, q']; out: the gradient [3][N] in FP64.
template <typename T, int EPT>
__global__ void __launch_bounds__(512)
k_grad_x(const T* __restrict__ in, double* __restrict__ gout, const typename Cx<T>::type* __restrict__ tw,
         Geometry g, AxisPlan xp, int tz, int lstride) {
  using T2 = typename Cx<T>::type;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  unsigned char* smem = smem_raw + tw_lds_bytes<T2>(g.n1);
  const T2* twl = stage_twiddles(smem_raw, tw, g.n1, threadIdx.x, blockDim.x);
  const int tid = threadIdx.x, nthr = blockDim.x;
  const int L = xcd_logical_block(blockIdx.x + gridDim.x * blockIdx.y, gridDim.x * gridDim.y);
  const int z0 = (L % gridDim.x) * tz, y = L / gridDim.x;
  const int n1 = g.n1, n2 = g.n2, n3 = g.n3;
  const size_t N = size_t(n1) * n2 * n3;
  const int nd = (tz + 1) >> 1, tot = tz * n1;
  T2* pl = reinterpret_cast<T2*>(smem);     // line zl: (a', b)
  T2* dl = pl + size_t(tz) * lstride;        // line j: (q' of zl = 2j, 2j+1)
  T2* csum = dl + size_t(nd) * lstride;
  struct In {
    T a, b, q;
  };
  gather_strided_dm<kDivU>(
      tid, nthr, tot, tz,
      [&](int, int x, int zl) {
        In r{T(0), T(0), T(0)};
        if (z0 + zl < n3) {
          const size_t idx = (size_t(x) * n2 + y) * n3 + z0 + zl;
          r.a = in[idx];
          r.b = in[N + idx];
          r.q = in[2 * N + idx];
        }
        return r;
      },
      [&](int, int x, int zl, const In& r) {
        pl[zl * lstride + lidx<>(x)] = T2{r.a, r.b};
        T* d = reinterpret_cast<T*>(dl + (zl >> 1) * lstride + lidx<>(x));
        d[zl & 1] = r.q;
        if (!(zl & 1) && zl + 1 == tz) d[1] = T(0);
      });
  __syncthreads();
  project_and_derive<EPT>(pl, tz, dl, nd, csum, lstride, xp, twl, tid, nthr);
  DivModStep it(tid, nthr, tz);
  for (int e = tid; e < tot; e += nthr, it.next()) {
    const int x = it.q, zl = it.r;
    if (z0 + zl < n3) {
      const size_t idx = (size_t(x) * n2 + y) * n3 + z0 + zl;
      const T2 p = pl[zl * lstride + lidx<>(x)], c = csum[zl];
      const T2 d = dl[(zl >> 1) * lstride + lidx<>(x)];
      const T sg = (x & 1) ? T(-1) : T(1);
      const double dz = double(p.x - sg * c.x), dy = double(p.y - sg * c.y);
      const double dx = double((zl & 1) ? d.y : d.x);
#pragma unroll
      for (int cc = 0; cc < 3; ++cc)
        gout[size_t(cc) * N + idx] = g.bvec[cc] * dx + g.bvec[3 + cc] * dy + g.bvec[6 + cc] * dz;
    }
  }
}

}  // namespace vdwxc
