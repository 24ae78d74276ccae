// Batched 1D FFTs of lines held in LDS, for gfx950 (64-wide wavefronts).
//
// A workgroup owns `nlines` lines of length n, stored in LDS at buf[l*lstride + lidx(i)].  Each radix-R
// stage is a Stockham autosort step: butterfly i (0 <= i < n/R) of a line reads the R elements
// i + r*n/R, applies twiddles exp(-+2 pi i r k/(pR)) with k = i mod p (p = product of the radices
// already done), runs an R-point DFT and writes element (i - k)*R + k + r*p.  Output is in natural
// order after the last stage.  A stage is two-phase: every thread first pulls its butterflies
// into registers, the workgroup synchronises, and then all threads write back in place, so one
// LDS buffer suffices.  The transforms are unnormalised; DIR = -1 is the forward direction
// exp(-2 pi i jm/n), DIR = +1 the inverse.
#pragma once
#include <hip/hip_runtime.h>

#include <type_traits>

namespace vdwxc {

constexpr int kMaxStages = 16;

// Position of element i of a line in LDS: one padding slot after every 2^kLdsPadShift elements,
// so the strided writes of the early Stockham stages (stride R, then groups of p) spread over the
// LDS banks.  A line of n elements occupies lds_span(n) slots.
#ifndef VDWXC_LDS_PAD_SHIFT
#define VDWXC_LDS_PAD_SHIFT 3
#endif
constexpr int kLdsPadShift = VDWXC_LDS_PAD_SHIFT;
constexpr int kNoPad = 31;
// kSwizzle: no padding; instead the low five index bits are XORed with bits 3..7 (a permutation of
// every aligned group of 32 elements, so lines take a multiple of 32 slots).  The Stockham stages
// read at unit stride and write at stride R p; the XOR spreads both over distinct banks without
// the extra LDS of padding.
constexpr int kSwizzle = 32;
template <int PS = kLdsPadShift>
__host__ __device__ constexpr int lidx(int i) {
  if constexpr (PS == kSwizzle) {
    return i ^ ((i >> 3) & 31);
  } else {
    return i + (i >> PS);
  }
}
template <int PS = kLdsPadShift>
__host__ __device__ constexpr int lds_span(int n) {
  if constexpr (PS == kSwizzle) {
    return (n + 31) & ~31;
  } else {
    return n <= 0 ? 0 : lidx<PS>(n - 1) + 1;
  }
}

// Radix schedule of one transform length: radices 16, 8, 4, 2, 3, 5, 7.  mnb[s] and mp[s] divide
// by n / radix[s] and by p_s (the product of the radices before stage s) without a division:
// x / d = umulhi(x, ceil(2^32 / d)), exact whenever x d < 2^32 (here x < 2^14, d <= 2^11);
// 0 encodes d = 1.
struct AxisPlan {
  int n;
  int nst;
  int linear;   // every stage meets the conditions of the LIN addressing (padded layouts)
  int radix[kMaxStages];
  unsigned mnb[kMaxStages], mp[kMaxStages];
};

inline unsigned div_magic(unsigned d) { return d <= 1 ? 0u : unsigned((0x100000000ull + d - 1) / d); }
__device__ __forceinline__ int fast_div(int x, unsigned m) { return m ? int(__umulhi(unsigned(x), m)) : x; }

template <typename T> struct Cx;
template <> struct Cx<float> { using type = float2; };
template <> struct Cx<double> { using type = double2; };

template <typename T2> __device__ __forceinline__ T2 cadd(T2 a, T2 b) { return T2{a.x + b.x, a.y + b.y}; }
template <typename T2> __device__ __forceinline__ T2 csub(T2 a, T2 b) { return T2{a.x - b.x, a.y - b.y}; }
template <typename T2> __device__ __forceinline__ T2 cmul(T2 a, T2 b) {
  return T2{a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
// multiply by -i (DIR=-1) or +i (DIR=+1)
template <int DIR, typename T2> __device__ __forceinline__ T2 rot90(T2 a) {
  return DIR < 0 ? T2{a.y, -a.x} : T2{-a.y, a.x};
}

// ---- small DFTs, in place on v[0..R-1] -------------------------------------------------------

template <int R, int DIR, typename T2> struct SmallDft;

template <int DIR, typename T2> struct SmallDft<2, DIR, T2> {
  __device__ __forceinline__ static void run(T2* v) {
    T2 a = v[0], b = v[1];
    v[0] = cadd(a, b);
    v[1] = csub(a, b);
  }
};

template <int DIR, typename T2> struct SmallDft<4, DIR, T2> {
  __device__ __forceinline__ static void run(T2* v) {
    T2 t0 = cadd(v[0], v[2]), t1 = csub(v[0], v[2]);
    T2 t2 = cadd(v[1], v[3]), t3 = rot90<DIR>(csub(v[1], v[3]));
    v[0] = cadd(t0, t2);
    v[2] = csub(t0, t2);
    v[1] = cadd(t1, t3);
    v[3] = csub(t1, t3);
  }
};

template <int DIR, typename T2> struct SmallDft<8, DIR, T2> {
  __device__ __forceinline__ static void run(T2* v) {
    using T = decltype(v[0].x);
    const T s = T(0.7071067811865475244008444);
    T2 e[4] = {v[0], v[2], v[4], v[6]};
    T2 o[4] = {v[1], v[3], v[5], v[7]};
    SmallDft<4, DIR, T2>::run(e);
    SmallDft<4, DIR, T2>::run(o);
    // o[k] *= exp(DIR * 2 pi i k / 8)
    o[1] = T2{s * (o[1].x - DIR * o[1].y), s * (o[1].y + DIR * o[1].x)};
    o[2] = rot90<DIR>(o[2]);
    o[3] = T2{-s * (o[3].x + DIR * o[3].y), s * (DIR * o[3].x - o[3].y)};
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      v[k] = cadd(e[k], o[k]);
      v[k + 4] = csub(e[k], o[k]);
    }
  }
};

// 16 = 4 x 4: DFT-4 over the four interleaved quarter sequences x[4a + b], twiddle by
// exp(DIR 2 pi i b c / 16), then DFT-4 across b; output c + 4 d.
template <int DIR, typename T2> struct SmallDft<16, DIR, T2> {
  template <typename T>
  __device__ __forceinline__ static T2 turn(T2 a, T c, T s) {   // a * (c + DIR i s)
    return T2{c * a.x - DIR * s * a.y, c * a.y + DIR * s * a.x};
  }
  __device__ __forceinline__ static void run(T2* v) {
    using T = decltype(v[0].x);
    const T c1 = T(0.9238795325112867561281832), s1 = T(0.3826834323650897717284600);
    const T h = T(0.7071067811865475244008444);
    T2 y[4][4];
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      y[b][0] = v[b]; y[b][1] = v[4 + b]; y[b][2] = v[8 + b]; y[b][3] = v[12 + b];
      SmallDft<4, DIR, T2>::run(y[b]);
    }
    y[1][1] = turn(y[1][1], c1, s1);
    y[1][2] = turn(y[1][2], h, h);
    y[1][3] = turn(y[1][3], s1, c1);
    y[2][1] = turn(y[2][1], h, h);
    y[2][2] = rot90<DIR>(y[2][2]);
    y[2][3] = turn(y[2][3], -h, h);
    y[3][1] = turn(y[3][1], s1, c1);
    y[3][2] = turn(y[3][2], -h, h);
    y[3][3] = turn(y[3][3], -c1, -s1);
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      T2 z[4] = {y[0][c], y[1][c], y[2][c], y[3][c]};
      SmallDft<4, DIR, T2>::run(z);
#pragma unroll
      for (int d = 0; d < 4; ++d) v[c + 4 * d] = z[d];
    }
  }
};

template <int DIR, typename T2> struct SmallDft<3, DIR, T2> {
  __device__ __forceinline__ static void run(T2* v) {
    using T = decltype(v[0].x);
    const T h = T(0.8660254037844386467637232);
    T2 t = cadd(v[1], v[2]);
    T2 s = csub(v[1], v[2]);
    T2 m = T2{v[0].x - T(0.5) * t.x, v[0].y - T(0.5) * t.y};
    T2 r = rot90<DIR>(T2{h * s.x, h * s.y});
    v[0] = cadd(v[0], t);
    v[1] = cadd(m, r);
    v[2] = csub(m, r);
  }
};

// odd radices 5 and 7: pairs (j, R-j) combine into cosine and sine sums
template <int R> struct OddTrig;
template <> struct OddTrig<5> {
  __device__ __forceinline__ static double c(int t) {
    return t == 1 || t == 4 ? 0.3090169943749474241022934 : -0.8090169943749474241022934;
  }
  __device__ __forceinline__ static double s(int t) {
    return t == 1 ? 0.9510565162951535721164393 : t == 2 ? 0.5877852522924731291687060
         : t == 3 ? -0.5877852522924731291687060 : -0.9510565162951535721164393;
  }
};
template <> struct OddTrig<7> {
  __device__ __forceinline__ static double c(int t) {
    return (t == 1 || t == 6) ? 0.6234898018587335305250049
         : (t == 2 || t == 5) ? -0.2225209339563144042889026 : -0.9009688679024191262361023;
  }
  __device__ __forceinline__ static double s(int t) {
    return t == 1 ? 0.7818314824680298087084445 : t == 2 ? 0.9749279121818236070181317
         : t == 3 ? 0.4338837391175581204757683 : t == 4 ? -0.4338837391175581204757683
         : t == 5 ? -0.9749279121818236070181317 : -0.7818314824680298087084445;
  }
};

template <int R, int DIR, typename T2> struct OddDft {
  __device__ __forceinline__ static void run(T2* v) {
    using T = decltype(v[0].x);
    constexpr int H = (R - 1) / 2;
    T2 A[H], B[H];
#pragma unroll
    for (int j = 1; j <= H; ++j) {
      A[j - 1] = cadd(v[j], v[R - j]);
      B[j - 1] = csub(v[j], v[R - j]);
    }
    T2 x0 = v[0];
    T2 sum = x0;
#pragma unroll
    for (int j = 0; j < H; ++j) sum = cadd(sum, A[j]);
#pragma unroll
    for (int k = 1; k <= H; ++k) {
      T2 cs = x0, sn = T2{T(0), T(0)};
#pragma unroll
      for (int j = 1; j <= H; ++j) {
        const T c = T(OddTrig<R>::c((j * k) % R));
        const T s = T(OddTrig<R>::s((j * k) % R));
        cs.x += c * A[j - 1].x;
        cs.y += c * A[j - 1].y;
        sn.x += s * B[j - 1].x;
        sn.y += s * B[j - 1].y;
      }
      // forward: X[k] = cs - i sn, X[R-k] = cs + i sn; inverse swaps the signs
      T2 isn = rot90<DIR>(sn);
      v[k] = cadd(cs, isn);
      v[R - k] = csub(cs, isn);
    }
    v[0] = sum;
  }
};
template <int DIR, typename T2> struct SmallDft<5, DIR, T2> : OddDft<5, DIR, T2> {};
template <int DIR, typename T2> struct SmallDft<7, DIR, T2> : OddDft<7, DIR, T2> {};

// ---- one Stockham stage on LDS lines ---------------------------------------------------------

// LIN (padded layout, plan.linear): with blocks of B = 2^PS slots, lidx(a + b) = lidx(a) + lidx(b)
// whenever a or b is a multiple of B.  In a linear plan every stage has B | n/R, B | pR and p | B or
// B | p, so a butterfly's reads at i + r n/R sit at the stage-uniform offsets lidx(r n/R) from
// lidx(i), and its writes at dst + r p at lidx(r p) from lidx(dst): one address per butterfly
// instead of index arithmetic per element.
template <int R, int MAXB, int DIR, int PS, bool LIN, typename T2>
__device__ __forceinline__ void fft_stage(T2* buf, int n, int nlines, int lstride, int p, unsigned mnb, unsigned mp,
                                          const T2* __restrict__ tw, int tid, int nthr) {
  const int nb = n / R;
  const int total = nb * nlines;
  const int twstep = n / (p * R);
  T2 v[MAXB][R];
  int dst[MAXB], wbase[MAXB];
#pragma unroll
  for (int c = 0; c < MAXB; ++c) {
    const int b = tid + c * nthr;
    dst[c] = -1;
    if (b < total) {
      const int l = fast_div(b, mnb);
      const int i = b - l * nb;
      const int k = i - fast_div(i, mp) * p;
      const T2* src = buf + l * lstride;
      if constexpr (LIN) {
        const T2* s0 = src + lidx<PS>(i);
#pragma unroll
        for (int r = 0; r < R; ++r) v[c][r] = s0[lidx<PS>(r * nb)];
      } else {
#pragma unroll
        for (int r = 0; r < R; ++r) v[c][r] = src[lidx<PS>(i + r * nb)];
      }
      if (p > 1) {
        // twiddle r is exp(-+2 pi i r k / (p R)) = tw[r k twstep]: a running index, no multiplies
        const int kt = k * twstep;
        int to = 0;
#pragma unroll
        for (int r = 1; r < R; ++r) {
          to += kt;
          T2 w = tw[to];
          if (DIR > 0) w.y = -w.y;
          v[c][r] = cmul(v[c][r], w);
        }
      }
      SmallDft<R, DIR, T2>::run(v[c]);
      dst[c] = (i - k) * R + k;
      wbase[c] = l * lstride + (LIN ? lidx<PS>(dst[c]) : 0);
    }
  }
  __syncthreads();
#pragma unroll
  for (int c = 0; c < MAXB; ++c) {
    if (dst[c] >= 0) {
      T2* d = buf + wbase[c];
      if constexpr (LIN) {
#pragma unroll
        for (int r = 0; r < R; ++r) d[lidx<PS>(r * p)] = v[c][r];
      } else {
#pragma unroll
        for (int r = 0; r < R; ++r) d[lidx<PS>(dst[c] + r * p)] = v[c][r];
      }
    }
  }
  __syncthreads();
}

// Transform `nlines` LDS lines of length plan.n.  Requires nlines * n <= nthr * EPT.  The caller
// must have synchronised after filling the lines; the lines are complete on return.  The plan
// lists its radices grouped (all 16s, then 8s, 4, 2, 3s, 5s, 7s), so each radix runs in its own loop
// and the register allocation of one stage kind does not inflate the others.
template <int R, int EPT, int DIR, int PS, bool LIN, typename T2>
__device__ __forceinline__ void run_stages(T2* buf, const AxisPlan& plan, int n, int count, int& s0, int& p,
                                           int nlines, int lstride, const T2* __restrict__ tw, int tid, int nthr) {
  for (int s = 0; s < count; ++s, ++s0) {
    fft_stage<R, (EPT + R - 1) / R, DIR, PS, LIN>(buf, n, nlines, lstride, p, plan.mnb[s0], plan.mp[s0], tw, tid,
                                                  nthr);
    p *= R;
  }
}

template <int EPT, int DIR, int PS, bool LIN, typename T2>
__device__ __forceinline__ void lds_fft_stages(T2* buf, const AxisPlan& plan, int n, int nlines, int lstride,
                                               const T2* __restrict__ tw, int tid, int nthr) {
  int cnt[7] = {0, 0, 0, 0, 0, 0, 0};   // radix 16, 8, 4, 2, 3, 5, 7
  for (int s = 0; s < plan.nst; ++s) {
    const int R = plan.radix[s];
    cnt[R == 16 ? 0 : R == 8 ? 1 : R == 4 ? 2 : R == 2 ? 3 : R == 3 ? 4 : R == 5 ? 5 : 6] += 1;
  }
  int p = 1, s0 = 0;
  run_stages<16, EPT, DIR, PS, LIN>(buf, plan, n, cnt[0], s0, p, nlines, lstride, tw, tid, nthr);
  run_stages<8, EPT, DIR, PS, LIN>(buf, plan, n, cnt[1], s0, p, nlines, lstride, tw, tid, nthr);
  run_stages<4, EPT, DIR, PS, LIN>(buf, plan, n, cnt[2], s0, p, nlines, lstride, tw, tid, nthr);
  run_stages<2, EPT, DIR, PS, LIN>(buf, plan, n, cnt[3], s0, p, nlines, lstride, tw, tid, nthr);
  run_stages<3, EPT, DIR, PS, LIN>(buf, plan, n, cnt[4], s0, p, nlines, lstride, tw, tid, nthr);
  run_stages<5, EPT, DIR, PS, LIN>(buf, plan, n, cnt[5], s0, p, nlines, lstride, tw, tid, nthr);
  run_stages<7, EPT, DIR, PS, LIN>(buf, plan, n, cnt[6], s0, p, nlines, lstride, tw, tid, nthr);
}

// ---- 512-point lines: three radix-8 stages with per-thread constants ---------------------------
// For n = 512 = 8 * 8 * 8 every stage has 64 butterflies per line, and a block of nthr threads
// (a multiple of 64) gives thread t the butterfly column i = t mod 64 of lines t / 64 + c nthr / 64.
// i is the same in all three stages and on every line of the thread, so are k = i mod p (p = 1, 8,
// 64 before the stage) and with them every LDS offset and twiddle of the thread:
//   reads of every stage, writes of the last:  i + 64 r
//   writes of stage 1 (p = 1, k = 0):          8 i + r
//   writes of stage 2 (p = 8, k = i mod 8):    8 (i - k) + k + 8 r
//   twiddles of stage 2: exp(-+2 pi i r k / 64) = tw[8 r k];  of stage 3: exp(-+2 pi i r i / 512) = tw[r i]
// so they are formed once per transform instead of once per butterfly and stage (the generic
// stage above recomputes the line, column and k of every butterfly, then each address and the
// twiddle index; that index arithmetic cost about as much as the butterfly itself).
// Where the first stage takes its inputs and the last stage puts its outputs: the LDS lines
// themselves (LdsLines), or a functor in(l, r, x) returning element x = i + 64 r of line l /
// out(l, r, x, v) storing it, e.g. straight from and to global memory when the lines are contiguous
// there, or from and to per-point registers of the caller (r is a compile-time index: element r of
// the thread's 8 per line).  64 consecutive threads access 64 consecutive elements of one line.
struct LdsLines {};

// Order a wave's own LDS accesses across this point (its earlier reads and writes complete before
// its later ones), without waiting for the other waves of the block.  WAVE = 0: a block barrier.
#ifndef VDWXC_FFT512_WAVESYNC
#define VDWXC_FFT512_WAVESYNC 1
#endif
template <int WAVE>
__device__ __forceinline__ void wave_lds_sync() {
  if constexpr (WAVE) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_s_waitcnt(0xc07f);   // lgkmcnt(0): the wave's LDS operations have completed
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  } else {
    __syncthreads();
  }
}

// END_SYNC: end with a block barrier (the caller then may read or reuse every line); without it
// (only with an output functor) the caller orders later LDS use itself.
template <int MAXB, int DIR, int PS, bool END_SYNC = true, typename T2, typename In = LdsLines, typename Out = LdsLines>
__device__ __forceinline__ void lds_fft512(T2* buf, int nlines, int lstride, const T2* __restrict__ tw, int tid,
                                           int nthr, In in = In{}, Out out = Out{}) {
  constexpr bool kInLds = std::is_same<In, LdsLines>::value, kOutLds = std::is_same<Out, LdsLines>::value;
  int i = tid & 63;
  // the offsets and twiddles below depend on the thread alone: without this the compiler shares
  // them between the transforms of one kernel, or hoists them out of a caller's loop, and keeps
  // them live (and the caller's registers spilled) in between
  asm volatile("" : "+v"(i));
  // a wave is 64 consecutive threads, so its line index is uniform over the wave: keep it scalar,
  // so that line bases (in LDS and in global memory) are scalar too
  const int l0 = __builtin_amdgcn_readfirstlane(tid >> 6), lstep = nthr >> 6;
  const int k2 = i & 7;
  int ro[8];
#pragma unroll
  for (int r = 0; r < 8; ++r) ro[r] = lidx<PS>(i + 64 * r);
#pragma unroll
  for (int s = 0; s < 3; ++s) {
    T2 w[8];
    if (s > 0) {
#pragma unroll
      for (int r = 1; r < 8; ++r) {
        w[r] = tw[s == 1 ? 8 * r * k2 : r * i];
        if (DIR > 0) w[r].y = -w[r].y;
      }
    }
    T2 v[MAXB][8];
    // all of the thread's loads first (several in flight), then the arithmetic
#pragma unroll
    for (int c = 0; c < MAXB; ++c) {
      const int l = l0 + c * lstep;
      if (l < nlines) {
        const T2* src = buf + l * lstride;
#pragma unroll
        for (int r = 0; r < 8; ++r) {
          if constexpr (!kInLds) {
            if (s == 0) {
              v[c][r] = in(l, r, i + 64 * r);
              continue;
            }
          }
          v[c][r] = src[ro[r]];
        }
      }
    }
#pragma unroll
    for (int c = 0; c < MAXB; ++c) {
      if (l0 + c * lstep < nlines) {
        if (s > 0) {
#pragma unroll
          for (int r = 1; r < 8; ++r) v[c][r] = cmul(v[c][r], w[r]);
        }
        SmallDft<8, DIR, T2>::run(v[c]);
      }
    }
    if (!kOutLds && s == 2) {
      // the last stage's outputs go straight to the caller (no LDS write, no barrier before it)
#pragma unroll
      for (int c = 0; c < MAXB; ++c) {
        const int l = l0 + c * lstep;
        if (l < nlines) {
#pragma unroll
          for (int r = 0; r < 8; ++r) {
            if constexpr (!kOutLds) out(l, r, i + 64 * r, v[c][r]);
          }
        }
      }
    } else {
      // every line is read and written by one wave only (lines l0 + c lstep), so between stages
      // the wave orders its own LDS accesses; the block synchronises only after the last stage.
      // (Twiddles in LDS must therefore be complete before the call: the caller's barrier.)
      wave_lds_sync<VDWXC_FFT512_WAVESYNC>();
      int wo[8];
#pragma unroll
      for (int r = 0; r < 8; ++r)
        wo[r] = s == 0 ? lidx<PS>(8 * i + r) : s == 1 ? lidx<PS>(8 * (i - k2) + k2 + 8 * r) : ro[r];
#pragma unroll
      for (int c = 0; c < MAXB; ++c) {
        const int l = l0 + c * lstep;
        if (l < nlines) {
          T2* dst = buf + l * lstride;
#pragma unroll
          for (int r = 0; r < 8; ++r) dst[wo[r]] = v[c][r];
        }
      }
    }
    if (s < 2) wave_lds_sync<VDWXC_FFT512_WAVESYNC>();
    else if (END_SYNC || kOutLds) __syncthreads();   // the caller reads the lines with its own mapping, or reuses them
  }
}

template <int EPT, int DIR, int PS = kLdsPadShift, typename T2>
__device__ void lds_fft(T2* buf, const AxisPlan& plan, int nlines, int lstride,
                        const T2* __restrict__ tw, int tid, int nthr) {
  // (uniform over the block; readfirstlane keeps it scalar where the compiler lost track of that)
  int n = __builtin_amdgcn_readfirstlane(plan.n);
  // keep the per-stage constants of this call from being hoisted into registers that stay live
  // across a caller's loop around the transform
  asm volatile("" : "+s"(n));
  if (n == 512 && (nthr & 63) == 0) {
    // nlines * 512 <= nthr * EPT, so a thread has at most ceil(EPT / 8) lines
    lds_fft512<(EPT + 7) / 8, DIR, PS>(buf, nlines, lstride, tw, tid, nthr);
  } else if (PS < kNoPad && plan.linear) {
    lds_fft_stages<EPT, DIR, PS, true>(buf, plan, n, nlines, lstride, tw, tid, nthr);
  } else {
    lds_fft_stages<EPT, DIR, PS, false>(buf, plan, n, nlines, lstride, tw, tid, nthr);
  }
}

}  // namespace vdwxc
