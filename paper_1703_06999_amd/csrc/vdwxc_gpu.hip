// Host runtime and C ABI of the vdW-DF nonlocal-correlation library (see include/vdwxc_gpu.h).
//
// A handle holds: the grid and cell, per-axis FFT plans, references to the shared read-only tables
// (the q-mesh with the second-derivative matrix of its natural helper splines, the kernel table in
// FP64 or FP32, the twiddle tables of its axis lengths) and one block of work memory: two complex
// work buffers A and B, the dE/dsigma and gradient buffers of the potential entry, the per-point
// spline state, the per-column energy partials and a NaN flag.  A calculate call only enqueues
// kernels on the handle's stream; the synchronous entry points then copy back one small result.
#include <dlfcn.h>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/vdwxc_gpu.h"
#include "kernels.h"

using namespace vdwxc;

namespace {

#ifndef VDWXC_DIV_ZT
#define VDWXC_DIV_ZT 16
#endif
// field pairs per inverse z transform in the assembly: two in FP64 (192^3: -20 % in that pass);
// one in FP32, where the second prefetch set spills under the 128-register cap and costs
// occupancy without it
// the register-state theta pass for N3 = 512 (k_theta_zfwd512): lines per block and waves per
// SIMD its registers allow, per precision
#ifndef VDWXC_T512_TILE64
#define VDWXC_T512_TILE64 8
#endif
#ifndef VDWXC_T512_WPE64
#define VDWXC_T512_WPE64 2
#endif
#ifndef VDWXC_T512_TILE32
#define VDWXC_T512_TILE32 8
#endif
template <typename T>
constexpr int t512_wpe() { return sizeof(T) == 8 ? VDWXC_T512_WPE64 : 4; }
#ifndef VDWXC_T512_PB64
#define VDWXC_T512_PB64 2
#endif
#ifndef VDWXC_T512_PB32
#define VDWXC_T512_PB32 1
#endif
template <typename T>
constexpr int t512_pb() { return sizeof(T) == 8 ? VDWXC_T512_PB64 : VDWXC_T512_PB32; }
// the register-state assembly for N3 = 512 (k_zinv_assemble512): lines per block, field pairs per
// transform and waves per SIMD, per precision
#ifndef VDWXC_A512_TILE64
#define VDWXC_A512_TILE64 8
#endif
#ifndef VDWXC_A512_PB64
#define VDWXC_A512_PB64 1
#endif
#ifndef VDWXC_A512_WPE64
#define VDWXC_A512_WPE64 2
#endif
#ifndef VDWXC_A512_TILE32
#define VDWXC_A512_TILE32 8
#endif
template <typename T>
constexpr int a512_pb() { return sizeof(T) == 8 ? VDWXC_A512_PB64 : 1; }
#ifndef VDWXC_A512_WPE32
#define VDWXC_A512_WPE32 2
#endif
// Measured at 512^3 when it was introduced: FP64 14.3 -> 12.6 ms (8-line blocks, no prefetch;
// prefetching the next pair measured 12.9), while in FP32 the register-state version lost to the
// general kernel (7.9 ms against 11.7 with 8-line blocks at four waves per SIMD, 9.5 with 4-line
// blocks at three).  With the interval byte array, the state read after the transforms and the
// wave-synchronised stages it wins in FP32 too at two waves per SIMD with the next pair prefetched:
// 5.24 -> 5.01 ms (four waves: 6.0 ms with spills; three: 8.0 ms).
#ifndef VDWXC_A512_FP32
#define VDWXC_A512_FP32 1
#endif
template <typename T>
constexpr bool a512_used() { return sizeof(T) == 8 ? true : VDWXC_A512_FP32; }
template <typename T>
constexpr int a512_wpe() { return sizeof(T) == 8 ? VDWXC_A512_WPE64 : VDWXC_A512_WPE32; }
#ifndef VDWXC_A512_PF64
#define VDWXC_A512_PF64 1
#endif
#ifndef VDWXC_A512_PF32
#define VDWXC_A512_PF32 1
#endif
template <typename T>
constexpr bool a512_pf() { return sizeof(T) == 8 ? VDWXC_A512_PF64 : VDWXC_A512_PF32; }
#ifndef VDWXC_ASM_PB64
#define VDWXC_ASM_PB64 2
#endif
template <typename T>
constexpr int asm_pb() { return sizeof(T) == 8 ? VDWXC_ASM_PB64 : 1; }
constexpr int kEPTA = 4;         // grid points (and FFT elements) per thread in the z assembly
constexpr int kEPT = 8;          // FFT elements per thread in the z and y passes
#ifndef VDWXC_EPTC
#define VDWXC_EPTC 20
#endif
// FFT elements per thread in the contraction pass: all 20 lines of a column in one transform
constexpr int kEPTC = VDWXC_EPTC;
#ifndef VDWXC_XCAP_MIN_THREADS
#define VDWXC_XCAP_MIN_THREADS 64   // smallest contraction block that uses the register-capped kernel
#endif
#ifndef VDWXC_XPAD
#define VDWXC_XPAD kSwizzle
#endif
constexpr int kXPad = VDWXC_XPAD;  // LDS line layout of the contraction pass (no padding)
constexpr int kMaxThreadsZ = 512;  // z passes
constexpr int kMaxThreadsY = 1024; // y passes
constexpr int kMaxThreadsX = 512;  // x passes: one thread per contraction slot
constexpr int kLineTile = 16;    // lines per block in the z and y passes
// Lines per block of the y passes.  Measured at 512^3: 8-line FP64 blocks (74 KB of LDS, two per
// CU) beat 16-line ones (139 KB, one per CU) by 19 % (forward) and 28 % (inverse) while the
// 512-point transform synchronised its stages over the block; with stages synchronised within each
// wave, the 512-point forward pass takes 16 lines (8.1 -> 7.2 ms), the inverse keeps 8 (16 lines:
// 8.2 -> 8.8 ms).  In FP32 the forward pass keeps 16 lines, whose transposed writes are then whole
// 128-byte rows (8 lines: +9 %), and the inverse takes 8 (-7 %).  4-line blocks are slower in both
// precisions.
#ifndef VDWXC_YTILE64
#define VDWXC_YTILE64 8
#endif
#ifndef VDWXC_YTILE64_512
#define VDWXC_YTILE64_512 16
#endif
#ifndef VDWXC_YTILE32
#define VDWXC_YTILE32 16
#endif
#ifndef VDWXC_YTILE64_INV
#define VDWXC_YTILE64_INV 8
#endif
#ifndef VDWXC_YTILE32_INV
#define VDWXC_YTILE32_INV 8
#endif
constexpr size_t kMaxLds = 160 * 1024;

thread_local std::string g_init_error;

struct Launch {
  int tile = 1, nthr = 64, lstride = 1;
  size_t lds = 0;
  int sets = 1;   // assembly: line sets (field pairs per transform)
};

// Device buffers of one evaluation.  A handle owns one set; the allocation-free entry point
// carves one out of the static scratch array.  `timed`: record the per-stage HIP events (never on
// the allocation-free path, where taking an event could allocate).
struct Work {
  void* A = nullptr;           // complex [f][x][kz][y] (z pass output), real fields of the div/grad passes
  void* B = nullptr;           // complex [f][kz][ky][x] (y pass output)
  double* S = nullptr;         // dE/dsigma of the potential entry [N]
  void* state = nullptr;       // per-point spline state Quad<T> [N], theta pass -> assembly
  unsigned char* sb = nullptr; // the spline interval alone [N] (512-point z lines), theta -> assembly
  double* G = nullptr;         // spectral gradient [3][N]
  double* partials = nullptr;  // per-column energy partials [N2 * H3]
  double* lda = nullptr;       // per-block sums of the LDA correlation pass [kLdaBlocks]
  int* flag = nullptr;         // [0]: NaN seen by the theta pass, [1]: the last evaluation's flag
  bool timed = true;
};

// byte offsets of the buffers of Work in one block (each 256-byte aligned) and its size
struct Layout {
  size_t A, B, S, state, sb, G, partials, lda, flag, total;
};

// bytes per grid point of the spline state passed from the theta pass to the assembly
size_t state_bytes(vdwxc_precision p) { return p == VDWXC_FP64 ? sizeof(Quad<double>) : sizeof(Quad<float>); }

size_t complex_buffer_bytes(int n1, int n2, int n3, vdwxc_precision p, int M) {
  const size_t nk = size_t(n1) * n2 * (n3 / 2 + 1);
  const size_t fields = (p == VDWXC_FP64) ? std::max(M, 3) * 16 : std::max<size_t>(M * 8, 3 * 16);
  return nk * fields;
}

Layout workspace_layout(int n1, int n2, int n3, vdwxc_precision p, int M) {
  auto al = [](size_t x) { return (x + 255) & ~size_t(255); };
  const size_t N = size_t(n1) * n2 * n3, cplx = complex_buffer_bytes(n1, n2, n3, p, M);
  Layout L{};
  size_t o = 0;
  L.A = o; o += al(cplx);
  L.B = o; o += al(cplx);
  L.S = o; o += al(N * sizeof(double));
  L.state = o; o += al(N * state_bytes(p));
  L.sb = o; o += al(n3 == 512 ? N : 0);
  L.G = o; o += al(3 * N * sizeof(double));
  L.partials = o; o += al(size_t(n2) * (n3 / 2 + 1) * sizeof(double));
  L.lda = o; o += al(kLdaBlocks * sizeof(double));
  L.flag = o; o += al(2 * sizeof(int));
  L.total = o;
  return L;
}

Work carve(void* base, const Layout& L) {
  unsigned char* b = static_cast<unsigned char*>(base);
  Work w;
  w.A = b + L.A;
  w.B = b + L.B;
  w.S = reinterpret_cast<double*>(b + L.S);
  w.state = b + L.state;
  w.sb = b + L.sb;
  w.G = reinterpret_cast<double*>(b + L.G);
  w.partials = reinterpret_cast<double*>(b + L.partials);
  w.lda = reinterpret_cast<double*>(b + L.lda);
  w.flag = reinterpret_cast<int*>(b + L.flag);
  return w;
}

// ---- read-only tables shared between handles --------------------------------------------------
// Handles on one device that use the same kernel table (q-mesh, k-grid and values, compared in
// full) in the same precision share one device copy of it, together with the q-mesh and the
// spline moments; handles whose grids share an axis length share its twiddle tables.  Entries are
// reference counted and freed with their last handle.
struct TableEntry {
  int device = 0;
  vdwxc_precision precision = VDWXC_FP64;
  int nq = 0, nk = 0;
  double kmax = 0.0;
  std::vector<double> qmesh, table;   // host copies of the inputs: the key
  double* d_q = nullptr;
  double* d_mm = nullptr;
  Quad<double>* d_table64 = nullptr;  // chunk-major pair table, see build_pair_table
  Quad<float>* d_table32 = nullptr;
  int refs = 0;
};
struct TwiddleEntry {
  int device = 0, n = 0;
  double2* d64 = nullptr;   // exp(-2 pi i t / n), t < n
  float2* d32 = nullptr;
  int refs = 0;
};
std::mutex g_cache_mutex;
std::vector<TableEntry*> g_tables;
std::vector<TwiddleEntry*> g_twiddles;

}  // namespace

// ---- static work memory of the allocation-free entry point ------------------------------------
// vdwxc_calculate_potential_noalloc runs with its work buffers in this array instead of the
// handle's own.  Each device the library runs on holds one copy of it until the process ends.  In
// host code the name `scratch` is only a stand-in for the symbol, not a device address: the address
// comes from hipGetSymbolAddress, taken once per device (with that device current) by the first
// vdwxc_init* on it, and kept in g_scratch_ptr.
constexpr size_t kScratchBytes = size_t(128) << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mutex;
void* g_scratch_ptr[kMaxDevices] = {};

// record the device address of `scratch` on `device` (the current device), once
hipError_t ensure_scratch_address(int device) {
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mutex);
  if (g_scratch_ptr[device]) return hipSuccess;
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return e;
  if (!p) return hipErrorInvalidSymbol;
  g_scratch_ptr[device] = p;
  return hipSuccess;
}

void* scratch_address(int device) {
  if (device < 0 || device >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lock(g_scratch_mutex);
  return g_scratch_ptr[device];
}
}  // namespace

struct vdwxc_ctx {
  int n1 = 0, n2 = 0, n3 = 0, h3 = 0;
  double cell[9] = {0};
  double omega = 0.0;
  vdwxc_flavour flavour = VDWXC_DF1;
  vdwxc_precision precision = VDWXC_FP64;
  int M = 0, nk = 0;
  double kmax = 0.0;
  std::vector<double> qmesh;
  hipStream_t stream = nullptr;
  int device = 0;
  Geometry geo{};
  AxisPlan plan[3]{};
  Launch zl64, zl32, za64, za32, yl64, yl64i, yl32, yl32i, xl64, xl32;
  Launch dz64, dz32, dy64, dy32, dx64, dx32;   // divergence passes (lds: the whole block)
  Launch gz, gy, gx;                           // gradient passes, FP64 (lds: the whole block)
  size_t lds_theta64 = 0, lds_theta32 = 0, lds_asm64 = 0, lds_asm32 = 0;
  bool x_capped = false;   // launch the register-capped contraction kernel
  bool z512 = false;       // N3 = 512: the register-state theta pass
  Launch t512_64, t512_32; // its launch (lds: the whole block)
  Launch a512_64, a512_32; // the register-state assembly for N3 = 512
  bool ortho = false;
  // shared read-only device tables (reference counted, see TableEntry / TwiddleEntry)
  TableEntry* tab = nullptr;
  TwiddleEntry* tw[3] = {nullptr, nullptr, nullptr};
  // the handle's own work memory: one allocation of `ws_bytes`, carved by workspace_layout
  void* d_ws = nullptr;
  size_t ws_bytes = 0;
  size_t buf_bytes = 0;        // each complex work buffer
  Work work;
  double* d_energy = nullptr;  // energy of the synchronous entries
  double* h_energy = nullptr;  // pinned
  int* h_flag = nullptr;       // pinned
  std::string last_error;
  // stage timing
  bool timing = false;
  std::vector<hipEvent_t> free_events;
  struct Pending { int stage; hipEvent_t start, stop; };
  std::vector<Pending> pending;
  double stage_ms[VDWXC_NUM_STAGES] = {0};
  long long stage_count[VDWXC_NUM_STAGES] = {0};
  hipEvent_t cur_start = nullptr;
};

namespace {

vdwxc_status fail(vdwxc_ctx* h, vdwxc_status s, const std::string& msg) {
  if (h) h->last_error = msg; else g_init_error = msg;
  return s;
}

#define HIP_TRY(h, expr)                                                                      \
  do {                                                                                        \
    hipError_t e_ = (expr);                                                                   \
    if (e_ != hipSuccess)                                                                     \
      return fail((h), e_ == hipErrorOutOfMemory ? VDWXC_ENOMEM : VDWXC_EDEVICE,              \
                  std::string(#expr) + ": " + hipGetErrorString(e_));                         \
  } while (0)

bool factor_axis(int n, AxisPlan& p) {
  p.n = n;
  p.nst = 0;
  int m = n;
  // power-of-two part 2^e in ceil(e / 3) stages of 8 (then one 4 or 2), except that a 16 replaces
  // an 8 where it saves a stage (2^7 = 16 * 8 rather than 8 * 8 * 2)
  int e = 0;
  while (m % 2 == 0) { m /= 2; ++e; }
  const int n16 = e % 3 == 1 && e >= 4 ? 1 : e % 3 == 2 && e >= 8 ? 2 : 0;
  for (int i = 0; i < n16; ++i) { p.radix[p.nst++] = 16; e -= 4; }
  while (e >= 3) { p.radix[p.nst++] = 8; e -= 3; }
  if (e > 0) p.radix[p.nst++] = 1 << e;
  for (int r : {3, 5, 7}) {
    while (m % r == 0) {
      if (p.nst >= kMaxStages) return false;
      p.radix[p.nst++] = r;
      m /= r;
    }
  }
  if (m != 1) return false;
  int prod = 1;
  const int B = 1 << kLdsPadShift;
  p.linear = 1;
  for (int s = 0; s < p.nst; ++s) {
    const int R = p.radix[s], nb = n / R;
    p.mnb[s] = div_magic(unsigned(nb));
    p.mp[s] = div_magic(unsigned(prod));
    if (nb % B != 0 || (prod * R) % B != 0 || (prod % B != 0 && B % prod != 0)) p.linear = 0;
    prod *= R;
  }
  return true;
}

double det3(const double* c) {
  return c[0] * (c[4] * c[8] - c[5] * c[7]) - c[1] * (c[3] * c[8] - c[5] * c[6]) + c[2] * (c[3] * c[7] - c[4] * c[6]);
}

// b_i with a_i . b_j = 2 pi delta_ij: rows of 2 pi (A^-1)^T
void reciprocal(const double* a, double* b) {
  const double d = det3(a);
  const double inv[9] = {
      (a[4] * a[8] - a[5] * a[7]) / d, (a[2] * a[7] - a[1] * a[8]) / d, (a[1] * a[5] - a[2] * a[4]) / d,
      (a[5] * a[6] - a[3] * a[8]) / d, (a[0] * a[8] - a[2] * a[6]) / d, (a[2] * a[3] - a[0] * a[5]) / d,
      (a[3] * a[7] - a[4] * a[6]) / d, (a[1] * a[6] - a[0] * a[7]) / d, (a[0] * a[4] - a[1] * a[3]) / d};
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) b[3 * i + j] = 2.0 * M_PI * inv[3 * j + i];
}

// largest |G|^2 of the grid (Nyquist components in quadrature): a convex form on every face of
// the index box, so the extreme signed frequencies and the Nyquist index are the candidates
double max_gnorm2(const int n[3], const double* b) {
  std::vector<int> cand[3];
  for (int i = 0; i < 3; ++i) {
    const int lo = (n[i] - 1) / 2;
    cand[i] = {-lo, lo};
    if (n[i] % 2 == 0) cand[i].push_back(n[i] / 2);
  }
  double best = 0.0;
  for (int fx : cand[0])
    for (int fy : cand[1])
      for (int fz : cand[2]) {
        const int f[3] = {fx, fy, fz};
        double reg[3] = {0, 0, 0}, nyq[3] = {0, 0, 0};
        for (int i = 0; i < 3; ++i) {
          const bool isn = (n[i] % 2 == 0) && f[i] == n[i] / 2;
          for (int c = 0; c < 3; ++c) (isn ? nyq : reg)[c] += f[i] * b[3 * i + c];
        }
        const double g2 = reg[0] * reg[0] + reg[1] * reg[1] + reg[2] * reg[2] + nyq[0] * nyq[0] +
                          nyq[1] * nyq[1] + nyq[2] * nyq[2];
        best = std::max(best, g2);
      }
  return best;
}

// second derivatives mm[a][b] of the natural cubic splines through p_a(q_b) = delta_ab
void natural_spline_moments(const std::vector<double>& q, std::vector<double>& mm) {
  const int M = int(q.size());
  mm.assign(size_t(M) * M, 0.0);
  std::vector<double> h(M - 1), diag(M), rhs(M), sup(M);
  for (int i = 0; i + 1 < M; ++i) h[i] = q[i + 1] - q[i];
  for (int a = 0; a < M; ++a) {
    // interior equations i = 1..M-2: h_{i-1} m_{i-1} + 2(h_{i-1}+h_i) m_i + h_i m_{i+1} = r_i
    std::vector<double> y(M, 0.0);
    y[a] = 1.0;
    const int K = M - 2;
    if (K <= 0) continue;
    std::vector<double> cprime(K), dprime(K);
    for (int r = 0; r < K; ++r) {
      const int i = r + 1;
      const double lower = h[i - 1], diagv = 2.0 * (h[i - 1] + h[i]), upper = h[i];
      const double rr = 6.0 * ((y[i + 1] - y[i]) / h[i] - (y[i] - y[i - 1]) / h[i - 1]);
      if (r == 0) {
        cprime[r] = upper / diagv;
        dprime[r] = rr / diagv;
      } else {
        const double den = diagv - lower * cprime[r - 1];
        cprime[r] = upper / den;
        dprime[r] = (rr - lower * dprime[r - 1]) / den;
      }
    }
    std::vector<double> m(M, 0.0);
    for (int r = K - 1; r >= 0; --r) m[r + 1] = dprime[r] - (r + 1 < K ? cprime[r] * m[r + 2] : 0.0);
    for (int b = 0; b < M; ++b) mm[size_t(a) * M + b] = m[b];
  }
}

template <typename T2, typename T>
std::vector<T2> twiddles(int n) {
  std::vector<T2> tw(std::max(n, 1));
  for (int t = 0; t < n; ++t) {
    const long double ang = 2.0L * 3.141592653589793238462643383279502884L * (long double)t / (long double)n;
    tw[t].x = T(cosl(ang));
    tw[t].y = T(-sinl(ang));
  }
  return tw;
}

int round_up(int v, int m) { return (v + m - 1) / m * m; }

// block size with >= `items / ept` threads, a multiple of 64, at most `maxt`
int threads_for(long items, int ept, int maxt) {
  const long t = (items + ept - 1) / ept;
  return int(std::min<long>(maxt, std::max<long>(64, round_up(int(std::min<long>(t, 1 << 20)), 64))));
}

// TILE lines of length n in one block (TILE <= min(16, other)), padded stride n + 1; the LDS
// size includes the twiddle table of the axis
bool line_launch(int maxt, int n, int other, size_t cplx_bytes, Launch& L, int ept = kEPT, int max_tile = kLineTile) {
  int tile = std::min(max_tile, std::max(1, other));
  while (tile > 1 && long(tile) * n > long(maxt) * ept) tile /= 2;
  if (long(tile) * n > long(maxt) * ept || n > kMaxAxis) return false;
  L.tile = tile;
  L.nthr = threads_for(long(tile) * n, ept, maxt);
  L.lstride = lds_span<>(n) | 1;   // odd: the transposed tile accesses hit distinct banks
  L.lds = ((size_t(n) * cplx_bytes + 15) & ~size_t(15)) + size_t(tile) * L.lstride * cplx_bytes;
  return L.lds + 4096 <= kMaxLds;
}


template <typename T>
size_t zstate_lds(const Launch& L, int n3, int per_point_values) {
  const size_t npts = size_t(L.tile) * n3;
  return L.lds + npts * per_point_values * sizeof(T) + ((npts + 15) & ~size_t(15)) + spline_lds_bytes<T>();
}

// Occupancy-driven z tile.  A z-pass block holds TILE lines plus TILE*n3 points of per-point state,
// so its LDS and thread count scale with the tile; how many blocks then share a CU depends on that
// and on the kernel's registers.  E.g. at n3 = 192 a 16-line theta block (6 waves, ~59 KB) leaves
// two blocks (12 waves) per CU where 8-line blocks (3 waves, ~30 KB) fit five (15 waves).  The
// largest tile whose resident waves per CU come within 10% of the best tile's wins: a block's
// set-up (twiddles, spline tables) and its barriers are shared by more lines, which measured
// worth more than the last wave or two (n3 = 192: 15 waves at 8 lines beat 16 waves at 4).
// Blocks of one wave are not considered unless no larger block fits.
bool zline_config(int tile, int n3, size_t cplx_bytes, int ept, Launch& L) {
  if (long(tile) * n3 > long(kMaxThreadsZ) * ept || n3 > kMaxAxis) return false;
  L.tile = tile;
  L.nthr = threads_for(long(tile) * n3, ept, kMaxThreadsZ);
  L.lstride = lds_span<>(n3) | 1;
  L.lds = ((size_t(n3) * cplx_bytes + 15) & ~size_t(15)) + size_t(tile) * L.lstride * cplx_bytes;
  return true;
}

template <typename K>
int resident_waves(K* kernel, int nthr, size_t lds) {
  int blocks = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, reinterpret_cast<const void*>(kernel), nthr, lds) !=
      hipSuccess) {
    (void)hipGetLastError();
    return 0;
  }
  return blocks * ((nthr + 63) / 64);
}

struct Cand {
  Launch L;   // L.lds: the lines and twiddles
  size_t lds; // the block's whole dynamic LDS
};

// The rule above over candidates listed from the largest tile down.
template <typename K>
bool pick_occupancy(K* kernel, const Cand* c, int nc, Launch& out, size_t& lds_out) {
  int waves[8] = {0}, best = 0;
  for (int i = 0; i < nc; ++i) best = std::max(best, waves[i] = resident_waves(kernel, c[i].L.nthr, c[i].lds));
  for (int i = 0; i < nc; ++i)
    if (10 * waves[i] >= 9 * best) {
      out = c[i].L;
      lds_out = c[i].lds;
      return true;
    }
  return false;
}

// z passes with per-point state: `values` values of type T per point sit next to the lines
// (zstate_lds).  Tiles halve from min(kLineTile, other).
template <typename T, typename K>
bool pick_ztile(K* kernel, int n3, int other, int values, int ept, Launch& out, size_t& lds_out, int line_sets = 1) {
  Cand c[8];
  int nc = 0;
  for (int tile = std::min(kLineTile, std::max(1, other)); tile >= 1 && nc < 8; tile /= 2) {
    Launch L;
    if (!zline_config(tile, n3, 2 * sizeof(T), ept, L)) continue;
    // one-wave blocks only where nothing larger fits: their per-block set-up is not repaid
    if (nc > 0 && L.nthr < 128) break;
    const size_t lds = zstate_lds<T>(L, n3, values) + size_t(line_sets - 1) * tile * L.lstride * 2 * sizeof(T);
    if (lds > kMaxLds) continue;
    L.sets = line_sets;
    c[nc++] = Cand{L, lds};
  }
  return pick_occupancy(kernel, c, nc, out, lds_out);
}

// One-axis passes of the divergence and gradient (k_div_*, k_grad_*): `tile` lines of the axis
// (length n) per block, held as np "P lines" and nd = ceil(tile / 2) "D lines" (complex, two real
// series each) plus one complex sum per P line; np = ceil(tile / 2) when the P lines pack pairs
// (p_half), else tile.  z passes (zpass) tile y lines like the other z passes (tiles halve from
// min(kLineTile, n2) down to 1); y and x passes tile z in powers of two from min(16, n3 rounded
// up), at least 2.  The chosen launch's L.lds is the block's whole LDS.
template <typename T, typename K>
bool pick_div(K* kernel, bool zpass, bool p_half, int n, int first_tile, Launch& out) {
  const size_t cplx = 2 * sizeof(T);
  Cand c[8];
  int nc = 0;
  for (int tile = first_tile; tile >= (zpass ? 1 : 2) && nc < 8; tile /= 2) {
    const int nd = (tile + 1) / 2, np = p_half ? nd : tile;
    if (long(zpass ? tile : nd) * n > long(kMaxThreadsZ) * kEPT || n > kMaxAxis) continue;
    Launch L;
    L.tile = tile;
    L.nthr = threads_for(long(zpass ? tile : std::max(np, nd)) * n, kEPT, kMaxThreadsZ);
    if (nc > 0 && L.nthr < 128) break;
    L.lstride = lds_span<>(n) | 1;
    L.lds = tw_lds_bytes<typename Cx<T>::type>(n) + size_t(np + nd) * L.lstride * cplx + size_t(np) * cplx;
    if (L.lds > kMaxLds) continue;
    c[nc++] = Cand{L, L.lds};
  }
  size_t lds = 0;
  return pick_occupancy(kernel, c, nc, out, lds);
}

template <typename F>
void set_lds_limit(F* kernel, size_t bytes) {
  (void)hipFuncSetAttribute(reinterpret_cast<const void*>(kernel), hipFuncAttributeMaxDynamicSharedMemorySize,
                            int(bytes));
}

vdwxc_status validate_common(const int grid[3], const double cell[9]) {
  if (!grid || !cell) return fail(nullptr, VDWXC_EINVAL, "grid and cell must not be NULL");
  for (int i = 0; i < 3; ++i)
    if (grid[i] < 1) return fail(nullptr, VDWXC_EINVAL, "grid sizes must be >= 1");
  for (int i = 0; i < 9; ++i)
    if (!std::isfinite(cell[i])) return fail(nullptr, VDWXC_EINVAL, "cell contains NaN/inf");
  if (!(det3(cell) > 0.0)) return fail(nullptr, VDWXC_EINVAL, "cell must have positive volume (right-handed)");
  return VDWXC_OK;
}

template <typename T>
hipError_t upload(T** dst, const T* src, size_t count) {
  hipError_t e = hipMalloc(reinterpret_cast<void**>(dst), count * sizeof(T));
  if (e != hipSuccess) return e;
  return hipMemcpy(*dst, src, count * sizeof(T), hipMemcpyHostToDevice);
}

void free_table(TableEntry* t) {
  auto f = [](void* p) { if (p) (void)hipFree(p); };
  f(t->d_q); f(t->d_mm); f(t->d_table64); f(t->d_table32);
  delete t;
}

void free_twiddles(TwiddleEntry* t) {
  if (t->d64) (void)hipFree(t->d64);
  if (t->d32) (void)hipFree(t->d32);
  delete t;
}

// drop one reference (device `dev` current); the entry is freed with its last handle
void release_table(TableEntry* t) {
  if (!t) return;
  std::lock_guard<std::mutex> lock(g_cache_mutex);
  if (--t->refs > 0) return;
  g_tables.erase(std::remove(g_tables.begin(), g_tables.end(), t), g_tables.end());
  free_table(t);
}

void release_twiddles(TwiddleEntry* t) {
  if (!t) return;
  std::lock_guard<std::mutex> lock(g_cache_mutex);
  if (--t->refs > 0) return;
  g_twiddles.erase(std::remove(g_twiddles.begin(), g_twiddles.end(), t), g_twiddles.end());
  free_twiddles(t);
}

void release(vdwxc_ctx* h) {
  if (!h) return;
  for (auto& p : h->pending) { (void)hipEventDestroy(p.start); (void)hipEventDestroy(p.stop); }
  for (auto e : h->free_events) (void)hipEventDestroy(e);
  release_table(h->tab);
  for (int i = 0; i < 3; ++i) release_twiddles(h->tw[i]);
  if (h->d_ws) (void)hipFree(h->d_ws);
  if (h->d_energy) (void)hipFree(h->d_energy);
  if (h->h_energy) (void)hipHostFree(h->h_energy);
  if (h->h_flag) (void)hipHostFree(h->h_flag);
  delete h;
}

// load chunk (groups of two pairs) of the contraction kernel in precision p
int table_chunk(vdwxc_precision p) { return p == VDWXC_FP64 ? x_chunk<double>() : x_chunk<float>(); }

// Device bytes of the contraction's pair table: per group of two unordered pairs and node j one
// Quad (T_j and T_j+1 - T_j of each pair), padded to whole chunks of the precision's chunk.
size_t pair_table_bytes(vdwxc_precision p, int nk) {
  const int ch = table_chunk(p), chunks = (kNumPairs / 2 + ch - 1) / ch;
  return size_t(chunks) * ch * size_t(nk) * (p == VDWXC_FP64 ? sizeof(Quad<double>) : sizeof(Quad<float>));
}

// The kernel table reordered for the contraction: per unordered pair p = (a <= b) (pair_index
// order, so the pairs of a q-mesh of M points are the first M(M+1)/2) and node j, T_j and
// T_j+1 - T_j (0 at the last node).  Pairs 2g and 2g+1 share entry (g, j) = (T_j(2g), D_j(2g),
// T_j(2g+1), D_j(2g+1)), stored chunk-major at [g / ch][j][g % ch] (the contraction reads
// a chunk's entries of one node together; the two lanes of a kx, -kx pair read one half each).
// Pairs with a or b >= nq stay zero.
std::vector<Quad<double>> build_pair_table(int nq, int nk, const double* table, int ch) {
  const int chunks = (kNumPairs / 2 + ch - 1) / ch;
  const size_t tn = size_t(chunks) * ch * nk;
  std::vector<Quad<double>> t64(tn, Quad<double>{0.0, 0.0, 0.0, 0.0});
  for (int a = 0; a < nq; ++a)
    for (int b = a; b < nq; ++b) {
      const int pr = kPairs.pos[a][b];
      for (int j = 0; j < nk; ++j) {
        const double tj = table[(size_t(j) * nq + a) * nq + b];
        const double dj = j + 1 < nk ? table[(size_t(j + 1) * nq + a) * nq + b] - tj : 0.0;
        const int grp = pr / 2;
        Quad<double>& q = t64[(size_t(grp / ch) * nk + j) * ch + grp % ch];
        if (pr % 2 == 0) {
          q.x = tj;
          q.y = dj;
        } else {
          q.z = tj;
          q.w = dj;
        }
      }
    }
  return t64;
}

// the shared device copy of a kernel table for `device` (current) and precision, created on first
// use; the caller holds one reference
hipError_t acquire_table(int device, vdwxc_precision precision, int nq, const double* qmesh, int nk, double kmax,
                         const double* table, TableEntry** out) {
  std::lock_guard<std::mutex> lock(g_cache_mutex);
  const size_t tsz = size_t(nk) * nq * nq;
  for (TableEntry* t : g_tables) {
    if (t->device == device && t->precision == precision && t->nq == nq && t->nk == nk && t->kmax == kmax &&
        std::memcmp(t->qmesh.data(), qmesh, nq * sizeof(double)) == 0 &&
        std::memcmp(t->table.data(), table, tsz * sizeof(double)) == 0) {
      ++t->refs;
      *out = t;
      return hipSuccess;
    }
  }
  TableEntry* t = new (std::nothrow) TableEntry();
  if (!t) return hipErrorOutOfMemory;
  t->device = device;
  t->precision = precision;
  t->nq = nq;
  t->nk = nk;
  t->kmax = kmax;
  t->qmesh.assign(qmesh, qmesh + nq);
  t->table.assign(table, table + tsz);
  std::vector<double> mm;
  natural_spline_moments(t->qmesh, mm);
  hipError_t e = upload(&t->d_q, qmesh, nq);
  if (e == hipSuccess) e = upload(&t->d_mm, mm.data(), mm.size());
  if (e == hipSuccess) {
    const std::vector<Quad<double>> t64 = build_pair_table(nq, nk, table, table_chunk(precision));
    if (precision == VDWXC_FP64) {
      e = upload(&t->d_table64, t64.data(), t64.size());
    } else {
      std::vector<Quad<float>> t32(t64.size());
      for (size_t i = 0; i < t64.size(); ++i)
        t32[i] = Quad<float>{float(t64[i].x), float(t64[i].y), float(t64[i].z), float(t64[i].w)};
      e = upload(&t->d_table32, t32.data(), t32.size());
    }
  }
  if (e != hipSuccess) {
    free_table(t);
    return e;
  }
  t->refs = 1;
  g_tables.push_back(t);
  *out = t;
  return hipSuccess;
}

// the shared twiddle tables (both precisions) of an axis of length n on `device` (current)
hipError_t acquire_twiddles(int device, int n, TwiddleEntry** out) {
  std::lock_guard<std::mutex> lock(g_cache_mutex);
  for (TwiddleEntry* t : g_twiddles)
    if (t->device == device && t->n == n) {
      ++t->refs;
      *out = t;
      return hipSuccess;
    }
  TwiddleEntry* t = new (std::nothrow) TwiddleEntry();
  if (!t) return hipErrorOutOfMemory;
  t->device = device;
  t->n = n;
  const auto t64 = twiddles<double2, double>(n);
  const auto t32 = twiddles<float2, float>(n);
  hipError_t e = upload(&t->d64, t64.data(), t64.size());
  if (e == hipSuccess) e = upload(&t->d32, t32.data(), t32.size());
  if (e != hipSuccess) {
    free_twiddles(t);
    return e;
  }
  t->refs = 1;
  g_twiddles.push_back(t);
  *out = t;
  return hipSuccess;
}

// NULL kernel-table path: $VDWXC_KERNEL_TABLE, else vdw_kernel_table.vdwk next to this library
std::string default_table_path() {
  if (const char* e = std::getenv("VDWXC_KERNEL_TABLE"))
    if (*e) return std::string(e);
  Dl_info info;
  if (dladdr(reinterpret_cast<void*>(&default_table_path), &info) && info.dli_fname) {
    const std::string p(info.dli_fname);
    const size_t k = p.rfind('/');
    return (k == std::string::npos ? std::string(".") : p.substr(0, k)) + "/vdw_kernel_table.vdwk";
  }
  return "vdw_kernel_table.vdwk";
}


}  // namespace

// ---------------------------------------------------------------------------------------------
// launches
// ---------------------------------------------------------------------------------------------
namespace {

template <typename T>
struct Prec;
template <> struct Prec<double> {
  static const Launch& z(const vdwxc_ctx* h) { return h->zl64; }
  static const Launch& za(const vdwxc_ctx* h) { return h->za64; }
  static const Launch& z512(const vdwxc_ctx* h) { return h->t512_64; }
  static const Launch& a512(const vdwxc_ctx* h) { return h->a512_64; }
  static const Launch& y(const vdwxc_ctx* h, int dir) { return dir < 0 ? h->yl64 : h->yl64i; }
  static const Launch& x(const vdwxc_ctx* h) { return h->xl64; }
  static const Launch& div(const vdwxc_ctx* h, int a) { return a == 2 ? h->dz64 : a == 1 ? h->dy64 : h->dx64; }
  static const double2* tw(const vdwxc_ctx* h, int a) { return h->tw[a]->d64; }
  static const Quad<double>* table(const vdwxc_ctx* h) { return h->tab->d_table64; }
  static size_t theta_lds(const vdwxc_ctx* h) { return h->lds_theta64; }
  static size_t asm_lds(const vdwxc_ctx* h) { return h->lds_asm64; }
};
template <> struct Prec<float> {
  static const Launch& z(const vdwxc_ctx* h) { return h->zl32; }
  static const Launch& za(const vdwxc_ctx* h) { return h->za32; }
  static const Launch& z512(const vdwxc_ctx* h) { return h->t512_32; }
  static const Launch& a512(const vdwxc_ctx* h) { return h->a512_32; }
  static const Launch& y(const vdwxc_ctx* h, int dir) { return dir < 0 ? h->yl32 : h->yl32i; }
  static const Launch& x(const vdwxc_ctx* h) { return h->xl32; }
  static const Launch& div(const vdwxc_ctx* h, int a) { return a == 2 ? h->dz32 : a == 1 ? h->dy32 : h->dx32; }
  static const float2* tw(const vdwxc_ctx* h, int a) { return h->tw[a]->d32; }
  static const Quad<float>* table(const vdwxc_ctx* h) { return h->tab->d_table32; }
  static size_t theta_lds(const vdwxc_ctx* h) { return h->lds_theta32; }
  static size_t asm_lds(const vdwxc_ctx* h) { return h->lds_asm32; }
};

hipEvent_t take_event(vdwxc_ctx* h) {
  if (!h->free_events.empty()) {
    hipEvent_t e = h->free_events.back();
    h->free_events.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

void stage_begin(vdwxc_ctx* h, const Work& w) {
  if (!h->timing || !w.timed) return;
  h->cur_start = take_event(h);
  if (h->cur_start) (void)hipEventRecord(h->cur_start, h->stream);
}

void stage_end(vdwxc_ctx* h, const Work& w, int stage) {
  if (!h->timing || !w.timed || !h->cur_start) return;
  hipEvent_t stop = take_event(h);
  if (!stop) return;
  (void)hipEventRecord(stop, h->stream);
  h->pending.push_back({stage, h->cur_start, stop});
  h->cur_start = nullptr;
}

template <typename T>
void enqueue_ypass(vdwxc_ctx* h, const Work& w, int nf, int dir, int stage) {
  using T2 = typename Cx<T>::type;
  const Launch& L = Prec<T>::y(h, dir);
  dim3 grid((h->n1 + L.tile - 1) / L.tile, h->h3, nf);
  T2* A = static_cast<T2*>(w.A);
  T2* B = static_cast<T2*>(w.B);
  stage_begin(h, w);
  if (dir < 0)
    hipLaunchKernelGGL((k_ypass<T, kEPT, -1>), grid, dim3(L.nthr), L.lds, h->stream, A, B, Prec<T>::tw(h, 1),
                       h->geo, h->plan[1], L.tile, L.lstride);
  else
    hipLaunchKernelGGL((k_ypass<T, kEPT, +1>), grid, dim3(L.nthr), L.lds, h->stream, B, A, Prec<T>::tw(h, 1),
                       h->geo, h->plan[1], L.tile, L.lstride);
  stage_end(h, w, stage);
}

// spectral gradient of the FP64 density n into out ([3][N], FP64), one axis at a time
// (k_grad_z, k_grad_y, k_grad_x); the intermediate real fields sit in the work buffers ([2][N] in
// A, [3][N] in B), in FP64 whatever the handle's precision, because the gradient feeds q0
void enqueue_gradient(vdwxc_ctx* h, const Work& w, const double* src, double* out) {
  double* F2 = static_cast<double*>(w.A);
  double* F3 = static_cast<double*>(w.B);
  stage_begin(h, w);
  hipLaunchKernelGGL((k_grad_z<double, kEPT>), dim3((h->n2 + h->gz.tile - 1) / h->gz.tile, h->n1), dim3(h->gz.nthr),
                     h->gz.lds, h->stream, src, F2, h->tw[2]->d64, h->geo, h->plan[2], h->gz.tile, h->gz.lstride);
  stage_end(h, w, VDWXC_STAGE_GRAD_Z);
  stage_begin(h, w);
  hipLaunchKernelGGL((k_grad_y<double, kEPT>), dim3((h->n3 + h->gy.tile - 1) / h->gy.tile, h->n1), dim3(h->gy.nthr),
                     h->gy.lds, h->stream, F2, F3, h->tw[1]->d64, h->geo, h->plan[1], h->gy.tile, h->gy.lstride);
  stage_end(h, w, VDWXC_STAGE_GRAD_Y);
  stage_begin(h, w);
  hipLaunchKernelGGL((k_grad_x<double, kEPT>), dim3((h->n3 + h->gx.tile - 1) / h->gx.tile, h->n2), dim3(h->gx.nthr),
                     h->gx.lds, h->stream, F3, out, h->tw[0]->d64, h->geo, h->plan[0], h->gx.tile, h->gx.lstride);
  stage_end(h, w, VDWXC_STAGE_GRAD_X);
}

// v -= spectral divergence of 2 S grad n, one axis at a time (k_div_z, k_div_y, k_div_x); the
// intermediate real fields sit in the work buffers ([3][N] in A, [2][N] in B)
template <typename T>
void enqueue_divergence(vdwxc_ctx* h, const Work& w, const double* S, const double* grad, double* v) {
  const Launch& Lz = Prec<T>::div(h, 2);
  const Launch& Ly = Prec<T>::div(h, 1);
  const Launch& Lx = Prec<T>::div(h, 0);
  T* F3 = static_cast<T*>(w.A);
  T* F2 = static_cast<T*>(w.B);
  stage_begin(h, w);
  hipLaunchKernelGGL((k_div_z<T, kEPT>), dim3((h->n2 + Lz.tile - 1) / Lz.tile, h->n1), dim3(Lz.nthr), Lz.lds,
                     h->stream, S, grad, F3, Prec<T>::tw(h, 2), h->geo, h->plan[2], Lz.tile, Lz.lstride);
  stage_end(h, w, VDWXC_STAGE_DIV_Z);
  stage_begin(h, w);
  hipLaunchKernelGGL((k_div_y<T, kEPT>), dim3((h->n3 + Ly.tile - 1) / Ly.tile, h->n1), dim3(Ly.nthr), Ly.lds,
                     h->stream, F3, F2, Prec<T>::tw(h, 1), h->geo, h->plan[1], Ly.tile, Ly.lstride);
  stage_end(h, w, VDWXC_STAGE_DIV_Y);
  stage_begin(h, w);
  hipLaunchKernelGGL((k_div_x<T, kEPT>), dim3((h->n3 + Lx.tile - 1) / Lx.tile, h->n2), dim3(Lx.nthr), Lx.lds,
                     h->stream, F2, v, Prec<T>::tw(h, 0), h->geo, h->plan[0], Lx.tile, Lx.lstride);
  stage_end(h, w, VDWXC_STAGE_DIV_X);
}

// the contraction pass for q-mesh bucket MB (FP32: the register-capped kernel where chosen)
template <typename T, int MB>
void launch_xcontract(vdwxc_ctx* h, const Work& w, typename Cx<T>::type* B) {
  const Launch& Lx = Prec<T>::x(h);
  if constexpr (sizeof(T) == 4) {
    if (h->x_capped) {
      hipLaunchKernelGGL((k_xcontract<T, kEPTC, kXPad, 4, MB>), dim3(h->n2, h->h3), dim3(Lx.nthr), Lx.lds, h->stream,
                         B, Prec<T>::table(h), w.partials, Prec<T>::tw(h, 0), h->geo, h->plan[0]);
      return;
    }
  }
  hipLaunchKernelGGL((k_xcontract<T, kEPTC, kXPad, 1, MB>), dim3(h->n2, h->h3), dim3(Lx.nthr), Lx.lds, h->stream, B,
                     Prec<T>::table(h), w.partials, Prec<T>::tw(h, 0), h->geo, h->plan[0]);
}

template <typename T, int MB>
void set_xcontract_lds(size_t lds) {
  set_lds_limit(k_xcontract<T, kEPTC, kXPad, 1, MB>, lds);
  if constexpr (sizeof(T) == 4) set_lds_limit(k_xcontract<T, kEPTC, kXPad, 4, MB>, lds);
}

// the five steps: theta + z FFT, y FFT, x FFT + contraction + inverse x, inverse y, inverse z +
// derivatives; then the energy sum
template <typename T>
void enqueue_main(vdwxc_ctx* h, const Work& w, const double* n, const double* sig, bool sig_from_grad, double* dedn,
                  double* dedsig, double* energy) {
  using T2 = typename Cx<T>::type;
  const Launch& Lz = Prec<T>::z(h);
  const Launch& Lx = Prec<T>::x(h);
  T2* A = static_cast<T2*>(w.A);
  T2* B = static_cast<T2*>(w.B);
  const TableEntry& tb = *h->tab;
  dim3 zgrid((h->n2 + Lz.tile - 1) / Lz.tile, h->n1);
  stage_begin(h, w);
  const size_t lds_theta = Prec<T>::theta_lds(h), lds_asm = Prec<T>::asm_lds(h);
  Quad<T>* state = static_cast<Quad<T>*>(w.state);
  if (h->z512) {
    // N3 = 512: the register-state theta pass (k_theta_zfwd512), 64 threads per line
    const Launch& L5 = Prec<T>::z512(h);
    const dim3 g5((h->n2 + L5.tile - 1) / L5.tile, h->n1);
    if (sig_from_grad)
      hipLaunchKernelGGL((k_theta_zfwd512<T, true, t512_wpe<T>(), t512_pb<T>()>), g5, dim3(L5.nthr), L5.lds, h->stream, n, sig, A, state, w.sb, w.flag,
                         tb.d_q, tb.d_mm, Prec<T>::tw(h, 2), h->geo, L5.tile, L5.lstride);
    else
      hipLaunchKernelGGL((k_theta_zfwd512<T, false, t512_wpe<T>(), t512_pb<T>()>), g5, dim3(L5.nthr), L5.lds, h->stream, n, sig, A, state, w.sb, w.flag,
                         tb.d_q, tb.d_mm, Prec<T>::tw(h, 2), h->geo, L5.tile, L5.lstride);
  } else if (sig_from_grad) {
    hipLaunchKernelGGL((k_theta_zfwd<T, kEPT, true>), zgrid, dim3(Lz.nthr), lds_theta, h->stream, n, sig, A, state,
                       w.flag, tb.d_q, tb.d_mm, Prec<T>::tw(h, 2), h->geo, h->plan[2], Lz.tile, Lz.lstride);
  } else {
    hipLaunchKernelGGL((k_theta_zfwd<T, kEPT, false>), zgrid, dim3(Lz.nthr), lds_theta, h->stream, n, sig, A, state,
                       w.flag, tb.d_q, tb.d_mm, Prec<T>::tw(h, 2), h->geo, h->plan[2], Lz.tile, Lz.lstride);
  }
  stage_end(h, w, VDWXC_STAGE_THETA_ZFWD);
  enqueue_ypass<T>(h, w, h->M, -1, VDWXC_STAGE_Y_FWD);
  stage_begin(h, w);
  switch (q_bucket(h->M)) {
    case 8: launch_xcontract<T, 8>(h, w, B); break;
    case 10: launch_xcontract<T, 10>(h, w, B); break;
    case 12: launch_xcontract<T, 12>(h, w, B); break;
    case 16: launch_xcontract<T, 16>(h, w, B); break;
    default: launch_xcontract<T, 20>(h, w, B); break;
  }
  stage_end(h, w, VDWXC_STAGE_X_CONTRACT);
  enqueue_ypass<T>(h, w, h->M, +1, VDWXC_STAGE_Y_INV);
  stage_begin(h, w);
  const Launch& La = Prec<T>::za(h);
  const dim3 agrid((h->n2 + La.tile - 1) / La.tile, h->n1);
  const double N = double(h->n1) * h->n2 * h->n3;
  if (h->z512 && a512_used<T>()) {
    // N3 = 512: the register-state assembly (k_zinv_assemble512), 64 threads per line
    const Launch& L5 = Prec<T>::a512(h);
    const dim3 g5((h->n2 + L5.tile - 1) / L5.tile, h->n1);
    hipLaunchKernelGGL((k_zinv_assemble512<T, a512_pb<T>(), a512_wpe<T>(), a512_pf<T>()>), g5, dim3(L5.nthr), L5.lds, h->stream, A,
                       state, w.sb, dedn, dedsig, tb.d_q, tb.d_mm, Prec<T>::tw(h, 2), h->geo, L5.tile, L5.lstride, w.partials,
                       h->n2 * h->h3, h->omega / (2.0 * N * N), w.flag, energy);
  } else {
    hipLaunchKernelGGL((k_zinv_assemble<T, kEPTA, kEPTA, asm_pb<T>()>), agrid, dim3(La.nthr), lds_asm, h->stream, A, state,
                       dedn, dedsig, tb.d_q, tb.d_mm, Prec<T>::tw(h, 2), h->geo, h->plan[2], La.tile, La.lstride,
                       w.partials, h->n2 * h->h3, h->omega / (2.0 * N * N), w.flag, energy, La.sets);
  }
  stage_end(h, w, VDWXC_STAGE_Z_ASSEMBLE);
}

vdwxc_status check_handle(vdwxc_ctx* h) {
  if (!h) return VDWXC_ESTATE;
  return VDWXC_OK;
}

// the handle and work memory for a call that runs in the handle's own (or attached) work memory
vdwxc_status check_work(vdwxc_ctx* h) {
  if (!h) return VDWXC_ESTATE;
  if (!h->work.A) return fail(h, VDWXC_ESTATE, "handle has no work memory (created without it; see vdwxc_set_workspace)");
  return VDWXC_OK;
}

vdwxc_status finish_launch(vdwxc_ctx* h) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(h, VDWXC_EDEVICE, std::string("kernel launch: ") + hipGetErrorString(e));
  return VDWXC_OK;
}

vdwxc_status run_partials(vdwxc_ctx* h, const Work& w, const double* n, const double* sigma, double* dedn,
                          double* dedsig, double* energy_dev) {
  HIP_TRY(h, hipSetDevice(h->device));
  if (h->precision == VDWXC_FP64)
    enqueue_main<double>(h, w, n, sigma, false, dedn, dedsig, energy_dev);
  else
    enqueue_main<float>(h, w, n, sigma, false, dedn, dedsig, energy_dev);
  return finish_launch(h);
}

vdwxc_status run_potential(vdwxc_ctx* h, const Work& w, const double* n, const double* grad, double* v,
                           double* energy_dev) {
  HIP_TRY(h, hipSetDevice(h->device));
  const double* g = grad;
  if (!g) {
    // the gradient feeds q0, so it is taken in FP64 in both precisions
    enqueue_gradient(h, w, n, w.G);
    g = w.G;
  }
  if (h->precision == VDWXC_FP64) {
    enqueue_main<double>(h, w, n, g, true, v, w.S, energy_dev);
    enqueue_divergence<double>(h, w, w.S, g, v);
  } else {
    enqueue_main<float>(h, w, n, g, true, v, w.S, energy_dev);
    enqueue_divergence<float>(h, w, w.S, g, v);
  }
  return finish_launch(h);
}

vdwxc_status run_lda(vdwxc_ctx* h, const Work& w, const double* n, double* v, double* energy_dev) {
  HIP_TRY(h, hipSetDevice(h->device));
  const long long N = (long long)h->n1 * h->n2 * h->n3;
  const long long per_block = (long long)kLdaThreads * kLdaUnroll;
  const int blocks = int(std::min<long long>(kLdaBlocks, (N + per_block - 1) / per_block));
  stage_begin(h, w);
  hipLaunchKernelGGL(k_lda_pw92, dim3(blocks), dim3(kLdaThreads), 0, h->stream, n, v, w.lda, N);
  hipLaunchKernelGGL(k_lda_energy, dim3(1), dim3(kLdaThreads), 0, h->stream, w.lda, blocks, h->omega / double(N),
                     energy_dev);
  stage_end(h, w, VDWXC_STAGE_LDA);
  return finish_launch(h);
}

// Spin-polarised evaluation: (n, sigma_eff) into the dedn_dn / dedsigma_dd outputs, the spin-paired
// partials pipeline from there into dedn_up / dedsigma_uu, then the conversion to the four spin
// partials in place (k_spin_in, k_spin_out).
vdwxc_status run_spin(vdwxc_ctx* h, const Work& w, const double* nu, const double* nd, const double* su,
                      const double* sd, double* dnu, double* dnd, double* dsu, double* dsd, double* energy_dev) {
  HIP_TRY(h, hipSetDevice(h->device));
  const long long N = (long long)h->n1 * h->n2 * h->n3;
  const int blocks = int(std::min<long long>(kSpinBlocks, (N + kSpinThreads - 1) / kSpinThreads));
  stage_begin(h, w);
  hipLaunchKernelGGL(k_spin_in<false>, dim3(blocks), dim3(kSpinThreads), 0, h->stream, nu, nd, su, sd, dnd, dsd,
                     nullptr, nullptr, h->geo.zab, N);
  stage_end(h, w, VDWXC_STAGE_SPIN);
  if (vdwxc_status st = run_partials(h, w, dnd, dsd, dnu, dsu, energy_dev); st != VDWXC_OK) return st;
  stage_begin(h, w);
  hipLaunchKernelGGL(k_spin_out<false>, dim3(blocks), dim3(kSpinThreads), 0, h->stream, nu, nd, su, sd, dnu, dnd,
                     dsu, dsd, h->geo.zab, N);
  stage_end(h, w, VDWXC_STAGE_SPIN);
  return finish_launch(h);
}

// Spin-polarised potentials: as run_spin with sigma_ss taken from the gradients, (n, sigma_eff) in
// v_dn and the work memory's gradient buffer G (sigma_uu, sigma_dd beside sigma_eff in G's other
// two thirds), the pipeline's partials in v_up and S, the spin partials converted in place
// (dE/dsigma_uu in S, dE/dsigma_dd in G), then one spectral divergence per spin:
// v_s = dE/dn_s - div(2 dE/dsigma_ss grad n_s).
template <typename T>
void enqueue_spin_potential(vdwxc_ctx* h, const Work& w, const double* nu, const double* nd, const double* gu,
                            const double* gd, double* vu, double* vd, double* energy_dev, int blocks) {
  const long long N = (long long)h->n1 * h->n2 * h->n3;
  stage_begin(h, w);
  double* suu = w.G + N;
  double* sdd = w.G + 2 * N;
  hipLaunchKernelGGL(k_spin_in<true>, dim3(blocks), dim3(kSpinThreads), 0, h->stream, nu, nd, gu, gd, vd, w.G, suu,
                     sdd, h->geo.zab, N);
  stage_end(h, w, VDWXC_STAGE_SPIN);
  enqueue_main<T>(h, w, vd, w.G, false, vu, w.S, energy_dev);
  stage_begin(h, w);
  hipLaunchKernelGGL(k_spin_out<false>, dim3(blocks), dim3(kSpinThreads), 0, h->stream, nu, nd, suu, sdd, vu, vd,
                     w.S, w.G, h->geo.zab, N);
  stage_end(h, w, VDWXC_STAGE_SPIN);
  enqueue_divergence<T>(h, w, w.S, gu, vu);
  enqueue_divergence<T>(h, w, w.G, gd, vd);
}

vdwxc_status run_spin_potential(vdwxc_ctx* h, const Work& w, const double* nu, const double* nd, const double* gu,
                                const double* gd, double* vu, double* vd, double* energy_dev) {
  HIP_TRY(h, hipSetDevice(h->device));
  const long long N = (long long)h->n1 * h->n2 * h->n3;
  const int blocks = int(std::min<long long>(kSpinBlocks, (N + kSpinThreads - 1) / kSpinThreads));
  if (h->precision == VDWXC_FP64)
    enqueue_spin_potential<double>(h, w, nu, nd, gu, gd, vu, vd, energy_dev, blocks);
  else
    enqueue_spin_potential<float>(h, w, nu, nd, gu, gd, vu, vd, energy_dev, blocks);
  return finish_launch(h);
}

// the arrays of a spin potential call: none NULL; v_up, v_dn overlapping neither each other nor the
// densities (N doubles) and gradients (3N)
vdwxc_status check_spin_potential_arrays(vdwxc_ctx* h, const double* nu, const double* nd, const double* gu,
                                         const double* gd, double* vu, double* vd) {
  const size_t N = size_t(h->n1) * h->n2 * h->n3;
  if (!nu || !nd || !vu || !vd) return fail(h, VDWXC_EINVAL, "array arguments must not be NULL");
  if (!gu || !gd) return fail(h, VDWXC_EINVAL, "the spin potential needs the gradients of n_up and n_dn");
  auto overlap = [](const double* a, size_t na, const double* b, size_t nb) { return a < b + nb && b < a + na; };
  for (double* v : {vu, vd}) {
    if (overlap(v, N, nu, N) || overlap(v, N, nd, N) || overlap(v, N, gu, 3 * N) || overlap(v, N, gd, 3 * N))
      return fail(h, VDWXC_EINVAL, "spin outputs must not overlap the inputs");
  }
  if (overlap(vu, N, vd, N)) return fail(h, VDWXC_EINVAL, "spin outputs must not overlap each other");
  return VDWXC_OK;
}

// the eight arrays of a spin call: none NULL, the outputs overlapping neither each other nor the
// inputs (N doubles each)
vdwxc_status check_spin_arrays(vdwxc_ctx* h, const double* const in[4], double* const out[4]) {
  const size_t N = size_t(h->n1) * h->n2 * h->n3;
  for (int i = 0; i < 4; ++i)
    if (!in[i] || !out[i]) return fail(h, VDWXC_EINVAL, "array arguments must not be NULL");
  auto overlap = [&](const double* a, const double* b) { return a < b + N && b < a + N; };
  for (int i = 0; i < 4; ++i) {
    for (int j = 0; j < 4; ++j)
      if (overlap(out[i], in[j])) return fail(h, VDWXC_EINVAL, "spin outputs must not overlap the inputs");
    for (int j = i + 1; j < 4; ++j)
      if (overlap(out[i], out[j])) return fail(h, VDWXC_EINVAL, "spin outputs must not overlap each other");
  }
  return VDWXC_OK;
}

vdwxc_status read_energy(vdwxc_ctx* h, double* energy_host) {
  HIP_TRY(h, hipMemcpyAsync(h->h_energy, h->d_energy, sizeof(double), hipMemcpyDeviceToHost, h->stream));
  HIP_TRY(h, hipMemcpyAsync(h->h_flag, h->work.flag + 1, sizeof(int), hipMemcpyDeviceToHost, h->stream));
  HIP_TRY(h, hipStreamSynchronize(h->stream));
  if (*h->h_flag) return fail(h, VDWXC_EINVAL, "density or gradient input contains NaN");
  *energy_host = *h->h_energy;
  return VDWXC_OK;
}

}  // namespace

// ---------------------------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------------------------
extern "C" {

const char* vdwxc_version(void) { return "vdwxc-gpu 0.1 (gfx950)"; }

const char* vdwxc_strerror(vdwxc_status s) {
  switch (s) {
    case VDWXC_OK: return "success";
    case VDWXC_EINVAL: return "invalid argument";
    case VDWXC_ENOMEM: return "out of memory";
    case VDWXC_EDEVICE: return "HIP device error";
    case VDWXC_ETABLE: return "malformed kernel table";
    case VDWXC_ESTATE: return "invalid or finalized handle";
  }
  return "unknown status";
}

const char* vdwxc_last_error(vdwxc_handle h) { return h ? h->last_error.c_str() : g_init_error.c_str(); }

size_t vdwxc_workspace_bytes_m(const int grid[3], vdwxc_precision precision, int nq) {
  if (!grid || grid[0] < 1 || grid[1] < 1 || grid[2] < 1 || nq < 1) return 0;
  if (precision != VDWXC_FP64 && precision != VDWXC_FP32_MIXED) return 0;
  return workspace_layout(grid[0], grid[1], grid[2], precision, nq).total;
}

size_t vdwxc_workspace_bytes(const int grid[3], vdwxc_precision precision) {
  return vdwxc_workspace_bytes_m(grid, precision, kMaxQ);
}

vdwxc_status vdwxc_init_table(vdwxc_handle* out, const int grid[3], const double cell[9], vdwxc_flavour flavour,
                              vdwxc_precision precision, int nq, const double* qmesh, int nk, double kmax,
                              const double* table, void* hip_stream) {
  return vdwxc_init_table_ex(out, grid, cell, flavour, precision, nq, qmesh, nk, kmax, table, hip_stream, 0u);
}

vdwxc_status vdwxc_init_table_ex(vdwxc_handle* out, const int grid[3], const double cell[9], vdwxc_flavour flavour,
                                 vdwxc_precision precision, int nq, const double* qmesh, int nk, double kmax,
                                 const double* table, void* hip_stream, unsigned flags) {
  if (!out) return fail(nullptr, VDWXC_EINVAL, "out must not be NULL");
  if (flags & ~unsigned(VDWXC_INIT_NO_WORKSPACE)) return fail(nullptr, VDWXC_EINVAL, "unknown init flags");
  *out = nullptr;
  vdwxc_status st = validate_common(grid, cell);
  if (st != VDWXC_OK) return st;
  if (flavour != VDWXC_DF1 && flavour != VDWXC_DF2) return fail(nullptr, VDWXC_EINVAL, "unknown flavour");
  if (precision != VDWXC_FP64 && precision != VDWXC_FP32_MIXED)
    return fail(nullptr, VDWXC_EINVAL, "unknown precision");
  if (!qmesh || !table) return fail(nullptr, VDWXC_ETABLE, "kernel table arrays must not be NULL");
  if (nq < 4 || nq > kMaxQ) return fail(nullptr, VDWXC_ETABLE, "q-mesh size must be in [4, 20]");
  if (nk < 2 || !(kmax > 0.0) || !std::isfinite(kmax)) return fail(nullptr, VDWXC_ETABLE, "bad kernel k-grid");
  for (int i = 0; i < nq; ++i) {
    if (!std::isfinite(qmesh[i]) || !(qmesh[i] > 0.0) || (i > 0 && !(qmesh[i] > qmesh[i - 1])))
      return fail(nullptr, VDWXC_ETABLE, "q-mesh must be positive and strictly increasing");
  }
  // q0 saturates at a = 5 (appendix); a mesh ending below it would leave q0 in (q_M-1, 5] outside
  // every spline interval
  if (!(qmesh[nq - 1] >= kSatA * (1.0 - 1e-12)))
    return fail(nullptr, VDWXC_ETABLE, "q-mesh must reach the saturation value q0 = 5 (last point >= 5)");
  // the contraction addresses the pair table with 32-bit byte offsets
  if (double(pair_table_bytes(VDWXC_FP64, nk)) >= 2147483648.0)
    return fail(nullptr, VDWXC_ETABLE, "kernel table has too many k nodes (its pair table must stay below 2 GiB)");
  const size_t tsz = size_t(nk) * nq * nq;
  for (size_t i = 0; i < tsz; ++i)
    if (!std::isfinite(table[i])) return fail(nullptr, VDWXC_ETABLE, "kernel table contains NaN/inf");
  for (int j = 0; j < nk; ++j)
    for (int a = 0; a < nq; ++a)
      for (int b = 0; b < a; ++b) {
        const double x = table[(size_t(j) * nq + a) * nq + b], y = table[(size_t(j) * nq + b) * nq + a];
        if (std::fabs(x - y) > 1e-12 * std::max(std::fabs(x), std::fabs(y)))
          return fail(nullptr, VDWXC_ETABLE, "kernel table must be symmetric in (a, b)");
      }

  vdwxc_ctx* h = new (std::nothrow) vdwxc_ctx();
  if (!h) return fail(nullptr, VDWXC_ENOMEM, "host allocation failed");
  h->n1 = grid[0];
  h->n2 = grid[1];
  h->n3 = grid[2];
  h->h3 = grid[2] / 2 + 1;
  std::memcpy(h->cell, cell, sizeof(h->cell));
  h->omega = det3(cell);
  h->flavour = flavour;
  h->precision = precision;
  h->M = nq;
  h->nk = nk;
  h->kmax = kmax;
  h->qmesh.assign(qmesh, qmesh + nq);
  h->stream = static_cast<hipStream_t>(hip_stream);

  const int n[3] = {h->n1, h->n2, h->n3};
  for (int a = 0; a < 3; ++a)
    if (!factor_axis(n[a], h->plan[a])) {
      release(h);
      return fail(nullptr, VDWXC_EINVAL, "grid sizes must be products of 2, 3, 5 and 7");
    }
  Geometry& g = h->geo;
  g.n1 = h->n1; g.n2 = h->n2; g.n3 = h->n3; g.h3 = h->h3; g.M = nq;
  g.zab = flavour == VDWXC_DF1 ? -0.8491 : -1.887;
  reciprocal(cell, g.bvec);
  g.kmax = kmax;
  g.nk = nk;
  g.inv_dk = double(nk - 1) / kmax;
  for (int i = 0; i < 3; ++i)
    g.bn2[i] = g.bvec[3 * i] * g.bvec[3 * i] + g.bvec[3 * i + 1] * g.bvec[3 * i + 1] + g.bvec[3 * i + 2] * g.bvec[3 * i + 2];
  {
    bool ortho = true;
    for (int i = 0; i < 3; ++i)
      for (int j = i + 1; j < 3; ++j) {
        const double d = cell[3 * i] * cell[3 * j] + cell[3 * i + 1] * cell[3 * j + 1] + cell[3 * i + 2] * cell[3 * j + 2];
        const double ni = std::sqrt(cell[3 * i] * cell[3 * i] + cell[3 * i + 1] * cell[3 * i + 1] + cell[3 * i + 2] * cell[3 * i + 2]);
        const double nj = std::sqrt(cell[3 * j] * cell[3 * j] + cell[3 * j + 1] * cell[3 * j + 1] + cell[3 * j + 2] * cell[3 * j + 2]);
        if (std::fabs(d) > 1e-14 * ni * nj) ortho = false;
      }
    h->ortho = ortho;
  }
  // |G| is even in kx exactly (bitwise, as the kernels compute it) when b1 has no y, z and b2, b3
  // no x component: then the kx and -kx lanes of the contraction share one table read
  g.xpair = (h->n1 % 2 == 0) && g.bvec[1] == 0.0 && g.bvec[2] == 0.0 && g.bvec[3] == 0.0 && g.bvec[6] == 0.0;
  if (!(max_gnorm2(n, g.bvec) < kmax * kmax)) {
    release(h);
    return fail(nullptr, VDWXC_EINVAL, "grid reaches |G| >= kmax of the kernel table (grid too fine)");
  }
  bool ok = line_launch(kMaxThreadsZ, h->n3, h->n2, 16, h->zl64) && line_launch(kMaxThreadsZ, h->n3, h->n2, 8, h->zl32) &&
            line_launch(kMaxThreadsY, h->n2, h->n1, 16, h->yl64, kEPT, h->n2 == 512 ? VDWXC_YTILE64_512 : VDWXC_YTILE64) &&
            line_launch(kMaxThreadsY, h->n2, h->n1, 16, h->yl64i, kEPT, VDWXC_YTILE64_INV) &&
            line_launch(kMaxThreadsY, h->n2, h->n1, 8, h->yl32, kEPT, VDWXC_YTILE32) &&
            line_launch(kMaxThreadsY, h->n2, h->n1, 8, h->yl32i, kEPT, VDWXC_YTILE32_INV);
  {
    // contraction pass: one thread per k-point up to kMaxThreadsX (the kernel strides beyond)
    Launch& L = precision == VDWXC_FP64 ? h->xl64 : h->xl32;
    // the contraction pass keeps its lines unpadded and reads twiddles from global memory, so
    // its LDS is exactly the N_alpha lines of one column
    L.tile = nq;
    L.nthr = std::min(kMaxThreadsX, std::max(64, round_up(h->n1, 64)));
    L.lstride = lds_span<kXPad>(h->n1);
    L.lds = std::max<size_t>(size_t(nq) * L.lstride * (precision == VDWXC_FP64 ? 16 : 8), 16 * sizeof(double));
    ok = ok && h->n1 <= L.nthr * kEPTC && h->n1 <= kMaxAxis && L.lds <= kMaxLds;
    // FP32: the register-capped kernel (128 VGPRs) fits four waves per SIMD, e.g. two 512-thread
    // blocks per CU at N1 = 512 when LDS allows; measured faster at every size tried
    h->x_capped = precision == VDWXC_FP32_MIXED && L.nthr >= VDWXC_XCAP_MIN_THREADS && 2 * L.lds <= kMaxLds;
  }
  // the z passes keep three per-point values in LDS next to the lines: shrink the tile until
  // they fit (the plain-field z passes use the same tile)
  auto fit_state = [&](Launch& L, size_t cplx, size_t real, int ept) {
    while (L.tile > 1) {
      const size_t npts = size_t(L.tile) * h->n3;
      const size_t need = L.lds + npts * 3 * real + ((npts + 15) & ~size_t(15)) + 4096;
      if (need <= kMaxLds) break;
      L.tile /= 2;
      L.nthr = threads_for(long(L.tile) * h->n3, ept, kMaxThreadsZ);
      L.lds = ((size_t(h->n3) * cplx + 15) & ~size_t(15)) + size_t(L.tile) * L.lstride * cplx;
    }
  };
  // the assembly pass: its own tile, 4 points per thread
  ok = ok && line_launch(kMaxThreadsZ, h->n3, h->n2, 16, h->za64, kEPTA) &&
       line_launch(kMaxThreadsZ, h->n3, h->n2, 8, h->za32, kEPTA);
  fit_state(h->zl64, 16, 8, kEPT);
  fit_state(h->zl32, 8, 4, kEPT);
  fit_state(h->za64, 16, 8, kEPTA);
  fit_state(h->za32, 8, 4, kEPTA);
  h->lds_theta64 = zstate_lds<double>(h->zl64, h->n3, 2);
  h->lds_theta32 = zstate_lds<float>(h->zl32, h->n3, 2);
  h->lds_asm64 = zstate_lds<double>(h->za64, h->n3, 3);
  h->lds_asm32 = zstate_lds<float>(h->za32, h->n3, 3);
  ok = ok && h->lds_asm64 <= kMaxLds && h->lds_asm32 <= kMaxLds;
  // assembly: every thread covers its kEPTA points and its share of the half spectrum (pair
  // prefetch depth kEPTA / 2 + 1)
  for (const Launch* L : {&h->za64, &h->za32})
    ok = ok && long(L->nthr) * kEPTA >= long(L->tile) * h->n3 && long(L->nthr) * (kEPTA / 2 + 1) >= long(L->tile) * h->h3;
  if (!ok) {
    release(h);
    return fail(nullptr, VDWXC_EINVAL, "grid too large for one block per line (see size limits in vdwxc_gpu.h)");
  }

  auto bail = [&](hipError_t e, const char* what) {
    release(h);
    return fail(nullptr, e == hipErrorOutOfMemory ? VDWXC_ENOMEM : VDWXC_EDEVICE,
                std::string(what) + ": " + hipGetErrorString(e));
  };
  hipError_t e = hipGetDevice(&h->device);
  if (e != hipSuccess) return bail(e, "hipGetDevice");
  if ((e = ensure_scratch_address(h->device)) != hipSuccess) return bail(e, "static work memory address");
  if ((e = acquire_table(h->device, precision, nq, qmesh, nk, kmax, table, &h->tab)) != hipSuccess)
    return bail(e, "kernel table upload");
  for (int a = 0; a < 3; ++a)
    if ((e = acquire_twiddles(h->device, n[a], &h->tw[a])) != hipSuccess) return bail(e, "twiddle upload");
  h->buf_bytes = complex_buffer_bytes(h->n1, h->n2, h->n3, precision, nq);
  const Layout lay = workspace_layout(h->n1, h->n2, h->n3, precision, nq);
  h->ws_bytes = lay.total;
  if (!(flags & VDWXC_INIT_NO_WORKSPACE)) {
    if ((e = hipMalloc(&h->d_ws, h->ws_bytes)) != hipSuccess) return bail(e, "work buffers");
    h->work = carve(h->d_ws, lay);
  }
  if ((e = hipMalloc(reinterpret_cast<void**>(&h->d_energy), sizeof(double))) != hipSuccess) return bail(e, "energy");
  if (h->d_ws) {
    // flag [0]: raised by the theta pass, [1]: the last evaluation's result (see energy_reduce_block)
    hipLaunchKernelGGL(k_clear_flags, dim3(1), dim3(64), 0, h->stream, h->work.flag);
    if ((e = hipGetLastError()) != hipSuccess || (e = hipStreamSynchronize(h->stream)) != hipSuccess)
      return bail(e, "flag");
  }
  if ((e = hipHostMalloc(reinterpret_cast<void**>(&h->h_energy), sizeof(double), hipHostMallocDefault)) != hipSuccess)
    return bail(e, "pinned energy");
  if ((e = hipHostMalloc(reinterpret_cast<void**>(&h->h_flag), sizeof(int), hipHostMallocDefault)) != hipSuccess)
    return bail(e, "pinned flag");

  // z tiles by occupancy (the plain-field z passes share the theta tile)
  set_lds_limit(k_theta_zfwd<double, kEPT, true>, kMaxLds);
  set_lds_limit(k_theta_zfwd<float, kEPT, true>, kMaxLds);
  set_lds_limit(k_zinv_assemble<double, kEPTA, kEPTA, asm_pb<double>()>, kMaxLds);
  set_lds_limit(k_zinv_assemble<float, kEPTA, kEPTA, asm_pb<float>()>, kMaxLds);
  if (!pick_ztile<double>(k_theta_zfwd<double, kEPT, true>, h->n3, h->n2, 2, kEPT, h->zl64, h->lds_theta64) ||
      !pick_ztile<float>(k_theta_zfwd<float, kEPT, true>, h->n3, h->n2, 2, kEPT, h->zl32, h->lds_theta32) ||
      !(pick_ztile<double>(k_zinv_assemble<double, kEPTA, kEPTA, asm_pb<double>()>, h->n3, h->n2, 3, kEPTA, h->za64,
                           h->lds_asm64, asm_pb<double>()) ||
        pick_ztile<double>(k_zinv_assemble<double, kEPTA, kEPTA, asm_pb<double>()>, h->n3, h->n2, 3, kEPTA, h->za64,
                           h->lds_asm64, 1)) ||
      !(pick_ztile<float>(k_zinv_assemble<float, kEPTA, kEPTA, asm_pb<float>()>, h->n3, h->n2, 3, kEPTA, h->za32,
                          h->lds_asm32, asm_pb<float>()) ||
        pick_ztile<float>(k_zinv_assemble<float, kEPTA, kEPTA, asm_pb<float>()>, h->n3, h->n2, 3, kEPTA, h->za32,
                          h->lds_asm32, 1))) {
    release(h);
    return fail(nullptr, VDWXC_EINVAL, "grid too large for one block per line (see size limits in vdwxc_gpu.h)");
  }
  {
    int zt = 2;   // first z tile of the y and x divergence passes: min(16, n3 rounded up), >= 2
    while (zt < std::min(VDWXC_DIV_ZT, h->n3)) zt *= 2;
    const int yt = std::min(kLineTile, h->n2);
    set_lds_limit(k_div_z<double, kEPT>, kMaxLds);
    set_lds_limit(k_div_y<double, kEPT>, kMaxLds);
    set_lds_limit(k_div_x<double, kEPT>, kMaxLds);
    set_lds_limit(k_div_z<float, kEPT>, kMaxLds);
    set_lds_limit(k_div_y<float, kEPT>, kMaxLds);
    set_lds_limit(k_div_x<float, kEPT>, kMaxLds);
    set_lds_limit(k_grad_z<double, kEPT>, kMaxLds);
    set_lds_limit(k_grad_y<double, kEPT>, kMaxLds);
    set_lds_limit(k_grad_x<double, kEPT>, kMaxLds);
    if (!pick_div<double>(k_div_z<double, kEPT>, true, false, h->n3, yt, h->dz64) ||
        !pick_div<double>(k_div_y<double, kEPT>, false, false, h->n2, zt, h->dy64) ||
        !pick_div<double>(k_div_x<double, kEPT>, false, true, h->n1, zt, h->dx64) ||
        !pick_div<float>(k_div_z<float, kEPT>, true, false, h->n3, yt, h->dz32) ||
        !pick_div<float>(k_div_y<float, kEPT>, false, false, h->n2, zt, h->dy32) ||
        !pick_div<float>(k_div_x<float, kEPT>, false, true, h->n1, zt, h->dx32) ||
        !pick_div<double>(k_grad_z<double, kEPT>, true, true, h->n3, yt, h->gz) ||
        !pick_div<double>(k_grad_y<double, kEPT>, false, false, h->n2, zt, h->gy) ||
        !pick_div<double>(k_grad_x<double, kEPT>, false, false, h->n1, zt, h->gx)) {
      release(h);
      return fail(nullptr, VDWXC_EINVAL, "grid too large for one block per line (see size limits in vdwxc_gpu.h)");
    }
  }

  // N3 = 512: the register-state theta pass takes 64 threads per line and VDWXC_T512_TILE* lines
  // per block (fewer when N2 is smaller); its LDS is the lines, the twiddles and the spline tables
  h->z512 = h->n3 == 512;
  if (h->z512) {
    for (Launch* L : {&h->t512_64, &h->t512_32}) {
      const size_t cplx = L == &h->t512_64 ? 16 : 8;
      const int pb = cplx == 16 ? t512_pb<double>() : t512_pb<float>();
      L->tile = std::min(cplx == 16 ? VDWXC_T512_TILE64 : VDWXC_T512_TILE32, h->n2);
      L->nthr = 64 * L->tile;
      L->lstride = lds_span<>(512);
      L->lds = tw_lds_bytes<double2>(512) * cplx / 16 + size_t(pb) * L->tile * L->lstride * cplx +
               (cplx == 16 ? spline_lds_bytes<double>() : spline_lds_bytes<float>()) + 16;
    }
    for (Launch* L : {&h->a512_64, &h->a512_32}) {
      const size_t cplx = L == &h->a512_64 ? 16 : 8;
      const int pb = cplx == 16 ? a512_pb<double>() : a512_pb<float>();
      L->tile = std::min(cplx == 16 ? VDWXC_A512_TILE64 : VDWXC_A512_TILE32, h->n2);
      L->nthr = 64 * L->tile;
      L->lstride = lds_span<>(512);
      L->lds = std::max(tw_lds_bytes<double2>(512) * cplx / 16 + size_t(pb) * L->tile * L->lstride * cplx +
                            (cplx == 16 ? spline_lds_bytes<double>() : spline_lds_bytes<float>()) + 16,
                        // the first block's energy sum uses one double per wave of LDS
                        tw_lds_bytes<double2>(512) * cplx / 16 + size_t(L->nthr / 64) * sizeof(double));
    }
    set_lds_limit(k_zinv_assemble512<double, a512_pb<double>(), a512_wpe<double>(), a512_pf<double>()>, h->a512_64.lds);
    set_lds_limit(k_zinv_assemble512<float, a512_pb<float>(), a512_wpe<float>(), a512_pf<float>()>, h->a512_32.lds);
    set_lds_limit(k_theta_zfwd512<double, true, t512_wpe<double>(), t512_pb<double>()>, h->t512_64.lds);
    set_lds_limit(k_theta_zfwd512<double, false, t512_wpe<double>(), t512_pb<double>()>, h->t512_64.lds);
    set_lds_limit(k_theta_zfwd512<float, true, t512_wpe<float>(), t512_pb<float>()>, h->t512_32.lds);
    set_lds_limit(k_theta_zfwd512<float, false, t512_wpe<float>(), t512_pb<float>()>, h->t512_32.lds);
  }

  // dynamic LDS above the default limit
  set_lds_limit(k_theta_zfwd<double, kEPT, false>, h->lds_theta64);
  set_lds_limit(k_theta_zfwd<double, kEPT, true>, h->lds_theta64);
  set_lds_limit(k_theta_zfwd<float, kEPT, false>, h->lds_theta32);
  set_lds_limit(k_theta_zfwd<float, kEPT, true>, h->lds_theta32);
  set_lds_limit(k_zinv_assemble<double, kEPTA, kEPTA, asm_pb<double>()>, h->lds_asm64);
  set_lds_limit(k_zinv_assemble<float, kEPTA, kEPTA, asm_pb<float>()>, h->lds_asm32);
  set_lds_limit(k_ypass<double, kEPT, -1>, h->yl64.lds);
  set_lds_limit(k_ypass<double, kEPT, +1>, h->yl64i.lds);
  set_lds_limit(k_ypass<float, kEPT, -1>, h->yl32.lds);
  set_lds_limit(k_ypass<float, kEPT, +1>, h->yl32i.lds);
  switch (q_bucket(nq)) {
    case 8: set_xcontract_lds<double, 8>(h->xl64.lds); set_xcontract_lds<float, 8>(h->xl32.lds); break;
    case 10: set_xcontract_lds<double, 10>(h->xl64.lds); set_xcontract_lds<float, 10>(h->xl32.lds); break;
    case 12: set_xcontract_lds<double, 12>(h->xl64.lds); set_xcontract_lds<float, 12>(h->xl32.lds); break;
    case 16: set_xcontract_lds<double, 16>(h->xl64.lds); set_xcontract_lds<float, 16>(h->xl32.lds); break;
    default: set_xcontract_lds<double, 20>(h->xl64.lds); set_xcontract_lds<float, 20>(h->xl32.lds); break;
  }
  set_lds_limit(k_grad_z<double, kEPT>, h->gz.lds);
  set_lds_limit(k_grad_y<double, kEPT>, h->gy.lds);
  set_lds_limit(k_grad_x<double, kEPT>, h->gx.lds);
  set_lds_limit(k_div_z<double, kEPT>, h->dz64.lds);
  set_lds_limit(k_div_y<double, kEPT>, h->dy64.lds);
  set_lds_limit(k_div_x<double, kEPT>, h->dx64.lds);
  set_lds_limit(k_div_z<float, kEPT>, h->dz32.lds);
  set_lds_limit(k_div_y<float, kEPT>, h->dy32.lds);
  set_lds_limit(k_div_x<float, kEPT>, h->dx32.lds);
  (void)hipGetLastError();
  *out = h;
  return VDWXC_OK;
}

vdwxc_status vdwxc_init(vdwxc_handle* out, const int grid[3], const double cell[9], vdwxc_flavour flavour,
                        vdwxc_precision precision, const char* kernel_table_path, void* hip_stream) {
  if (!out) return fail(nullptr, VDWXC_EINVAL, "out must not be NULL");
  *out = nullptr;
  const std::string path = kernel_table_path ? std::string(kernel_table_path) : default_table_path();
  kernel_table_path = path.c_str();
  FILE* f = std::fopen(kernel_table_path, "rb");
  if (!f) return fail(nullptr, VDWXC_ETABLE, std::string("cannot open kernel table ") + kernel_table_path);
  char magic[4];
  unsigned int hdr[3];
  double kmax = 0.0;
  bool ok = std::fread(magic, 1, 4, f) == 4 && std::memcmp(magic, "VDWK", 4) == 0 &&
            std::fread(hdr, sizeof(unsigned int), 3, f) == 3 && hdr[0] == 1 && hdr[1] >= 4 &&
            hdr[1] <= unsigned(kMaxQ) && hdr[2] >= 2 && hdr[2] < (1u << 24) && std::fread(&kmax, sizeof(double), 1, f) == 1;
  std::vector<double> q, t;
  if (ok) {
    q.resize(hdr[1]);
    t.resize(size_t(hdr[2]) * hdr[1] * hdr[1]);
    ok = std::fread(q.data(), sizeof(double), q.size(), f) == q.size() &&
         std::fread(t.data(), sizeof(double), t.size(), f) == t.size();
  }
  std::fclose(f);
  if (!ok) return fail(nullptr, VDWXC_ETABLE, std::string("malformed kernel table file ") + kernel_table_path);
  return vdwxc_init_table(out, grid, cell, flavour, precision, int(hdr[1]), q.data(), int(hdr[2]), kmax, t.data(),
                          hip_stream);
}

vdwxc_status vdwxc_calculate_async(vdwxc_handle h, const double* n, const double* sigma, double* dedn,
                                   double* dedsigma, double* energy_dev) {
  if (vdwxc_status st0 = check_work(h); st0 != VDWXC_OK) return st0;
  if (!n || !sigma || !dedn || !dedsigma || !energy_dev)
    return fail(h, VDWXC_EINVAL, "array arguments must not be NULL");
  return run_partials(h, h->work, n, sigma, dedn, dedsigma, energy_dev);
}

vdwxc_status vdwxc_calculate(vdwxc_handle h, const double* n, const double* sigma, double* dedn, double* dedsigma,
                             double* energy_host) {
  if (vdwxc_status st0 = check_work(h); st0 != VDWXC_OK) return st0;
  if (!n || !sigma || !dedn || !dedsigma || !energy_host)
    return fail(h, VDWXC_EINVAL, "array arguments must not be NULL");
  vdwxc_status st = run_partials(h, h->work, n, sigma, dedn, dedsigma, h->d_energy);
  if (st != VDWXC_OK) return st;
  return read_energy(h, energy_host);
}

vdwxc_status vdwxc_calculate_spin_async(vdwxc_handle h, const double* n_up, const double* n_dn,
                                        const double* sigma_uu, const double* sigma_dd, double* dedn_up,
                                        double* dedn_dn, double* dedsigma_uu, double* dedsigma_dd,
                                        double* energy_dev) {
  if (vdwxc_status st0 = check_work(h); st0 != VDWXC_OK) return st0;
  const double* in[4] = {n_up, n_dn, sigma_uu, sigma_dd};
  double* out[4] = {dedn_up, dedn_dn, dedsigma_uu, dedsigma_dd};
  if (!energy_dev) return fail(h, VDWXC_EINVAL, "array arguments must not be NULL");
  if (vdwxc_status st = check_spin_arrays(h, in, out); st != VDWXC_OK) return st;
  return run_spin(h, h->work, n_up, n_dn, sigma_uu, sigma_dd, dedn_up, dedn_dn, dedsigma_uu, dedsigma_dd, energy_dev);
}

vdwxc_status vdwxc_calculate_spin(vdwxc_handle h, const double* n_up, const double* n_dn, const double* sigma_uu,
                                  const double* sigma_dd, double* dedn_up, double* dedn_dn, double* dedsigma_uu,
                                  double* dedsigma_dd, double* energy_host) {
  if (vdwxc_status st0 = check_work(h); st0 != VDWXC_OK) return st0;
  const double* in[4] = {n_up, n_dn, sigma_uu, sigma_dd};
  double* out[4] = {dedn_up, dedn_dn, dedsigma_uu, dedsigma_dd};
  if (!energy_host) return fail(h, VDWXC_EINVAL, "array arguments must not be NULL");
  if (vdwxc_status st = check_spin_arrays(h, in, out); st != VDWXC_OK) return st;
  vdwxc_status st = run_spin(h, h->work, n_up, n_dn, sigma_uu, sigma_dd, dedn_up, dedn_dn, dedsigma_uu, dedsigma_dd,
                             h->d_energy);
  if (st != VDWXC_OK) return st;
  return read_energy(h, energy_host);
}

vdwxc_status vdwxc_calculate_spin_potential_async(vdwxc_handle h, const double* n_up, const double* n_dn,
                                                  const double* grad_up, const double* grad_dn, double* v_up,
                                                  double* v_dn, double* energy_dev) {
  if (vdwxc_status st0 = check_work(h); st0 != VDWXC_OK) return st0;
  if (!energy_dev) return fail(h, VDWXC_EINVAL, "array arguments must not be NULL");
  if (vdwxc_status st = check_spin_potential_arrays(h, n_up, n_dn, grad_up, grad_dn, v_up, v_dn); st != VDWXC_OK)
    return st;
  return run_spin_potential(h, h->work, n_up, n_dn, grad_up, grad_dn, v_up, v_dn, energy_dev);
}

vdwxc_status vdwxc_calculate_spin_potential(vdwxc_handle h, const double* n_up, const double* n_dn,
                                            const double* grad_up, const double* grad_dn, double* v_up, double* v_dn,
                                            double* energy_host) {
  if (vdwxc_status st0 = check_work(h); st0 != VDWXC_OK) return st0;
  if (!energy_host) return fail(h, VDWXC_EINVAL, "array arguments must not be NULL");
  if (vdwxc_status st = check_spin_potential_arrays(h, n_up, n_dn, grad_up, grad_dn, v_up, v_dn); st != VDWXC_OK)
    return st;
  vdwxc_status st = run_spin_potential(h, h->work, n_up, n_dn, grad_up, grad_dn, v_up, v_dn, h->d_energy);
  if (st != VDWXC_OK) return st;
  return read_energy(h, energy_host);
}

vdwxc_status vdwxc_calculate_potential_async(vdwxc_handle h, const double* n, const double* grad_n, double* v,
                                             double* energy_dev) {
  if (vdwxc_status st0 = check_work(h); st0 != VDWXC_OK) return st0;
  if (!n || !v || !energy_dev) return fail(h, VDWXC_EINVAL, "array arguments must not be NULL");
  return run_potential(h, h->work, n, grad_n, v, energy_dev);
}

vdwxc_status vdwxc_calculate_potential(vdwxc_handle h, const double* n, const double* grad_n, double* v,
                                       double* energy_host) {
  if (vdwxc_status st0 = check_work(h); st0 != VDWXC_OK) return st0;
  if (!n || !v || !energy_host) return fail(h, VDWXC_EINVAL, "array arguments must not be NULL");
  vdwxc_status st = run_potential(h, h->work, n, grad_n, v, h->d_energy);
  if (st != VDWXC_OK) return st;
  return read_energy(h, energy_host);
}

vdwxc_status vdwxc_calculate_potential_noalloc(vdwxc_handle h, const double* n, const double* grad_n, double* v,
                                               double* energy_dev) {
  if (check_handle(h) != VDWXC_OK) return VDWXC_ESTATE;
  if (!n || !v || !energy_dev) return fail(h, VDWXC_EINVAL, "array arguments must not be NULL");
  const Layout lay = workspace_layout(h->n1, h->n2, h->n3, h->precision, h->M);
  if (lay.total > kScratchBytes)
    return fail(h, VDWXC_EINVAL, "grid needs " + std::to_string(lay.total) + " bytes of work memory, more than the " +
                                     std::to_string(kScratchBytes) + " of the static work memory");
  void* base = scratch_address(h->device);
  if (!base) return fail(h, VDWXC_ESTATE, "no static work memory address for this device");
  Work w = carve(base, lay);
  w.timed = false;   // taking a timing event may allocate
  HIP_TRY(h, hipSetDevice(h->device));
  // the array keeps the last call's contents: the NaN flags must start at zero
  hipLaunchKernelGGL(k_clear_flags, dim3(1), dim3(64), 0, h->stream, w.flag);
  return run_potential(h, w, n, grad_n, v, energy_dev);
}

vdwxc_status vdwxc_calculate_lda_async(vdwxc_handle h, const double* n, double* v, double* energy_dev) {
  if (vdwxc_status st0 = check_work(h); st0 != VDWXC_OK) return st0;
  if (!n || !v || !energy_dev) return fail(h, VDWXC_EINVAL, "array arguments must not be NULL");
  if (n == v) return fail(h, VDWXC_EINVAL, "v must not be the density array");
  return run_lda(h, h->work, n, v, energy_dev);
}

vdwxc_status vdwxc_set_workspace(vdwxc_handle h, void* workspace, size_t bytes) {
  if (check_handle(h) != VDWXC_OK) return VDWXC_ESTATE;
  const Layout lay = workspace_layout(h->n1, h->n2, h->n3, h->precision, h->M);
  if (workspace) {
    if (bytes < lay.total)
      return fail(h, VDWXC_EINVAL, "workspace of " + std::to_string(bytes) + " bytes, the handle needs " +
                                       std::to_string(lay.total));
    if (reinterpret_cast<uintptr_t>(workspace) % 256 != 0) return fail(h, VDWXC_EINVAL, "workspace must be 256-byte aligned");
    h->work = carve(workspace, lay);
  } else {
    h->work = h->d_ws ? carve(h->d_ws, lay) : Work{};
  }
  if (!h->work.A) return VDWXC_OK;
  HIP_TRY(h, hipSetDevice(h->device));
  // the NaN flags live in the work memory and must start at zero
  hipLaunchKernelGGL(k_clear_flags, dim3(1), dim3(64), 0, h->stream, h->work.flag);
  return finish_launch(h);
}

const char* vdwxc_stage_name(int stage) {
  static const char* names[VDWXC_NUM_STAGES] = {
      "theta_zfwd", "y_fwd", "x_contract", "y_inv", "z_assemble", "grad_z", "grad_y",
      "grad_x", "div_z", "div_y", "div_x", "lda", "spin"};
  return (stage >= 0 && stage < VDWXC_NUM_STAGES) ? names[stage] : "?";
}

vdwxc_status vdwxc_enable_timing(vdwxc_handle h, int enable) {
  if (check_handle(h) != VDWXC_OK) return VDWXC_ESTATE;
  HIP_TRY(h, hipStreamSynchronize(h->stream));
  for (auto& p : h->pending) {
    h->free_events.push_back(p.start);
    h->free_events.push_back(p.stop);
  }
  h->pending.clear();
  for (int i = 0; i < VDWXC_NUM_STAGES; ++i) { h->stage_ms[i] = 0.0; h->stage_count[i] = 0; }
  h->timing = enable != 0;
  return VDWXC_OK;
}

vdwxc_status vdwxc_read_timing(vdwxc_handle h, double* ms, long long* launches) {
  if (check_handle(h) != VDWXC_OK) return VDWXC_ESTATE;
  if (!ms || !launches) return fail(h, VDWXC_EINVAL, "timing arrays must not be NULL");
  HIP_TRY(h, hipStreamSynchronize(h->stream));
  for (auto& p : h->pending) {
    float t = 0.f;
    HIP_TRY(h, hipEventElapsedTime(&t, p.start, p.stop));
    h->stage_ms[p.stage] += t;
    h->stage_count[p.stage] += 1;
    h->free_events.push_back(p.start);
    h->free_events.push_back(p.stop);
  }
  h->pending.clear();
  for (int i = 0; i < VDWXC_NUM_STAGES; ++i) {
    ms[i] = h->stage_ms[i];
    launches[i] = h->stage_count[i];
    h->stage_ms[i] = 0.0;
    h->stage_count[i] = 0;
  }
  return VDWXC_OK;
}

vdwxc_status vdwxc_set_stream(vdwxc_handle h, void* hip_stream) {
  if (check_handle(h) != VDWXC_OK) return VDWXC_ESTATE;
  h->stream = static_cast<hipStream_t>(hip_stream);
  return VDWXC_OK;
}

vdwxc_status vdwxc_print(vdwxc_handle h) {
  if (check_handle(h) != VDWXC_OK) return VDWXC_ESTATE;
  std::printf("vdwxc_gpu handle: grid %d x %d x %d, cell [%g %g %g | %g %g %g | %g %g %g] bohr, volume %g bohr^3\n",
              h->n1, h->n2, h->n3, h->cell[0], h->cell[1], h->cell[2], h->cell[3], h->cell[4], h->cell[5],
              h->cell[6], h->cell[7], h->cell[8], h->omega);
  std::printf("  flavour %s (Z_ab = %g), precision %s, q-mesh %d points [%g .. %g], kernel table %d x %d x %d to "
              "k = %g\n",
              h->flavour == VDWXC_DF1 ? "vdW-DF1" : "vdW-DF2", h->geo.zab,
              h->precision == VDWXC_FP64 ? "FP64" : "FP32_MIXED", h->M, h->qmesh.front(), h->qmesh.back(), h->nk,
              h->M, h->M, h->kmax);
  std::printf("  work buffers 2 x %.3f MB, work memory %.3f MB at %p, device %d\n", h->buf_bytes / 1e6,
              h->ws_bytes / 1e6, h->d_ws, h->device);
  std::fflush(stdout);
  return VDWXC_OK;
}

vdwxc_status vdwxc_finalize(vdwxc_handle* hp) {
  if (!hp || !*hp) return VDWXC_ESTATE;
  vdwxc_ctx* h = *hp;
  (void)hipSetDevice(h->device);
  (void)hipStreamSynchronize(h->stream);
  release(h);
  *hp = nullptr;
  return VDWXC_OK;
}

}  // extern "C"
