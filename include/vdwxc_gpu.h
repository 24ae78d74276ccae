/* vdwxc_gpu.h - C ABI of the MI355X (gfx950) vdW-DF nonlocal-correlation library.
 *
 * The library evaluates the nonlocal correlation energy of the vdW-DF family,
 *     E_c^nl = 1/2 \iint n(r) phi(q0(r), q0(r'), |r - r'|) n(r') dr dr'        (paper eq. 2)
 * in the Roman-Perez--Soler spline/FFT form (paper Sec. 2), with the five steps of the paper's
 * Sec. 3 procedure: theta_a(r) = n p_a(q0) on an N_alpha-point q-mesh, forward 3D FFTs, the
 * per-k contraction F_a(k) = sum_b phi_ab(|k|) theta_b(k) against a tabulated kernel that is
 * linearly interpolated in k (with the energy, eq. enlk), inverse 3D FFTs, and the partial
 * derivatives dE/dn, dE/dsigma (paper eqs. dedn, dedsigma); q0 follows the paper's appendix.
 * Everything runs on one GPU in hand-written HIP kernels.
 *
 * Conventions shared by every call:
 *  - Units: Hartree atomic units (bohr, electrons/bohr^3, Hartree).
 *  - Grids: N1 x N2 x N3 points of a periodic cell, stored row-major [N1][N2][N3] (N3 fastest),
 *    point (i,j,k) at r = (i/N1) a1 + (j/N2) a2 + (k/N3) a3.  Each N_i must be >= 1 and a product
 *    of the primes 2, 3, 5, 7.  Limits: N2, N3 <= 2048; the N_alpha lines of one x column must
 *    fit the 160 KiB of LDS of a compute unit, N_alpha * N1' * 16 bytes in FP64 and * 8 bytes in
 *    FP32_MIXED with N1' = N1 rounded up to a multiple of 32 (N1 <= 512 and 1024 at
 *    N_alpha = 20).  vdwxc_init rejects larger grids with VDWXC_EINVAL.
 *  - cell[9]: the lattice vectors a1, a2, a3 as rows, bohr; det(cell) must be > 0.
 *  - Arrays: every array argument of a calculate call is a DEVICE pointer to float64 data owned
 *    by the caller (e.g. a torch tensor); the library never frees or retains it after the call
 *    returns, and never writes inputs.  Outputs are overwritten, not accumulated.
 *  - Streams: all device work of a handle is enqueued on its HIP stream (hipStream_t passed as
 *    void*; NULL = the default stream).  One handle must not be used by two host threads at once,
 *    and calls on one handle are ordered by its stream.  Different handles are independent.
 *  - Errors: every call returns a vdwxc_status; nothing throws across the ABI.  On error the
 *    outputs are unspecified and vdwxc_last_error() holds a message.
 */
#ifndef VDWXC_GPU_H
#define VDWXC_GPU_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct vdwxc_ctx* vdwxc_handle; /* opaque: plans, tables, workspace, stream */

typedef enum {
  VDWXC_OK = 0,
  VDWXC_EINVAL = 1,  /* bad argument: grid, cell, NULL pointer, unsupported size, NaN input */
  VDWXC_ENOMEM = 2,  /* device or pinned-host allocation failed */
  VDWXC_EDEVICE = 3, /* a HIP runtime call failed */
  VDWXC_ETABLE = 4,  /* malformed kernel table (file or arrays) */
  VDWXC_ESTATE = 5   /* handle is NULL or already finalized */
} vdwxc_status;

/* Functional flavour: the gradient coefficient Z_ab of q0 (paper appendix). */
typedef enum { VDWXC_DF1 = 1 /* Z_ab = -0.8491 */, VDWXC_DF2 = 2 /* Z_ab = -1.887 */ } vdwxc_flavour;

/* Arithmetic of the path.  FP64: everything in double precision (the paper's choice, Sec. 6).
 * FP32_MIXED: in FP64 - q0 with its saturation and its two partial derivatives (every point, the
 * vacuum tail included), the spectral gradient of n, the per-k energy accumulation and the final
 * energy sum, and the sums of the derivative assembly over the fields; in FP32 - the spline state
 * handed from q0 to theta and to the assembly (interval position t, n dq0/dn, n dq0/dsigma), the
 * cubic spline weights and theta_a = n p_a(q0), every FFT, the kernel table, its interpolation and
 * the contraction, and the products F_a * (spline factor) before they enter the FP64 sums. */
typedef enum { VDWXC_FP64 = 0, VDWXC_FP32_MIXED = 1 } vdwxc_precision;

/* Create a handle for one grid and cell (paper Sec. 6, steps 1-3: vdwxc_new, set_unit_cell,
 * init).  grid[3] = {N1, N2, N3}; cell[9] as above.  The kernel table is read from
 * kernel_table_path, a binary file: bytes "VDWK", uint32 version (=1), uint32 M (q-mesh points,
 * 4 <= M <= 20), uint32 nk (>= 2), float64 kmax, float64 qmesh[M] (strictly increasing, > 0, the
 * last point >= 5, the saturation value of q0 in the paper's appendix), float64 table[nk][M][M]
 * with table[j][a][b] = phi_ab(j*kmax/(nk-1)) (symmetric in a, b), all little endian; nk is
 * limited so that the reordered table stays below 2 GiB (about 639 000 nodes), else VDWXC_ETABLE.
 * kernel_table_path NULL means the default table: the file named by the environment variable
 * VDWXC_KERNEL_TABLE, else vdw_kernel_table.vdwk in the directory of this library (written by
 * the build).  The grid's largest |G| must be below kmax (else VDWXC_EINVAL).  hip_stream is the
 * stream later calls enqueue on.  On success *out receives the handle; it owns device memory of
 * vdwxc_workspace_bytes_m() for its work buffers until vdwxc_finalize.  The read-only tables (the
 * q-mesh with its spline moments, the kernel table in the handle's precision, the twiddles of each
 * axis length) are shared by all handles on the device that use the same table and lengths,
 * reference counted, and freed with the last of them. */
vdwxc_status vdwxc_init(vdwxc_handle* out, const int grid[3], const double cell[9], vdwxc_flavour flavour,
                        vdwxc_precision precision, const char* kernel_table_path, void* hip_stream);

/* As vdwxc_init, with the kernel table given as HOST arrays (read during the call; the caller
 * keeps ownership): qmesh[nq], table[nk][nq][nq] as in the file format, the same limits. */
vdwxc_status vdwxc_init_table(vdwxc_handle* out, const int grid[3], const double cell[9], vdwxc_flavour flavour,
                              vdwxc_precision precision, int nq, const double* qmesh, int nk, double kmax,
                              const double* table, void* hip_stream);

/* Flags of vdwxc_init_table_ex. */
#define VDWXC_INIT_NO_WORKSPACE 1u /* the handle allocates no work memory: attach some with vdwxc_set_workspace */

/* As vdwxc_init_table, with flags (0 or VDWXC_INIT_NO_WORKSPACE; other bits give VDWXC_EINVAL).  With
 * VDWXC_INIT_NO_WORKSPACE the handle holds its plans and the shared tables but no work memory, so
 * it is cheap to keep many resident (e.g. one per grid shape and stream of a server); its calculate
 * calls return VDWXC_ESTATE until work memory is attached with vdwxc_set_workspace.  Nothing is
 * synchronised in that case. */
vdwxc_status vdwxc_init_table_ex(vdwxc_handle* out, const int grid[3], const double cell[9], vdwxc_flavour flavour,
                                 vdwxc_precision precision, int nq, const double* qmesh, int nk, double kmax,
                                 const double* table, void* hip_stream, unsigned flags);

/* Run the handle's later calculate calls (all but vdwxc_calculate_potential_noalloc) in caller-owned
 * device memory: workspace, 256-byte aligned, of bytes >= vdwxc_workspace_bytes_m(grid, precision,
 * N_alpha) (else VDWXC_EINVAL and nothing changes).  The caller keeps ownership, must keep the memory
 * alive until the stream has passed the work enqueued with it, and must not let two handles use it
 * at the same time (their streams would race).  workspace NULL returns the handle to its own work
 * memory (none for a VDWXC_INIT_NO_WORKSPACE handle).  The handle's own memory is kept, not freed, so
 * the call never synchronises: it only enqueues a small kernel on the handle's stream that clears the
 * NaN flags held in the work memory.  For pools of work buffers shared between handles, so that
 * switching a request to another buffer allocates and frees nothing. */
vdwxc_status vdwxc_set_workspace(vdwxc_handle h, void* workspace, size_t bytes);

/* The paper's evaluation (Sec. 3 steps 1-5, Sec. 6 step 4): from the density n and
 * sigma = |grad n|^2 (device, [N1][N2][N3]) compute the energy E_c^nl (written to *energy_host,
 * a host pointer) and the partial derivatives dedn = dE/dn|_sigma, dedsigma = dE/dsigma|_n per
 * grid point (device outputs, eqs. dedn and dedsigma; the derivative of E with respect to the
 * value n_j at one point is dedn_j * Omega/N).  Points with n < 1e-30 are vacuum: their dedn and
 * dedsigma are 0.  A NaN in n or sigma gives VDWXC_EINVAL.  Synchronises the handle's stream. */
vdwxc_status vdwxc_calculate(vdwxc_handle h, const double* n, const double* sigma, double* dedn,
                             double* dedsigma, double* energy_host);

/* The potential v = dE/dn|_sigma - div(2 dE/dsigma grad n), the functional derivative delta E/delta n
 * of paper Sec. 2 with sigma = |grad n|^2.  grad_n (device, [3][N1][N2][N3], Cartesian
 * components) is the caller's gradient of n; NULL means the library takes the spectral gradient
 * of n itself (then E is a function of n alone and dE/dn_j = v_j * Omega/N exactly).  The
 * divergence is spectral; frequencies on a Nyquist index are dropped in both derivatives.
 * Writes v (device, [N1][N2][N3]) and *energy_host (host).  Synchronises the handle's stream. */
vdwxc_status vdwxc_calculate_potential(vdwxc_handle h, const double* n, const double* grad_n, double* v,
                                       double* energy_host);

/* As vdwxc_calculate_potential but fully asynchronous on the handle's stream: the energy is
 * written to energy_dev (a device double) when the stream reaches it, NaN if the input held a
 * NaN.  The caller must keep n, grad_n, v and energy_dev alive until the stream has passed. */
vdwxc_status vdwxc_calculate_potential_async(vdwxc_handle h, const double* n, const double* grad_n, double* v,
                                             double* energy_dev);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc): vdwxc_calculate_potential_async with the handle's work
 * buffers replaced by a static array of 128 MiB that the library holds on each device until the
 * process ends.  The call allocates nothing (no hipMalloc, hipFree or allocating library routine;
 * per-stage timing events are not recorded) and enqueues the same kernels, so the results are
 * bitwise those of vdwxc_calculate_potential_async.  Grids whose work memory
 * (vdwxc_workspace_bytes_m) exceeds 128 MiB are rejected with VDWXC_EINVAL before any device work,
 * e.g. 64^3 fits in both precisions and 96^3 in neither.  All calls on one device share the array
 * and it keeps the last call's contents: calls that overlap on one device (other streams, other
 * threads, other handles) race and give wrong results, so the caller orders them.  The handle
 * must have been created on the device it runs on (vdwxc_init* records the array's address). */
vdwxc_status vdwxc_calculate_potential_noalloc(vdwxc_handle h, const double* n, const double* grad_n, double* v,
                                               double* energy_dev);

/* As vdwxc_calculate but asynchronous: the energy goes to the device double energy_dev. */
vdwxc_status vdwxc_calculate_async(vdwxc_handle h, const double* n, const double* sigma, double* dedn,
                                   double* dedsigma, double* energy_dev);

/* The semilocal LDA part of the vdW-DF correlation (paper eq. 1 splits E_c into E_c^LDA + E_c^nl):
 * the spin-paired Perdew-Wang (PW92) correlation energy per electron eps_c(r_s) of the paper's
 * appendix, r_s = (3/(4 pi n))^(1/3).  From the density n (device, [N1][N2][N3]) writes
 * E_c^LDA = \int n eps_c dr, the grid sum times Omega/N, to the device double energy_dev, and
 * v_c^LDA = d(n eps_c)/dn = eps_c - (r_s/3) d eps_c/d r_s per point to v (device, [N1][N2][N3];
 * it must not overlap n, which is rejected with VDWXC_EINVAL when v == n).  Arithmetic is FP64 in
 * both precisions; one streaming pass (8 bytes read and 8 written per point) and a fixed-order sum,
 * so equal inputs give equal bits.  Vacuum points (n < 1e-30) give v = 0 and no energy; a NaN in n
 * gives NaN at that point and in the energy.  Asynchronous on the handle's stream; it uses the
 * handle's work memory, so it is ordered with the handle's other calls by the stream. */
vdwxc_status vdwxc_calculate_lda_async(vdwxc_handle h, const double* n, double* v, double* energy_dev);

/* Spin-polarised vdW-DF (paper Sec. 7 announces the variant; the paper prints only the spin-paired
 * q0, so the spin q0 here is a stated reading): from the spin densities n_up, n_dn and
 * sigma_uu = |grad n_up|^2, sigma_dd = |grad n_dn|^2 (device, [N1][N2][N3] each) compute E_c^nl with
 * theta_a = n p_a(q0) for the total density n = n_up + n_dn (Sec. 2) and
 *   q0 = sum_s [(n_s/n) k_s - (Z_ab/36) sigma_ss / (n n_s k_s)] - (4 pi/3) eps_c(r_s, zeta),
 * k_s = (6 pi^2 n_s)^(1/3): the appendix's gradient-corrected LDA exchange spin-scaled
 * (E_x[n_up, n_dn] = (E_x[2 n_up] + E_x[2 n_dn])/2) and the spin-resolved Perdew-Wang 1992 correlation
 * (the appendix's eps_c(r_s, 0) with the published fits of eps_c(r_s, 1) and the spin stiffness);
 * saturation, clamp and vacuum as spin-paired, spin densities below 1e-30 (or negative) taken as
 * zero.  At n_up = n_dn it is the spin-paired functional (dedn_up = dedn_dn = dedn, dedsigma_ss =
 * 2 dedsigma).  Writes the partial derivatives dE/dn_up, dE/dn_dn, dE/dsigma_uu, dE/dsigma_dd per point
 * (device, [N1][N2][N3] each, normalised as in vdwxc_calculate) and the energy to the device double
 * energy_dev.  The four outputs serve as scratch during the call (they hold n and the equivalent
 * spin-paired sigma between the passes); they must not overlap each other or the inputs
 * (VDWXC_EINVAL).  Arithmetic of the conversions is FP64 in both precisions; the pipeline in
 * between runs in the handle's precision.  A NaN input gives NaN in the energy (the synchronous
 * form returns VDWXC_EINVAL).  Asynchronous on the handle's stream, in its work memory. */
vdwxc_status vdwxc_calculate_spin_async(vdwxc_handle h, const double* n_up, const double* n_dn,
                                        const double* sigma_uu, const double* sigma_dd, double* dedn_up,
                                        double* dedn_dn, double* dedsigma_uu, double* dedsigma_dd,
                                        double* energy_dev);

/* As vdwxc_calculate_spin_async with the energy written to *energy_host (a host pointer);
 * synchronises the handle's stream. */
vdwxc_status vdwxc_calculate_spin(vdwxc_handle h, const double* n_up, const double* n_dn, const double* sigma_uu,
                                  const double* sigma_dd, double* dedn_up, double* dedn_dn, double* dedsigma_uu,
                                  double* dedsigma_dd, double* energy_host);

/* Spin-polarised potentials v_up = dE/dn_up|sigma - div(2 dE/dsigma_uu grad n_up) and the same for
 * n_dn: the functional derivatives of the spin-polarised E of vdwxc_calculate_spin_async, which
 * depends on the gradients only through sigma_uu = |grad n_up|^2 and sigma_dd = |grad n_dn|^2 (paper
 * Sec. 2's potential, per spin).  grad_up, grad_dn (device, [3][N1][N2][N3] each, Cartesian
 * components) are the caller's gradients and are required (NULL: VDWXC_EINVAL); the divergences are
 * spectral with every Nyquist frequency dropped, as in vdwxc_calculate_potential.  Writes v_up, v_dn
 * (device, [N1][N2][N3]; v_dn serves as scratch for n during the call; neither may overlap the
 * inputs or the other, VDWXC_EINVAL) and the energy to the device double energy_dev.  Runs in the
 * handle's work memory, asynchronously on its stream. */
vdwxc_status vdwxc_calculate_spin_potential_async(vdwxc_handle h, const double* n_up, const double* n_dn,
                                                  const double* grad_up, const double* grad_dn, double* v_up,
                                                  double* v_dn, double* energy_dev);

/* As vdwxc_calculate_spin_potential_async with the energy written to *energy_host (a host pointer);
 * synchronises the handle's stream; a NaN input gives VDWXC_EINVAL. */
vdwxc_status vdwxc_calculate_spin_potential(vdwxc_handle h, const double* n_up, const double* n_dn,
                                            const double* grad_up, const double* grad_dn, double* v_up, double* v_dn,
                                            double* energy_host);

/* Device memory a handle for this grid allocates for its work buffers (excluding the shared
 * tables), for admission control, with the paper's N_alpha = 20 q-mesh points; 0 if the grid or
 * precision is invalid.  Host-only. */
size_t vdwxc_workspace_bytes(const int grid[3], vdwxc_precision precision);

/* As vdwxc_workspace_bytes for a q-mesh of nq points (4 <= nq <= 20). */
size_t vdwxc_workspace_bytes_m(const int grid[3], vdwxc_precision precision, int nq);

/* Change the stream later calls enqueue on. */
vdwxc_status vdwxc_set_stream(vdwxc_handle h, void* hip_stream);

/* Print the handle's state (grid, cell, precision, table, memory) to stdout (paper Sec. 6). */
vdwxc_status vdwxc_print(vdwxc_handle h);

/* Release all memory of *h and set *h = NULL (paper Sec. 6, step 5).  Waits for the stream. */
vdwxc_status vdwxc_finalize(vdwxc_handle* h);

/* Static description of a status code. */
const char* vdwxc_strerror(vdwxc_status s);

/* Message of the last failing call on h; with h == NULL, of the last failing vdwxc_init* call
 * of this thread.  Valid until the next call on the same handle / thread. */
const char* vdwxc_last_error(vdwxc_handle h);

/* Kernel stages of one evaluation, for the timing calls below. */
typedef enum {
  VDWXC_STAGE_THETA_ZFWD = 0,   /* q0, splines, theta, forward z FFT (Sec. 3 steps 1-2) */
  VDWXC_STAGE_Y_FWD = 1,        /* forward y FFT of the theta fields */
  VDWXC_STAGE_X_CONTRACT = 2,   /* forward x FFT, k-space contraction + energy, inverse x FFT (steps 2-4) */
  VDWXC_STAGE_Y_INV = 3,        /* inverse y FFT of the F fields */
  VDWXC_STAGE_Z_ASSEMBLE = 4,   /* inverse z FFT and dE/dn, dE/dsigma (steps 4-5); fixed-order energy sum */
  VDWXC_STAGE_GRAD_Z = 5,       /* spectral gradient of n (no gradient given), one axis per pass: */
  VDWXC_STAGE_GRAD_Y = 6,       /* z, y, x */
  VDWXC_STAGE_GRAD_X = 7,
  VDWXC_STAGE_DIV_Z = 8,        /* spectral divergence of 2 dE/dsigma grad n, one axis per pass: */
  VDWXC_STAGE_DIV_Y = 9,        /* z, y, x (the x pass subtracts it from the potential) */
  VDWXC_STAGE_DIV_X = 10,
  VDWXC_STAGE_LDA = 11,         /* LDA correlation pass (vdwxc_calculate_lda_async) */
  VDWXC_STAGE_SPIN = 12,        /* spin conversions before and after the pipeline (vdwxc_calculate_spin*) */
  VDWXC_NUM_STAGES = 13
} vdwxc_stage;

/* Per-stage timing with HIP events recorded on the handle's stream around every kernel launch
 * (off by default; recording adds no work to the kernels themselves).  enable != 0 turns it on
 * and clears the accumulators. */
vdwxc_status vdwxc_enable_timing(vdwxc_handle h, int enable);

/* Synchronise the handle's stream and return, per stage, the summed kernel time in ms and the
 * number of launches since the last enable/read (host arrays of VDWXC_NUM_STAGES entries); the
 * accumulators are then cleared. */
vdwxc_status vdwxc_read_timing(vdwxc_handle h, double* ms, long long* launches);

/* Short name of a stage ("theta_zfwd", "x_contract", ...); "?" if out of range. */
const char* vdwxc_stage_name(int stage);

/* Library version string. */
const char* vdwxc_version(void);

#ifdef __cplusplus
}
#endif

#endif /* VDWXC_GPU_H */
