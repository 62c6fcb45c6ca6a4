/*
 * bpm.h -- C ABI of the MI355X (gfx950) FFT beam-propagation z-march.
 *
 * The library advances the two slowly varying envelopes of a two-beam Bragg
 * problem -- psi~_+ (transmitted band, carrier +h/2) and psi~_- (reflected
 * band, carrier -h/2), Eq. fov7 -- through Nz split steps of length dz,
 * independently for each of Nomega frequency slices of a pulse (Eq. tdp).
 * One step (Eq. fov10 with the Zassenhaus-like factor of Section 2.1) is
 *
 *   a_p = F^-1[ P+(K) F[a] ],  b_p = F^-1[ P-(K) F[b] ],
 *       P+-(K) = exp(i dz sqrt(k^2 - (K +- h/2)^2))          (Eq. fov4)
 *   inside the crystal (Pi = 1):
 *   a' = d0 a_p + d+1 exp(+i h u) b_p,  b' = d0 b_p + d-1 exp(-i h u) a_p
 *   outside (Pi = 0): a' = a_p, b' = b_p,
 *
 * with d0, d+-1 the n = 0, +-1 Jacobi-Anger coefficients of the
 * susceptibility exponential (Eqs. fov9, fov11, fov12, generalised to
 * chih != chihbar; d0 times exp(q/8), q = (k dz)^2 chih chihbar / cos^2 alpha)
 * and u the displacement along h (Eq. Authier, printed sign).
 *
 * Units: SI (metres, radians).  Sample j of a field sits at
 * x_j = (j - Nx/2) dx; row n of u is used by step n (z_n = n dz).
 * k0 = 2 pi / lambda, h = 2 k0 sin(theta_B), k = k0 (1 + delta_w) for slice w,
 * cos(alpha) = sqrt(1 - (h / 2k)^2).
 *
 * Memory: every field pointer is DEVICE memory, row-major [Nomega][Nx],
 * interleaved complex (re, im): complex128 for BPM_PREC_FP64, complex64 for
 * BPM_PREC_FP32 and BPM_PREC_FP32S.  u_field is device float64 [Nz][Nx].
 * The caller owns all field buffers; the plan owns only its constants.
 *
 * Errors: functions return BPM_OK (0) or a negative code and never abort;
 * bpm_last_error() gives a message for the calling thread.  Launches are
 * asynchronous on the given stream (a hipStream_t passed as void*, NULL for
 * the default stream); buffers must stay alive until the stream has
 * completed the work.  Three calls block the host: the first call that uses
 * a plan uploads its constants (hipMalloc and a blocking copy),
 * bpm_batch_create uploads its work lists, and bpm_plan_destroy /
 * bpm_batch_destroy free device memory with hipFree, which waits for the
 * device to finish its outstanding work.
 */
#ifndef BPM_H
#define BPM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct { double re, im; } bpm_complex;
typedef struct bpm_plan bpm_plan;

enum {
  BPM_OK = 0,
  BPM_EINVAL = -1,        /* invalid argument or plan state */
  BPM_ENOMEM = -2,        /* device allocation failed */
  BPM_EHIP = -3,          /* a HIP runtime call or kernel launch failed */
  BPM_EUNSUPPORTED = -4   /* valid but not implemented (size, option) */
};

enum {
  BPM_PREC_FP64 = 0,      /* complex128 fields, FP64 arithmetic throughout */
  BPM_PREC_FP32 = 1,      /* complex64 fields, FP32 FFT butterflies; FP64
                             phases (propagator and deformation reduced mod
                             2 pi in FP64) and FP64 pointwise multiplies */
  BPM_PREC_FP32S = 2      /* complex64 fields and on-chip storage, FP64
                             butterflies and pointwise arithmetic */
};

/* Transform schedules of the march (all give the same result to rounding):
 * STOCKHAM -- radix-R Stockham passes, one work-group barrier per pass;
 * FOURSTEP -- radix-W across the W wavefronts of a slice plus a Stockham
 * transform inside each wavefront, two barriers per z-step;
 * SPLIT -- the two envelopes on separate wavefronts: for Nx = 256 one
 * wavefront per envelope (no forward exchange, one barrier per step), for
 * Nx = 512, 1024 and 2048 FOURSTEP split by envelope in k space (twice the
 * wavefronts, half the registers each) with the x samples shared by all
 * threads, FOURSTEP at Nx = 4096;
 * AUTO -- the library's measured default for (precision, Nx) (currently
 * SPLIT at every size). */
enum { BPM_SCHED_AUTO = -1, BPM_SCHED_STOCKHAM = 0, BPM_SCHED_FOURSTEP = 1,
       BPM_SCHED_SPLIT = 2 };

/* Create a plan for Nomega slices of an Nx-point window (Section 2.1 problem
 * statement: grid dx, step dz, Nz steps, susceptibilities chi0, chih,
 * chihbar, Bragg angle theta_B in radians, wavelength lambda in metres).
 * Nx must be a power of two in [256, 4096]; Nz, Nomega >= 1; dx, dz,
 * lambda > 0; 0 < theta_B < pi/2.  Defaults: precision FP64, crystal slab
 * x >= 0 (x_front = 0, infinite thickness), first-order splitting with the
 * Zassenhaus factor, detuning grid of Nomega cell-centred offsets spanning
 * +-5 Darwin widths |sqrt(chih chihbar)| / sin^2(theta_B) (zero for a
 * single slice).  Returns NULL on invalid input (see bpm_last_error). */
bpm_plan* bpm_plan_create(int Nx, double dx, double dz, int Nz,
                          bpm_complex chi0, bpm_complex chih,
                          bpm_complex chihbar, double theta_B, double lambda,
                          int Nomega);

/* Create a plan on a 3D grid: Ny rows (spacing dy) along y, any Nx along x
 * (the axis of h), marching along z (Section 2.1: the step of Eq. fov4 with
 * both transverse wavenumbers, P+-(Kx, Ky) = exp(i dz sqrt(k^2 -
 * (Kx +- h/2)^2 - Ky^2)); the coupling of Eq. fov10 at every (x, y); the grid
 * of the finite-element example of Section 3.4, 22 x 4267 x 1842, is one).
 * Sample (i, j) sits at y_i = (i - Ny/2) dy, x_j = (j - Nx/2) dx (integer
 * division); the crystal is the slab of bpm_plan_set_crystal for every y.
 * Fields are device [Nomega][Ny][Nx] and u_field device float64
 * [Nz][Ny][Nx].  Nx in [2, 8192]: the propagator step of a row, a cyclic
 * convolution of length Nx, runs on L = Nx for powers of two Nx >= 64, else
 * on the smallest L >= 2 Nx - 1 among the powers of two >= 64 and 4608 =
 * 9 x 512, 9216 = 9 x 1024; Ny in [1, 32]; BPM_PREC_FP64 needs L <= 9216
 * (Nx <= 4608 or a power of two <= 8192; otherwise the propagate returns
 * BPM_EUNSUPPORTED).  On
 * its first propagate the plan builds and keeps on the device FP64 row
 * tables of 32 Nomega (Ny/2 + 1) L bytes (for L != Nx with host FFTs of the
 * device-evaluated propagator, once).  Other arguments and defaults as
 * bpm_plan_create.  A 3D plan supports bpm_propagate, bpm_propagate_ws (the
 * workspace holds the deformation table, as for a 2D plan), the precision,
 * crystal, detuning and time-grid setters (the pulse transforms treat every
 * (y, x) sample as a column; Ny Nx must be even), and the splitting options
 * (orders 1, 2, 4, with or without the Zassenhaus factor; one row-table set
 * per distinct A sub-step length, two for order 4), bpm_deformation_table
 * (Nz Ny Nx cells), bpm_march and bpm_march_segment (which chain bitwise
 * for BPM_PREC_FP64 only: between the two coupling sub-steps at a segment
 * boundary the state is stored in the storage type), and a general crystal
 * mask [Nz][Ny][Nx]; the batch, schedule and no-allocation calls return
 * BPM_EUNSUPPORTED for it.
 * Returns NULL on invalid input. */
bpm_plan* bpm_plan_create_3d(int Nx, int Ny, double dx, double dy, double dz, int Nz,
                             bpm_complex chi0, bpm_complex chih, bpm_complex chihbar,
                             double theta_B, double lambda, int Nomega);

/* Setters: allowed until the plan's first propagate, BPM_EINVAL after. */
int bpm_plan_set_precision(bpm_plan* plan, int precision);
/* Crystal mask Pi_j = [x_front <= x_j < x_front + thickness]; thickness may
 * be +inf.  (Symmetric Bragg slab, Section 2.1.) */
int bpm_plan_set_crystal(bpm_plan* plan, double x_front, double thickness);
/* Relative frequency offsets delta_w of the Nomega slices (host array of
 * Nomega doubles, copied): slice w has the wavenumber k = k0 (1 + delta_w).
 * These are the frequencies omega_i of the independent stationary problems
 * into which Section 3 splits a pulse (Eq. tdp); the default grid is the
 * one described at bpm_plan_create (the paper fixes none).  BPM_EINVAL for a
 * NULL array or an offset that is not finite or is <= -1 (k <= 0). */
int bpm_plan_set_detuning(bpm_plan* plan, const double* delta);
/* General crystal mask Pi(x, z) replacing the slab (asymmetric Bragg, Laue,
 * wedges, any shape in the (x, z) plane): host array [Nz][Nx] of bytes
 * ([Nz][Ny][Nx], Pi(x, y, z), for a 3D plan),
 * nonzero = crystal, row n used by every sub-step of step n; copied into
 * the plan (uploaded to the device once, on first use); NULL returns to the
 * slab of bpm_plan_set_crystal.  Outside the crystal the coupling is the
 * identity (Section 2.1, the susceptibility vanishes in vacuum). */
int bpm_plan_set_mask(bpm_plan* plan, const unsigned char* mask);
/* Pulse grid (Section 3, Eq. tdp): the Nomega slices become the discrete
 * Fourier partners of Nomega time samples t_i = (i - N/2) dt, i.e. slice j
 * gets the detuning delta_j = Omega_j / omega_0 with Omega_j = (j - N/2)
 * 2 pi / (N dt) and omega_0 = 2 pi c / lambda (replaces any detuning set).
 * Needs Nomega a power of two in [256, 4096]; BPM_EINVAL otherwise or for
 * dt <= 0.  Enables bpm_time_to_frequency / bpm_frequency_to_time. */
int bpm_plan_set_time_grid(bpm_plan* plan, double dt);
/* split_order: 1 -- A(dz) B(dz) per step (Eq. fov4); 2 -- B(dz/2) A(dz)
 * B(dz/2); 4 -- B(t dz/2) A(t dz) B((1-t) dz/2) A((1-2t) dz) B((1-t) dz/2)
 * A(t dz) B(t dz/2), t = 1/(2 - 2^(1/3)) (Eq. split-op).  A is the free
 * propagation, B the coupling with the deformation row of the step.  Every
 * schedule and precision supports all three; order 4 costs three transform
 * round trips per step.  zassenhaus: 0 or 1 (the e^{q/8} factor of d0 per B
 * sub-step, end of Section 2.1).  BPM_EINVAL for other values. */
int bpm_plan_set_options(bpm_plan* plan, int split_order, int zassenhaus);

/* Transform schedule (BPM_SCHED_*); default AUTO.  get returns the
 * schedule a propagate would use. */
int bpm_plan_set_schedule(bpm_plan* plan, int schedule);
int bpm_plan_get_schedule(const bpm_plan* plan);

/* Host-only diagnostic: the FP64 constants of slice w for B sub-step 0,
 * out[0..7] = k, cos(alpha), d0.re, d0.im, d+1.re, d+1.im, d-1.re, d-1.im
 * (Section 2.1: cos(alpha) = sqrt(1 - (h/2k)^2), Eqs. fov11, fov12 and the
 * Zassenhaus factor).  Touches no device. */
int bpm_plan_get_constants(const bpm_plan* plan, int w, double* out);

/* Bytes of device workspace a deformed propagate needs: the per-cell
 * deformation-phase table exp(i h u), shared by all slices (Nz Nx cells,
 * Nz Ny Nx for a 3D plan; 16 bytes a cell in FP64, 8 otherwise). */
size_t bpm_workspace_bytes(const bpm_plan* plan);

/* Run the march for all slices: Nz steps of Eq. fov10 (the split step of
 * Eq. fov4 applied to the two envelopes, with the deformation phase of
 * Eq. Authier), each slice an independent stationary problem (Eq. tdp).
 * E0_in: psi~_+ at z = 0, device [Nomega][Nx] (psi~_- starts at zero).
 * u_field: device float64 [Nz][Nx], or NULL (undeformed crystal).  E0_out,
 * Eh_out: device [Nomega][Nx], receive psi~_+ and psi~_- after Nz steps;
 * they must not alias E0_in or each other (BPM_EINVAL).  The caller owns
 * every buffer.  The deformation workspace (bpm_workspace_bytes) is
 * allocated stream-ordered on the stream and released on it (BPM_ENOMEM if
 * that fails); launch failures return BPM_EHIP. */
int bpm_propagate(const bpm_plan* plan, const void* E0_in,
                  const double* u_field, void* E0_out, void* Eh_out,
                  void* stream);

/* As bpm_propagate, with a caller-owned workspace of at least
 * bpm_workspace_bytes(plan) bytes (ignored when u_field is NULL). */
int bpm_propagate_ws(const bpm_plan* plan, const void* E0_in,
                     const double* u_field, void* E0_out, void* Eh_out,
                     void* workspace, void* stream);

/* The two halves of bpm_propagate_ws, for callers that time or schedule
 * them separately.
 * bpm_deformation_table: fill the workspace with exp(i h u) for every cell
 * (Eq. Authier; h u reduced modulo 2 pi in FP64 before an FP32 sincos for
 * the FP32 precisions, FP64 sincos for BPM_PREC_FP64).
 * bpm_march: the Nz-step march of all slices reading that table (or none
 * when table is NULL, i.e. u = 0). */
int bpm_deformation_table(const bpm_plan* plan, const double* u_field,
                          void* workspace, void* stream);
int bpm_march(const bpm_plan* plan, const void* E0_in, const void* table,
              void* E0_out, void* Eh_out, void* stream);

/* One entry of a batch: a plan and its buffers (workspace as in
 * bpm_propagate_ws, required when u_field is not NULL).  Jobs must not share
 * output buffers or workspaces. */
typedef struct {
  const bpm_plan* plan;
  const void* E0_in;
  const double* u_field;
  void* E0_out;
  void* Eh_out;
  void* workspace;
} bpm_job;

typedef struct bpm_batch bpm_batch;

/* Prepare many independent problems (any mix of sizes and precisions, the
 * data-parallel axis of Eq. tdp extended across problems): freezes the
 * plans, splits every job into its frequency slices, groups the slices by
 * (precision, Nx) and assigns each group's slices, longest march first, to
 * the work groups that are resident at once on the device.  Allocates the
 * device work lists (synchronous).  NULL on error. */
bpm_batch* bpm_batch_create(const bpm_job* jobs, int njobs);

/* Enqueue a prepared batch on the stream: one deformation pre-pass per
 * deformed job, then one persistent launch per (precision, Nx) group.
 * Kernel launches only -- no allocation, memset or synchronisation -- so
 * the call may be captured in a hipGraph and replayed.  Every slice runs the
 * same code as bpm_propagate_ws, so results are bitwise identical to running
 * each job alone. */
int bpm_batch_launch(const bpm_batch* batch, void* stream);

/* Diagnostics: persistent launches, slices and work groups of a batch. */
int bpm_batch_info(const bpm_batch* batch, int* n_launches, int* n_slices,
                   int* n_workgroups);

/* Free a prepared batch (hipFree: waits for the device).  NULL is ignored. */
void bpm_batch_destroy(bpm_batch* batch);

/* One-shot batch: create (work lists allocated stream-ordered and filled
 * from host memory the stream releases once copied), launch, and release
 * the work lists on the stream.  Not capturable: BPM_EINVAL while the
 * stream is capturing a graph (a replay would copy from released host
 * memory); capture bpm_batch_launch of a bpm_batch_create batch instead. */
int bpm_propagate_batch(const bpm_job* jobs, int njobs, void* stream);

/* Time <-> frequency transform of a pulse along the slice axis (Section 3,
 * Eq. tdp), on the grid of bpm_plan_set_time_grid:
 *   bpm_time_to_frequency:  psi(Omega_j, x) = dt sum_i psi(t_i, x) exp(+i Omega_j t_i)
 *   bpm_frequency_to_time:  psi(t_i, x) = 1/(N dt) sum_j psi(Omega_j, x) exp(-i Omega_j t_i)
 * (the inverse with dOmega / 2 pi, so the pair is the identity).  Fields are
 * device [Nomega][Nx] interleaved complex of the plan's field type (time or
 * frequency index first); the input may be the output (in place).  A pulse
 * is propagated as bpm_time_to_frequency of the incident envelope,
 * bpm_propagate, then bpm_frequency_to_time of both outputs.  Asynchronous on
 * the stream; BPM_EINVAL for NULL pointers or a plan without a time grid. */
int bpm_time_to_frequency(const bpm_plan* plan, const void* field_t, void* field_w,
                          void* stream);
int bpm_frequency_to_time(const bpm_plan* plan, const void* field_w, void* field_t,
                          void* stream);

/* Segment of the march (checkpoint / resume, z-resolved fields): starting
 * from psi~_+ = E0_in and psi~_- = Eh_in (NULL: zero) at step n0, march
 * steps n0 .. n0+nsteps-1 (deformation table rows n0.., table NULL for
 * u = 0) and write the envelopes after them.  A step depends only on its
 * index, so segments chained through their outputs reproduce bpm_march
 * bitwise for BPM_PREC_FP64 and BPM_PREC_FP32 (register state = storage
 * type).  BPM_PREC_FP32S keeps FP64 registers, so each boundary rounds the
 * state to FP32, after which the chained and monolithic marches round
 * independently and differ at the level of the mode's rounding noise.
 * Outputs may overwrite their own envelope's input (in place);
 * 0 <= n0, n0 + nsteps <= Nz. */
int bpm_march_segment(const bpm_plan* plan, const void* E0_in,
                      const void* Eh_in, const void* table, int n0, int nsteps,
                      void* E0_out, void* Eh_out, void* stream);

/* Bytes of the static device workspace of bpm_propagate_noalloc: 128 MiB,
 * held on every device the library runs on until the process ends. */
#define BPM_NOALLOC_MAX_BYTES (128u << 20)

/* For callers that cannot allocate device memory (code under hipGraph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * march as bpm_propagate, with the same arguments and bitwise the same
 * results, that calls no hipMalloc / hipFree / allocating routine.  Its
 * deformation table -- and the plan's per-slice constants and crystal mask
 * while the plan has not uploaded them itself through an earlier call --
 * live in one static device array of BPM_NOALLOC_MAX_BYTES per device
 * instead: Nz * Nx * (16 for BPM_PREC_FP64, 8 otherwise) bytes of table
 * when u_field is not NULL, plus 208 * Nomega bytes of constants and
 * Nz * Nx bytes of mask when they are staged.  A problem that needs more
 * returns BPM_EINVAL (use bpm_propagate_ws).  Constants and mask are
 * copied from the plan's host memory on the stream, so the plan must stay
 * alive until the stream has completed the call.  Every call on a device
 * shares that device's array, which keeps the last call's contents: calls
 * on one stream are ordered, but calls that overlap on one device (other
 * streams, other threads) race and give wrong results. */
int bpm_propagate_noalloc(const bpm_plan* plan, const void* E0_in,
                          const double* u_field, void* E0_out, void* Eh_out,
                          void* stream);

/* Free a plan and its device constants (hipFree: waits for the device, so
 * work launched with the plan has completed first).  NULL is ignored. */
void bpm_plan_destroy(bpm_plan* plan);

/* Message for the last error on the calling thread ("" if none). */
const char* bpm_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* BPM_H */
