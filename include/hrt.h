/*
 * hrt.h - C ABI of the MI355X (gfx950) hyperbolic Radon transform library.
 *
 * The library evaluates the forward hyperbolic Radon transform of a CMP
 * gather and its exact transpose with the log-polar method of Nikitin,
 * Andersson, Carlsson and Duchkov, "Fast hyperbolic Radon transform
 * represented as convolutions in log-polar coordinates":
 *
 *   forward  R_h f(tau, q) = integral over 0 <= x <= X of
 *                            f(sqrt(tau^2 + q^2 x^2), x) dx     (eq. Rhdef,
 *            one-sided since data exist only for x >= 0), computed as
 *            (t, x) -> (t^2, x^2) resampling with the 1/(2 sqrt y) weight
 *            (eq. f), cubic B-spline smearing onto an equally spaced
 *            log-polar lattice (eq. B3tx2), FFT convolution with the
 *            precomputed kernel spectrum (eqs. finiteconv, lok), and B-spline
 *            interpolation back to (tau, q) (eq. B3tauq);
 *   adjoint  the transpose of that discrete operator, <R f, g> = <f, R* g>
 *            (Section 3, eq. inner), by running the chain in reverse.
 *
 * Grids follow the paper's statement of the problem (Section 2.2, eqs.
 * Rgrid, Qgrid): the gather is sampled regularly on 0 <= t <= T,
 * x0 <= x <= X and is zero outside; the Radon panel is regular in tau and q.
 *
 * Conventions shared by every entry point
 *  - All functions return hrt_status; HRT_OK is 0.  No C++ exception crosses
 *    the ABI.  On failure hrt_last_error() returns a thread-local message.
 *  - Array arguments of the transforms are DEVICE pointers to contiguous
 *    float32 arrays on the device the plan was created on:
 *      data   f[k][j] = f(t_j, x_k),    t_j = j*dt,            x_k = x0 + k*dx
 *      Radon  g[l][i] = g(tau_i, q_l),  tau_i = tau0 + i*dtau, q_l = q0 + l*dq
 *    The caller owns them.  Inputs and outputs must not overlap.
 *  - Units: t, tau, dt, dtau in s; x in km; q in s/km (any consistent units
 *    work: the transform scales with the offset unit).
 *  - hrt_forward / hrt_adjoint / hrt_direct_* only enqueue kernels on the
 *    given HIP stream (NULL = the default stream); they never allocate,
 *    never synchronize the host, and overwrite their output completely.
 *  - A plan may be used by one stream at a time; distinct plans are
 *    independent.  Device faults surface as HRT_ERR_HIP on a later call.
 *  - A NaN or infinity anywhere in a transform's input makes its whole
 *    output NaN (the adjoint's: every sample inside the trapezoid); within
 *    a batch, only the output of the gather that holds it.
 */
#ifndef HRT_H_
#define HRT_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct hrt_plan_s* hrt_plan_t;

typedef enum {
  HRT_OK = 0,
  HRT_ERR_INVALID_ARG = 1, /* null pointer, bad size, bad handle contents   */
  HRT_ERR_GEOMETRY = 2,    /* grids that the method cannot represent        */
  HRT_ERR_OOM = 3,         /* device allocation failed                      */
  HRT_ERR_HIP = 4,         /* a HIP call or kernel launch failed            */
  HRT_ERR_BAD_HANDLE = 5,  /* destroyed or foreign plan handle              */
  HRT_ERR_UNSUPPORTED = 6  /* sizes beyond what the kernels were built for  */
} hrt_status;

/* Grid description (Section 2.2, eqs. Rgrid and Qgrid).
 * Requirements (checked, HRT_ERR_INVALID_ARG otherwise):
 *   nt, nx, ntau, nq >= 4;  dt, dx, dtau, dq > 0;  q0 >= 0;  x0 >= 0;
 *   tau0 >= 0 and tau0 + (ntau-1)*dtau <= (nt-1)*dt;  oversample >= 1.5. */
typedef struct {
  int32_t nt, nx;      /* time samples per trace, number of traces          */
  double dt, x0, dx;   /* t_j = j*dt, x_k = x0 + k*dx                       */
  int32_t ntau, nq;    /* Radon samples: tau_i = tau0 + i*dtau, q_l = q0+l*dq */
  double tau0, dtau, q0, dq;
  double oversample;   /* log-polar oversampling sigma (2.0 is the default) */
  int32_t flags;       /* HRT_TUNE_* bits (0: defaults); others must be 0    */
} hrt_desc;

/* Kernel variants, for tuning (results do not depend on them beyond float32
 * rounding): FFT radices at most 8 along the angle / the log radius (default
 * 16); two columns per workgroup in the column pass (default one); row bands
 * of the spread and gather kernels at most 4 or 2 lattice rows high (default
 * 8, or lower where the LDS needs it; BAND2 wins over BAND4); spread chunks
 * of at most 2560 point entries (default 5120); gather chunks of at most
 * 8192 entries (default 4096). */
#define HRT_TUNE_ROW_RADIX8 1
#define HRT_TUNE_COL_RADIX8 2
#define HRT_TUNE_COL_PAIRS 4
#define HRT_TUNE_BAND4 8
#define HRT_TUNE_BAND2 16
#define HRT_TUNE_SPREAD_HALF 32
#define HRT_TUNE_GATHER_DOUBLE 64
#define HRT_TUNE_MASK 127

/* Behaviour flags (also in hrt_desc.flags):
 * HRT_ACCUMULATE_OUTPUT  hrt_forward, hrt_adjoint, hrt_forward_noalloc and
 *                        the split transforms add their result into the
 *                        output array instead of overwriting it (samples the
 *                        adjoint does not reach are left as they are).
 *                        Refused by hrt_normal and by batches
 *                        (HRT_ERR_INVALID_ARG); the composite entry points
 *                        (ISTA, power iteration, demultiple) always
 *                        overwrite their work arrays.
 * HRT_DETERMINISTIC      accepted, changes nothing: every path already
 *                        gives the same bits on every run (the spread sums
 *                        exactly in integers, every float sum runs in a
 *                        fixed order, no float atomics). */
#define HRT_ACCUMULATE_OUTPUT 256
#define HRT_DETERMINISTIC 512

/* What a plan computed (all host values). */
typedef struct {
  double T, X;                    /* rescaling lengths, eq. hypnorm         */
  double alpha, beta, a, O1, O2;  /* sector and square, Section 2.1         */
  double a_r;                     /* first non-zero log-polar radius        */
  double dtheta0, drho0;          /* eq. lpsamples maxima                   */
  double dtheta, drho, beta_k;    /* lattice spacing, kernel half-width     */
  int32_t m_theta, m_rho;         /* lattice size (angle, log radius)       */
  int32_t k1_kept, k2_kept;       /* non-negative kept frequencies per axis */
  int32_t row_lo, row_hi;         /* lattice rows the data and outputs use  */
  int32_t band_rows, n_bands;     /* row bands of the spread/gather kernels */
  int64_t n_kept;                 /* data samples inside the trapezoid      */
  int64_t workspace_bytes;        /* device memory owned by the plan (0 from
                                     hrt_plan_describe: nothing allocated)  */
  double alg_bytes_fwd;           /* algorithmic HBM bytes of one forward   */
  double alg_bytes_adj;           /* ... and of one adjoint                 */
} hrt_info;

/* Geometry and sizes only: the plan's host computation (rescaling, sector
 * placement, lattice spacing, row bands) with no GPU call.  Usable on a
 * machine without a GPU.  Returns HRT_ERR_INVALID_ARG for bad grids. */
hrt_status hrt_plan_describe(const hrt_desc* desc, hrt_info* out);

/* Build a plan on the current HIP device: the host geometry, the kernel
 * spectrum of eq. finiteconv evaluated by Gauss-Legendre quadrature in
 * float64 on the device, the per-trace and per-slowness tables, and all
 * device workspace.  Synchronizes the device once.  *out receives the
 * handle, to be released with hrt_plan_destroy. */
hrt_status hrt_plan_create(const hrt_desc* desc, hrt_plan_t* out);

/* Forward transform g = R_h f: f is float32[nx][nt], g is float32[nq][ntau],
 * both device pointers.  `stream` is a hipStream_t (NULL = default). */
hrt_status hrt_forward(hrt_plan_t plan, const float* f, float* g,
                       void* stream);

/* Adjoint transform f = R_h^T g (exact transpose of hrt_forward up to
 * float32 rounding): g is float32[nq][ntau], f is float32[nx][nt]; samples
 * outside the trapezoid t >= q0*x are set to zero. */
hrt_status hrt_adjoint(hrt_plan_t plan, const float* g, float* f,
                       void* stream);

/* hrt_forward for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same kernels and the same result, bit for bit, as hrt_forward, but
 * the per-call workspace (half spectrum, spread partial rows, real lattice
 * rows, input maxima) is taken from a fixed 64 MiB array in device memory
 * that each GPU the library runs on holds until the process ends, instead
 * of the plan's own.  It calls no allocator.  Every call on one GPU shares
 * that GPU's array, so calls that overlap on a GPU (concurrent streams,
 * threads) race and must be serialised by the caller; a call leaves its
 * workspace contents behind, and no call depends on what an earlier one
 * left.  Same arrays and stream rules as hrt_forward.  Returns
 * HRT_ERR_UNSUPPORTED, before any launch, for a plan whose forward
 * workspace exceeds 64 MiB (the C3 grid, 2048 x 1024 -> 2048 x 1024, needs
 * about 47 MB). */
hrt_status hrt_forward_noalloc(hrt_plan_t plan, const float* f, float* g, void* stream);

/* Normal operator: g = R_h f, then fa = R_h^T g (the forward followed by the
 * adjoint of its output, as in the power iteration for ||R_h||^2 and in the
 * iterative schemes of Section 3, which apply both operators in turn).
 * f and fa are float32[nx][nt], g is
 * float32[nq][ntau], all device pointers; both outputs are written and are
 * bit-identical to hrt_forward(f -> g) followed by hrt_adjoint(g -> fa).
 * One launch fewer than the two calls: the forward's last kernel also
 * records the largest |g| that the adjoint's fixed-point scale needs.
 * g must not overlap f or fa; fa may be f itself (f is read only before fa
 * is written).  Same stream rules as hrt_forward; HRT_ERR_INVALID_ARG for a
 * null or overlapping array. */
hrt_status hrt_normal(hrt_plan_t plan, const float* f, float* g, float* fa,
                      void* stream);

/* Reference method of Section 5: direct summation over hyperbolas with
 * Keys cubic interpolation in time and the trapezoid rule in offset, in
 * float32 on the GPU (forward), and its exact transpose (adjoint).  Same
 * arrays and stream rules as hrt_forward / hrt_adjoint. */
hrt_status hrt_direct_forward(hrt_plan_t plan, const float* f, float* g,
                              void* stream);
hrt_status hrt_direct_adjoint(hrt_plan_t plan, const float* g, float* f,
                              void* stream);

/* Soft-thresholding iterations for sparse Radon representations and trace
 * interpolation (Section 3, eq. itersmd):
 *   g <- S_{c2 mu}(g + c2 R_h(f - chi_S R_h^T g)),
 * S_mu(v) = v - mu/2 for v >= mu/2, 0 for |v| < mu/2, v + mu/2 for
 * v <= -mu/2.  f float32[nx][nt] is the recorded gather (0 where traces are
 * missing); mask float32[nx][nt] is chi_S (1 where recorded, 0 where missing;
 * NULL: everything recorded, which is eq. iters); g float32[nq][ntau] is the
 * Radon panel, updated in place `iters` times.  work_data float32[nx][nt] and
 * work_radon float32[nq][ntau] are caller-owned scratch.  c2 > 0 is the step
 * c^2 (convergence needs c2 * ||R_h||^2 < 1, see hrt_opnorm2), mu >= 0 the
 * sparsity weight.  Enqueues only (no allocation, no host synchronization),
 * so it may be captured in a HIP graph.  All arrays device pointers; none
 * may overlap another. */
hrt_status hrt_ista_iterate(hrt_plan_t plan, const float* f, const float* mask, float* g,
                            float* work_data, float* work_radon, int32_t iters, float c2,
                            float mu, void* stream);

/* The same iterations captured once into an executable HIP graph (the
 * arrays are bound at capture; replays reuse them).  Allocates the graph;
 * launch with hrt_graph_launch on any stream, release with
 * hrt_graph_destroy.  Not while a profile (hrt_profile_begin) is active. */
typedef struct hrt_graph_s* hrt_graph_t;
hrt_status hrt_ista_graph_create(hrt_plan_t plan, const float* f, const float* mask,
                                 float* g, float* work_data, float* work_radon,
                                 int32_t iters, float c2, float mu, hrt_graph_t* out);
hrt_status hrt_graph_launch(hrt_graph_t graph, void* stream);
void hrt_graph_destroy(hrt_graph_t graph);

/* ||R_h||^2, the largest eigenvalue of R_h^T R_h, by `iters` steps of the
 * power iteration from a start vector drawn from `seed` (splitmix64,
 * uniform in [-1, 1)): v <- R^T R v / ||R^T R v||, estimate <v, R^T R v>
 * with |v| = 1.  The operators run in float32, every inner product and norm
 * is accumulated in float64.  work_data, work_data2 float32[nx][nt] and
 * work_radon float32[nq][ntau] are caller-owned scratch.  Synchronizes the
 * stream at every step; writes the estimate to *out (host). */
hrt_status hrt_opnorm2(hrt_plan_t plan, int32_t iters, uint64_t seed, float* work_data,
                       float* work_data2, float* work_radon, double* out, void* stream);

/* Multiple attenuation in the Radon domain (Section 6): given the gather f
 * float32[nx][nt] and a (sparse) Radon panel g float32[nq][ntau] of it, for
 * instance from hrt_ista_iterate, keep the multiples' part of the panel,
 * the samples with q_l > qb0 + qb_slope * tau_i (slower moveout than the
 * border line; the decision in float64, q_l = q0 + l dq, tau_i = tau0 +
 * i dtau), take it back to the gather with the adjoint, and subtract:
 *   out = f - R_h^T (g restricted to the multiples' side).
 * out float32[nx][nt] receives the primaries; work_radon float32[nq][ntau]
 * is caller-owned scratch.  Enqueues only; arrays must not overlap (f and g
 * may be read-only). */
hrt_status hrt_demultiple(hrt_plan_t plan, const float* f, const float* g, double qb0,
                          double qb_slope, float* out, float* work_radon, void* stream);

/* Uneven batches: n gathers of different grids transformed by one launch
 * per kernel for the whole batch (every kernel's work items cover all
 * gathers, largest gathers first), so that small gathers fill the GPU
 * together.  hrt_batch_create builds one plan per description (as
 * hrt_plan_create) and the batch tables; the batch owns its plans.  Arrays
 * are packed: gather i's data f_i[nx_i][nt_i] starts at f + data_off[i] and
 * its Radon panel at g + radon_off[i] (offsets in floats, from
 * hrt_batch_offsets, n + 1 entries each, the last being the total).  The
 * batch calls enqueue only; the member plans' workspaces are shared with
 * them, so a batch and its plans must not run concurrently. */
typedef struct hrt_batch_s* hrt_batch_t;
hrt_status hrt_batch_create(const hrt_desc* descs, int32_t n, hrt_batch_t* out);
hrt_status hrt_batch_offsets(hrt_batch_t batch, int64_t* data_off, int64_t* radon_off);
hrt_status hrt_batch_forward(hrt_batch_t batch, const float* f_packed, float* g_packed,
                             void* stream);
hrt_status hrt_batch_adjoint(hrt_batch_t batch, const float* g_packed, float* f_packed,
                             void* stream);
/* The plan of gather i (owned by the batch; do not destroy it). */
hrt_status hrt_batch_plan(hrt_batch_t batch, int32_t i, hrt_plan_t* out);
void hrt_batch_destroy(hrt_batch_t batch);

/* Soft-thresholding iterations (Section 3, eq. itersmd, as
 * hrt_ista_iterate) for every gather of a batch at once: per iteration one
 * batched adjoint, the residual over all packed samples, one batched
 * forward and the update g_i <- S_{c2_i mu_i}(g_i + c2_i d_i), each gather
 * with its own step c2[i] > 0 and weight mu[i] >= 0 (host arrays of n
 * floats).  f, mask (NULL: every sample recorded) and work_data are packed
 * data arrays, g and work_radon packed Radon arrays (hrt_batch_offsets);
 * they must not overlap.  hrt_batch_ista_iterate enqueues (after a small
 * host-to-device copy of the per-gather parameters into the batch);
 * hrt_batch_ista_graph_create captures the same work into a HIP graph that
 * keeps its own copy of the parameters (launch with hrt_graph_launch). */
hrt_status hrt_batch_ista_iterate(hrt_batch_t batch, const float* f, const float* mask,
                                  float* g, float* work_data, float* work_radon,
                                  int32_t iters, const float* c2, const float* mu,
                                  void* stream);
hrt_status hrt_batch_ista_graph_create(hrt_batch_t batch, const float* f, const float* mask,
                                       float* g, float* work_data, float* work_radon,
                                       int32_t iters, const float* c2, const float* mu,
                                       hrt_graph_t* out);

/* Splitting into parts (Section 4, eq. tsplit: the integral over t cut at
 * intermediate times, so that each part gets the log-polar lattice its own
 * samples need; Section 5 applies the same to the slowness range).  The
 * time samples are cut into n_t bands [t_edges[it], t_edges[it+1]) and the
 * slowness rows into n_q bands [q_edges[iq], q_edges[iq+1]) (edges strictly
 * increasing, t_edges[0] = 0, t_edges[n_t] = nt, q_edges[0] = 0,
 * q_edges[n_q] = nq; 1 to 64 bands per axis).  Part iq*n_t + it is a plain
 * problem of its own, rescaled by its own T and X (eq. hypnorm):
 *   data   t_j, j < nt_p = min(nt, t_edges[it+1] + 2), only the samples of
 *          its time band taken in; the traces with a kept sample in the band
 *          (j dt >= q0_p x_k, q0_p = q0 + q_edges[iq] dq) plus one;
 *   Radon  slowness rows of its band, tau_i <= (nt_p - 1) dt.
 * The split transform is the sum of the parts' transforms, each placed in
 * the whole arrays f float32[nx][nt] and g float32[nq][ntau]; a part's
 * adjoint is its exact transpose, so the split adjoint is the transpose of
 * the split forward.  One band per axis gives the plain transform.
 * A part without a kept sample or a Radon sample is an error
 * (HRT_ERR_INVALID_ARG), as is a part whose grids a plain plan rejects.
 *
 * hrt_split_describe: host only, no GPU; part `part`'s grid description
 * (sub_out), its time band and slowness rows (window_out[4] = j_lo, j_hi,
 * l_lo, l_hi) and its summary (info_out, computed only when non-null).
 * hrt_split_create: one plan per part (as hrt_plan_create; the split owns
 * them).  hrt_split_forward / hrt_split_adjoint enqueue the parts one after
 * another on `stream` (every output sample is stored by one part and added
 * to by the others); inputs and outputs must not overlap.  Calls on one
 * split must not run concurrently. */
typedef struct hrt_split_s* hrt_split_t;
hrt_status hrt_split_describe(const hrt_desc* desc, int32_t n_t, const int32_t* t_edges,
                              int32_t n_q, const int32_t* q_edges, int32_t part,
                              hrt_desc* sub_out, int32_t* window_out, hrt_info* info_out);
hrt_status hrt_split_create(const hrt_desc* desc, int32_t n_t, const int32_t* t_edges,
                            int32_t n_q, const int32_t* q_edges, hrt_split_t* out);
hrt_status hrt_split_forward(hrt_split_t split, const float* f, float* g, void* stream);
hrt_status hrt_split_adjoint(hrt_split_t split, const float* g, float* f, void* stream);
/* Copy of part `part`'s summary. */
hrt_status hrt_split_query(hrt_split_t split, int32_t part, hrt_info* out);
void hrt_split_destroy(hrt_split_t split);

/* Copy of the plan's summary. */
hrt_status hrt_query(hrt_plan_t plan, hrt_info* out);

/* Copy the kernel multiplier K[k1][k2] (k1 < k1_kept, 0 <= k2 < k2_kept,
 * complex as two floats, unnormalised: zeta^/(dtheta drho b^2 b^2) of
 * eq. B3tauq) to host memory `host_out` of 2*k1_kept*k2_kept floats.
 * Synchronizes the device. */
hrt_status hrt_plan_kernel(hrt_plan_t plan, float* host_out);

/* Per-kernel timing for measurement tools.  hrt_profile_begin creates
 * 2*max_records HIP events (the only allocation; none happens later) and
 * from then on hrt_forward / hrt_adjoint / hrt_normal record an event on
 * the launch stream before and after each of their kernels, until
 * max_records kernels have been recorded.  hrt_profile_end synchronizes on
 * the recorded events, writes the summed milliseconds and the launch count
 * per kernel into ms_sum[HRT_PROFILE_SLOTS] and count[HRT_PROFILE_SLOTS]
 * (order: forward input maximum, spread, row FFT, column pass, row inverse
 * FFT, gather, then the same six of the adjoint; hrt_normal launches no
 * adjoint input maximum) and releases the events.  Either output may be
 * NULL. */
#define HRT_PROFILE_SLOTS 12
hrt_status hrt_profile_begin(hrt_plan_t plan, int32_t max_records);
hrt_status hrt_profile_end(hrt_plan_t plan, double* ms_sum, int64_t* count);

/* Release a plan and its device memory.  NULL is ignored. */
void hrt_plan_destroy(hrt_plan_t plan);

const char* hrt_status_string(hrt_status s);
const char* hrt_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* HRT_H_ */
