/*
 * prism.h - C ABI of the MI355X PRISM / multislice STEM library (libprism).
 *
 * Method: C. Ophus, "A Fast Image Simulation Algorithm for Scanning
 * Transmission Electron Microscopy" (arXiv:1702.01904).
 *
 * Conventions shared by every entry point
 *   - Arrays are row-major and indexed [y][x]; pixel (i, j) of an n x n grid
 *     sits at (i d/n, j d/n) for a square cell of side d (Angstrom).
 *   - "dev" pointers are HIP device pointers owned by the caller; "host"
 *     pointers are read during the call only (or copied into the plan).
 *   - The library never allocates device memory. Every device buffer it
 *     needs beyond inputs and outputs comes from a caller-supplied workspace
 *     whose minimum size the *_workspace_bytes queries return.
 *   - Compute entry points are asynchronous on the given HIP stream (pass a
 *     hipStream_t cast to void*, or NULL for the default stream). Device
 *     faults surface at the caller's next synchronisation.
 *   - Every call returns PRISM_OK (0) or a negative status. All argument
 *     checks run on the host before anything is enqueued. prism_last_error()
 *     returns a thread-local message for the last failing call.
 *   - Complex values are interleaved float pairs (re, im) ("c64").
 *   - A plan fills host-side caches (beam sets, aperture rows, detector pixel
 *     lists) on first use and never rewrites an entry: calls on one plan
 *     from several host threads at once must be serialised by the caller;
 *     different plans are independent.
 *   - Every call that takes an S-matrix pointer also takes the byte size of
 *     the caller's buffer and rejects one smaller than prism_smatrix_bytes
 *     for its f and alpha_max (PRISM_EINVAL), so no kernel can read or write
 *     past it.
 *   - The anti-aliasing aperture is the paper's half of the maximum
 *     frequency (compact S-matrix paragraph of "The PRISM Algorithm"):
 *     kx^2 + ky^2 < (n/4)^2. It is not a parameter: the quarter-size
 *     S-matrix and the window side W = n / (2 f) follow from it, and a
 *     wider band would no longer fit the n/2 x n/2 storage.
 *
 * Limits of this implementation: n is 2^k, 3 * 2^k or 9 * 2^k in
 * [128, 2048] (128, 192, 256, 384, 512, 576, 768, 1024, 1152, 1536, 2048);
 * the PRISM window side W = n / (2 f) is a power of two in [8, 256] or one
 * of 12, 18, 24, 36, 48, 72, 96, 144, 192; at most PRISM_MAX_DET detector
 * bins.
 */
#ifndef PRISM_H
#define PRISM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define PRISM_OK 0
#define PRISM_EINVAL (-1)     /* bad argument, shape or unsupported size       */
#define PRISM_ENOSPACE (-2)   /* workspace smaller than the minimum required   */
#define PRISM_EHIP (-3)       /* HIP launch/API error (text in last_error)     */
#define PRISM_ENOTREADY (-4)  /* potential slices not set                      */

#define PRISM_MAX_DET 32

/* Operand precision of the PRISM window sum (Eq. PRISMfinal). */
#define PRISM_PREC_FP32 0 /* FP32 operands, FP32 accumulation (default)        */
#define PRISM_PREC_BF16 1 /* bfloat16 S-matrix and coefficients, FP32 accumulation */
#define PRISM_PREC_FP16 2 /* float16 S-matrix and coefficients, FP32 accumulation  */

typedef struct prism_plan prism_plan; /* opaque, host-side state only */

/* Sampling of the specimen (Fig. 1a-b: slices and their projected
 * potentials). slice_thickness_A is copied at plan creation. */
typedef struct {
  int n;                           /* grid side in pixels (fine grid)        */
  double cell_A;                   /* square cell side d in Angstrom         */
  double energy_keV;               /* beam kinetic energy                    */
  int n_slices;                    /* H                                      */
  const double* slice_thickness_A; /* host [n_slices], t_p in Angstrom       */
} prism_geometry;

/* Probe-forming optics: hard aperture of semi-angle alpha (aperture
 * equation) and aberration phase chi = pi lambda q^2 C1 +
 * (pi/2) lambda^3 q^4 C3 (chi equation). Probe tilt (theta_x, theta_y):
 * aperture and chi are centred on q_t = theta / lambda, and the position
 * term of the coefficient equation uses r0 - h tan(theta) with h the total
 * slice thickness, so that the exit probe is centred on r0. Zero tilt is the
 * untilted probe. */
typedef struct {
  double alpha_mrad;
  double C1_A;
  double C3_A;
  double tilt_x_mrad;
  double tilt_y_mrad;
} prism_optics;

/* Virtual detectors (Fig. 1f): bin j collects the intensity at angles
 * edges[2j] <= theta < edges[2j+1] (mrad), theta = lambda |q|. */
typedef struct {
  int n_det;                  /* 1 .. PRISM_MAX_DET                         */
  const double* edges_mrad;   /* host [n_det][2]                            */
} prism_detector;

/* Create a plan for one grid/cell/energy/slicing. Returns PRISM_EINVAL for
 * n outside the supported sizes, non-positive cell, energy or thickness. */
int prism_plan_create(prism_plan** out, const prism_geometry* geometry);
void prism_plan_destroy(prism_plan* plan);

/* Relativistic electron wavelength (Angstrom) used by the plan. */
int prism_wavelength(const prism_plan* plan, double* lambda_A);

/* The paper's choice of the beam-set limit ("The PRISM Algorithm", the
 * paragraph on alpha_max): the largest probe semi-angle plus one
 * interpolated beam spacing, alpha_max = alpha + f lambda dq (mrad), so
 * that the set covers the aperture with a margin of one beam.
 * Errors: PRISM_EINVAL for a null pointer, f < 1, n % (2 f) != 0, or alpha
 * not positive and finite. */
int prism_alpha_max(const prism_plan* plan, int f, double alpha_mrad, double* alpha_max_mrad);

/* PRISM beam set (the plane-wave initial conditions): integer pairs (m, n)
 * with sqrt(m^2+n^2) f lambda dq <= alpha_max and (m f)^2 + (n f)^2 <
 * (n/4)^2 so that each survives the half-band anti-aliasing aperture, in
 * lexicographic (m, n) order. alpha_max_mrad must be positive (the paper's
 * rule: prism_alpha_max). Requires n % (2 f) == 0. */
int prism_beam_count(const prism_plan* plan, int f, double alpha_max_mrad, int* n_beams);
/* Writes min(count, capacity) pairs to mn (host [capacity][2]). */
int prism_beams(const prism_plan* plan, int f, double alpha_max_mrad, int32_t* mn, int capacity);

/* Number B_A of beams of the set inside the probe aperture (the beams whose
 * coefficient is non-zero; the probe step sums only these, as the paper's
 * discussion of skipping zero coefficients allows). Aperture test as in
 * prism_optics. Errors: those of prism_beam_count and the optics checks of
 * the probe step. */
int prism_active_beam_count(const prism_plan* plan, int f, double alpha_max_mrad,
                            const prism_optics* optics, int* n_active);

/* Bytes of the compact S-matrix: c64 [B][n/2][n/2] (quarter-size storage
 * enabled by the half-angle anti-aliasing aperture). */
int prism_smatrix_bytes(const prism_plan* plan, int f, double alpha_max_mrad, size_t* bytes);

/* Workspace sizes. *_min_bytes is the smallest accepted workspace; larger
 * workspaces let the library process more beams / probes per launch up to
 * the preferred size returned by *_workspace_bytes. */
int prism_build_workspace_bytes(const prism_plan* plan, int f, double alpha_max_mrad,
                                size_t* preferred, size_t* minimum);
int prism_multislice_workspace_bytes(const prism_plan* plan, int n_det, size_t* preferred,
                                     size_t* minimum);
int prism_probe_workspace_bytes(const prism_plan* plan, int f, double alpha_max_mrad,
                                const prism_optics* optics, size_t* preferred, size_t* minimum);

/* Number of consecutive probes the PRISM probe step treats as one tile.
 * Probes whose windows overlap (e.g. a gx x gy patch of a raster scan)
 * should be adjacent in the probe list: a tile shares one union window, so
 * scattered tiles cost more but still give the same results. */
int prism_probe_group(const prism_plan* plan, int f, int* group, int* tile_x, int* tile_y);

/* A processing order for scattered probe positions: perm (host int32 [P])
 * such that probe_xy[perm[0]], probe_xy[perm[1]], ... visits the probes in
 * spatially compact runs, so that consecutive probes share union windows.
 * Probes are sorted by the Morton index of their window centre pixel (the
 * centre of Eq. RegionBounds) on cells of min(16, W/8) S-matrix pixels, ties
 * in input order; a raster at two S-pixels per step comes out in 8 x 8
 * tiles. probe_xy_host: float64 [P][2] (Angstrom), read during the call.
 * Results of the probe step do not depend on the order, only its time.
 * Errors: PRISM_EINVAL (null pointers, P < 0, invalid f). */
int prism_probe_order(const prism_plan* plan, int f, const double* probe_xy_host, int n_probes,
                      int32_t* perm);

/* Select the operand precision of prism_probe_outputs for this plan
 * (PRISM_PREC_*; PRISM_EINVAL otherwise). With BF16/FP16 each call first
 * packs the active beams of the S-matrix into a pixel-major 16-bit copy in
 * the workspace (each beam scaled by an exact power of two so that its
 * largest component is below 1, the coefficient divided by the same factor)
 * and runs the window sum on 16-bit matrix cores with FP32 accumulation;
 * everything after the window sum stays FP32/FP64. The workspace sizes
 * returned by prism_probe_workspace_bytes follow the plan's precision, so
 * query them after this call. Setting the precision is not stream-ordered:
 * do it between calls. */
int prism_set_probe_precision(prism_plan* plan, int precision);

/* Record the projected phase sigma V_p of every slice (Eq. 4): device
 * float32 [n_slices][n][n], radians. The pointer is BORROWED: it must stay
 * valid and unchanged until the stream has passed the last build or
 * multislice call that reads it. Nothing is copied. */
int prism_set_potential_slices(prism_plan* plan, const float* phase_dev);

/* Fig. 1c: multislice every beam of the set through all slices (Eq. 5 with
 * the half-band aperture in the propagator) and store each exit wave at
 * quarter size: smatrix_dev c64 [B][n/2][n/2], S(i', j') = psi_exit(2i', 2j'),
 * smatrix_bytes the size of that buffer (at least prism_smatrix_bytes).
 * ws/ws_bytes: device workspace, at least the build minimum. */
int prism_build_smatrix(prism_plan* plan, int f, double alpha_max_mrad, void* smatrix_dev,
                        size_t smatrix_bytes, void* ws, size_t ws_bytes, void* stream);

/* Batched S-matrix build (Fig. 1c for several specimens at once). Each item
 * names a plan (its geometry and potential slices, set as for
 * prism_build_smatrix), an interpolation factor, an alpha_max and the
 * item's output S-matrix (c64 [B][n/2][n/2]) with the byte size of its
 * buffer (at least prism_smatrix_bytes).
 * Items whose plans share the grid, cell, energy and the thicknesses of their
 * common slices form one group: the waves of all their beams run through the
 * same launches, slice by slice, each wave multiplying by its own specimen's
 * transmission (specimens with fewer slices drop out of later launches);
 * groups run one after another. An item with at least four such launches'
 * worth of beams gains nothing from sharing and is built on its own (as
 * prism_build_smatrix, with its plan's launch shapes). The results equal
 * prism_build_smatrix of each item alone, bit for bit.
 * Workspace (prism_build_batch_workspace_bytes): per group the
 * transmissions of every member (sum of H n^2 complex64), the beam lists and
 * up to 256 MiB of wave state per launch (larger launches lose the cache
 * reuse of the transmissions); the minimum holds one wave of state.
 * Errors: PRISM_EINVAL (null or invalid item, negative count), the checks of
 * prism_build_smatrix for every item (message prefixed by the item index),
 * PRISM_ENOSPACE, PRISM_EHIP. count == 0 is a no-op. The plans must not be
 * used concurrently on other streams while the batch is in flight. */
typedef struct {
  prism_plan* plan;
  int f;
  double alpha_max_mrad;
  void* smatrix_dev;
  size_t smatrix_bytes;
} prism_build_item;

int prism_build_batch_workspace_bytes(const prism_build_item* items, int count,
                                      size_t* preferred, size_t* minimum);
int prism_build_smatrix_batch(const prism_build_item* items, int count, void* ws,
                              size_t ws_bytes, void* stream);

/* Fig. 1d-f: for each probe position r0 (probe_xy_dev float64 [P][2],
 * Angstrom) sum the A = 1 beams of the S-matrix, weighted by
 * alpha_{m,n}(r0) = A e^{-i chi} e^{-2 pi i q.r0} / (W sqrt(B_A)), over the
 * W x W window of Eq. RegionBounds (centre pixel floor(x0/dx_S + 1/2),
 * periodic wrap), Fourier transform, and integrate |Psi|^2 / W^2 over each
 * detector bin: out_dev float64 [P][n_det]. The S-matrix (smatrix_bytes: the
 * size of its buffer) must come from prism_build_smatrix with the same f and
 * alpha_max_mrad, and the probe
 * semi-angle plus the tilt magnitude may not exceed alpha_max_mrad
 * (PRISM_EINVAL): every beam inside the aperture must be in the set. Several optics (defocus, C3, semi-angle)
 * can be evaluated on one resident S-matrix. */
int prism_probe_outputs(prism_plan* plan, int f, double alpha_max_mrad, const void* smatrix_dev,
                        size_t smatrix_bytes, const double* probe_xy_dev, int n_probes,
                        const prism_optics* optics, const prism_detector* detector,
                        double* out_dev, void* ws, size_t ws_bytes, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc):
 * prism_probe_outputs with no workspace argument. Its scratch is a
 * library-held device array of PRISM_NOALLOC_SCRATCH_BYTES per GPU, part of
 * the library's code object (each GPU the library runs on holds one until
 * the process ends). Results equal prism_probe_outputs'.
 * Limit: PRISM_ENOSPACE, before anything is enqueued, when the probe step's
 * minimum workspace (prism_probe_workspace_bytes) exceeds the array, e.g.
 * 305 active beams on a 512^2 S-matrix (649 MiB in FP32, 329 MiB in BF16);
 * 69 active beams at 512^2 need 193 MiB. Other errors as
 * prism_probe_outputs.
 * Every call on one GPU shares that GPU's array, and it keeps the last
 * call's contents: calls that overlap on one GPU (other streams, other host
 * threads) race and must be ordered by the caller. Nothing in the array has
 * to start at zero: each call writes every scratch value it reads. */
#define PRISM_NOALLOC_SCRATCH_BYTES ((size_t)256 << 20)
int prism_probe_outputs_noalloc(prism_plan* plan, int f, double alpha_max_mrad,
                                const void* smatrix_dev, size_t smatrix_bytes,
                                const double* probe_xy_dev, int n_probes,
                                const prism_optics* optics, const prism_detector* detector,
                                double* out_dev, void* stream);

/* The same probe step with the full diffraction pattern as output (Fig. 1f:
 * the CBED alternative to virtual detectors): cbed_dev float32 [P][W][W],
 * I(kw) = |FFT_W psi|^2 / W^2 with both axes in W-point fftfreq order (window
 * frequency kw sits at full-grid frequency f kw). Workspace, precision and
 * errors as prism_probe_outputs; PRISM_EINVAL for a null cbed_dev. */
int prism_probe_cbed(prism_plan* plan, int f, double alpha_max_mrad, const void* smatrix_dev,
                     size_t smatrix_bytes, const double* probe_xy_dev, int n_probes,
                     const prism_optics* optics, float* cbed_dev, void* ws, size_t ws_bytes,
                     void* stream);

/* The probe step (Fig. 1d-f, Eqs. RegionBounds and PRISMfinal) for several
 * requests in one call: each request is the work of one prism_probe_outputs
 * (detector != NULL) or prism_probe_cbed (detector == NULL) call, or of
 * their _accumulate forms (accumulate != 0: out += weight * result), with
 * its own plan, f, alpha_max, S-matrix, positions, optics and outputs; the
 * optics and detector edges are read during the call. Results equal those
 * of the separate calls bit for bit. Requests whose plans give the same
 * window side n/(2f), probe group, window tiles (prism_tuning) and operand
 * precision, and that ask for the same output kind, share each chunk's
 * window-sum and window-transform launches (several specimens in one
 * launch); each distinct (S-matrix, active beam set) is packed once per
 * workspace fill. Requests of one batch must write disjoint outputs. All
 * plans must be on the device of the stream; none of them may be used
 * concurrently on another stream while the batch is in flight.
 * Workspace: prism_probe_batch_workspace_bytes gives the size that runs
 * each launch class in one fill (preferred) and the size of the largest
 * single request's minimum (minimum); with less than preferred the call
 * runs the requests in several fills, in order.
 * Errors: PRISM_EINVAL (null or invalid request, negative count; the checks
 * of the single calls, message prefixed by the request index), then
 * PRISM_ENOSPACE, PRISM_EHIP. Every request is checked before anything is
 * enqueued. count == 0 is a no-op. */
typedef struct {
  prism_plan* plan;
  int f;
  double alpha_max_mrad;
  const void* smatrix_dev;
  size_t smatrix_bytes;
  const double* probe_xy_dev;      /* [n_probes][2], Angstrom            */
  int n_probes;
  const prism_optics* optics;
  const prism_detector* detector;  /* NULL: full CBED output             */
  double* out_dev;                 /* detector: float64 [n_probes][n_det] */
  float* cbed_dev;                 /* CBED: float32 [n_probes][W][W]      */
  int accumulate;                  /* 0: store; 1: add weight * result   */
  double weight;
} prism_probe_request;

/* Launch class of the probe step for (plan, f): requests of one
 * prism_probe_batch call with equal keys and the same output kind share
 * their window-sum and window launches (the key encodes the window side,
 * probe group, window tiles and operand precision; its value has no other
 * meaning). Errors: PRISM_EINVAL for an invalid f or window side. */
int prism_probe_class(const prism_plan* plan, int f, unsigned long long* key);
int prism_probe_batch_workspace_bytes(const prism_probe_request* requests, int count,
                                      size_t* preferred, size_t* minimum);
int prism_probe_batch(const prism_probe_request* requests, int count, void* ws,
                      size_t ws_bytes, void* stream);

/* Conventional multislice STEM (Eq. 5 run once per probe): incident probe
 * iFFT[A e^{-i chi} e^{-2 pi i q.r0}] n / sqrt(N_A) (tilt as in prism_optics),
 * H slice steps,
 * I = |FFT psi_H|^2 / n^2 integrated per detector bin: out_dev float64
 * [P][n_det]. */
int prism_multislice_outputs(prism_plan* plan, const double* probe_xy_dev, int n_probes,
                             const prism_optics* optics, const prism_detector* detector,
                             double* out_dev, void* ws, size_t ws_bytes, void* stream);

/* Frozen-phonon averaging ("Simulation and Analysis Implementation": the
 * calculation is repeated for several configurations of randomly displaced
 * atoms and the intensities are summed incoherently). The _accumulate forms
 * run the same computation as the call they extend but store
 *     out[i] = out[i] + weight * result[i]
 * instead of overwriting: with one S-matrix (or one set of potential slices)
 * per configuration and weight = 1/K, K calls into the same output leave the
 * configuration average, with no extra buffer. The caller initialises the
 * output (e.g. with zeros or with a first non-accumulating call). Each output
 * element is read and written by one thread of one kernel, so the sum is
 * formed in call order; FP64 for detector sums, the FP32 value of each term
 * for CBED (the sum is formed in FP64 per term, then rounded to FP32).
 * Errors: those of the extended call, and PRISM_EINVAL for a weight that is
 * not finite. Calls that accumulate into the same output must be ordered
 * (same stream or events). */
int prism_probe_outputs_accumulate(prism_plan* plan, int f, double alpha_max_mrad,
                                   const void* smatrix_dev, size_t smatrix_bytes,
                                   const double* probe_xy_dev, int n_probes,
                                   const prism_optics* optics,
                                   const prism_detector* detector, double weight,
                                   double* out_dev, void* ws, size_t ws_bytes, void* stream);
int prism_probe_cbed_accumulate(prism_plan* plan, int f, double alpha_max_mrad,
                                const void* smatrix_dev, size_t smatrix_bytes,
                                const double* probe_xy_dev, int n_probes,
                                const prism_optics* optics, double weight,
                                float* cbed_dev, void* ws, size_t ws_bytes, void* stream);
int prism_multislice_outputs_accumulate(prism_plan* plan, const double* probe_xy_dev,
                                        int n_probes, const prism_optics* optics,
                                        const prism_detector* detector, double weight,
                                        double* out_dev, void* ws, size_t ws_bytes,
                                        void* stream);

/* ---------------------------------------------------------------------
 * Serving: resident S-matrices, builds and probe queries that arrive while
 * others run (continuous batching).
 *
 * An S-matrix, once built, serves any probe positions and probe settings
 * ("PRISM Simulations with Varying Probe Size": the S-matrix is re-used as
 * long as the specimen and f stay the same). A server keeps admitted
 * S-matrices under a byte budget and queues S-matrix builds and probe
 * queries. Each flush dispatches what arrived since the previous one:
 *   - queued builds in arrival order on the server's build stream, each
 *     once prism_smatrix_bytes of it fits the budget (memory-based
 *     admission); with LRU eviction on, idle S-matrices (no queued query,
 *     nothing in flight) are released least recently used first to make
 *     room, and reported by prism_server_evictions;
 *   - the queued queries whose specimen's build has been dispatched,
 *     bucketed by launch class (prism_probe_class) in arrival order and
 *     merged into prism_probe_batch calls of up to max_probes positions:
 *     queries of different specimens and optics in one bucket share the
 *     window-sum and window launches, and the queries of one (specimen,
 *     optics, detector) form one request. Each call goes to the first query
 *     slot (one of n_streams HIP streams, default priority) whose earlier
 *     calls have all finished, else to the slot with the fewest calls in
 *     flight. A call's slot waits on the device for the builds of the
 *     S-matrices it reads, so builds and other specimens' queries overlap.
 * A query's result is the prism_probe_outputs result for its own positions
 * (bit for bit, whatever it was merged with).
 *
 * Workspace: the caller's device buffer, split into one region per query
 * slot; a region holds the staged positions (max_probes x 2 doubles) and
 * outputs (max_probes x max_det doubles) of one merged call plus the
 * probe-step workspace (probe_ws_bytes, at least the probe step's minimum
 * for every admitted specimen and optics; prism_server_submit checks it).
 * Buffers named in admit, submit_build and submit (S-matrix, build
 * workspace, positions, outputs) must stay valid until the server is done
 * with them: positions and outputs until the query is reported done by poll
 * or wait, a build workspace until its build is reported done, an S-matrix
 * until it is evicted (explicitly, or reported by prism_server_evictions).
 * The server's streams are non-blocking and wait for no other stream: a
 * query's positions and a plan's potential slices must be written (their
 * streams synchronised) before the flush that dispatches them, and outputs
 * are complete only once poll or wait reports them. A server is used by one
 * host thread at a time.
 * --------------------------------------------------------------------- */
typedef struct prism_server prism_server;

int prism_server_workspace_bytes(int n_streams, int max_probes, int max_det,
                                 size_t probe_ws_bytes, size_t* bytes);
/* n_streams in [1, 16], max_probes >= 1, max_det in [1, PRISM_MAX_DET].
 * PRISM_ENOSPACE if ws_bytes is below the staging size. */
int prism_server_create(prism_server** server, size_t smatrix_budget_bytes, int n_streams,
                        int max_probes, int max_det, void* ws, size_t ws_bytes);
/* Waits for the server's streams, then frees the host state (never the
 * caller's device buffers). */
void prism_server_destroy(prism_server* server);
/* Admit one specimen's S-matrix now (prism_smatrix_bytes of it must fit in
 * the remaining budget, after LRU eviction when enabled, else
 * PRISM_ENOSPACE; smatrix_bytes is the size of the caller's buffer,
 * PRISM_EINVAL if smaller). With build_ws != NULL the server builds it with
 * prism_build_smatrix on its build stream, where every build runs, so
 * builds are ordered among themselves and may share one build workspace;
 * the plan's potential slices must be set and written (their stream
 * synchronised) before the call. With build_ws == NULL smatrix_dev must
 * already hold it (built by the caller and synchronised). *id names it. */
int prism_server_admit(prism_server* server, prism_plan* plan, int f, double alpha_max_mrad,
                       void* smatrix_dev, size_t smatrix_bytes, void* build_ws,
                       size_t build_ws_bytes, int* id);
/* Queue the build of one specimen's S-matrix (Fig. 1c), dispatched by a
 * later flush once its bytes fit the budget. smatrix_dev/smatrix_bytes and
 * build_ws/build_ws_bytes as in prism_build_smatrix; the build workspace
 * may be shared by every queued build (builds run one after another on the
 * build stream). *id names the specimen at once: queries may be submitted
 * against it before its build runs (they wait for it). *ticket is reported
 * by poll / wait when the S-matrix is complete.
 * Errors: PRISM_EINVAL (null argument, the checks of prism_build_smatrix's
 * sizes), PRISM_ENOSPACE (S-matrix larger than the whole budget, build
 * workspace below the build minimum). */
int prism_server_submit_build(prism_server* server, prism_plan* plan, int f,
                              double alpha_max_mrad, void* smatrix_dev, size_t smatrix_bytes,
                              void* build_ws, size_t build_ws_bytes, int* id, long long* ticket);
/* LRU eviction (enable != 0): admission may release idle S-matrices, least
 * recently used first (off by default: admission then fails or waits). */
int prism_server_set_lru_eviction(prism_server* server, int enable);
/* Dispatch limit (calls_per_slot > 0): a flush sends queries only while
 * some slot holds fewer than calls_per_slot probe-step calls in flight;
 * the rest stay queued and are merged with later arrivals at a later flush
 * (continuous batching: queries join the next call as slots free up).
 * 0 (the default): every flush dispatches everything it can. */
int prism_server_set_dispatch_limit(prism_server* server, int calls_per_slot);
/* Specimens released by LRU eviction since the previous call: up to
 * capacity ids into ids, *count of them. Their S-matrix buffers are the
 * caller's again. */
int prism_server_evictions(prism_server* server, int* ids, int capacity, int* count);
/* Release a specimen's budget after its dispatched calls have finished
 * (waits for the server's streams). PRISM_EINVAL if queries are queued or
 * its build has not been dispatched. */
int prism_server_evict(prism_server* server, int id);
/* Queue one query: n_probes in [0, max_probes] positions (device float64
 * [P][2], A), optics and detector as in prism_probe_outputs (copied), out_dev
 * float64 [P][n_det]. Returns a ticket. Nothing runs before the next flush.
 * Every check of the probe step (optics, alpha_max, detector edges, window
 * size, workspace region) runs here, so a queued query cannot fail a flush. */
int prism_server_submit(prism_server* server, int id, const double* probe_xy_dev, int n_probes,
                        const prism_optics* optics, const prism_detector* detector,
                        double* out_dev, long long* ticket);
/* Dispatch the queued builds that fit and the queued queries whose
 * specimen's build has been dispatched (as above). */
int prism_server_flush(prism_server* server);
/* Report finished queries and builds: up to capacity tickets into done,
 * *count of them. A ticket is reported once (by poll or by wait). */
int prism_server_poll(prism_server* server, long long* done, int capacity, int* count);
/* Block until one dispatched query or build is done (PRISM_EINVAL if it is
 * still queued or unknown). */
int prism_server_wait(prism_server* server, long long ticket);
/* Admitted S-matrix bytes (dispatched builds included), queued queries and
 * builds, and dispatched-but-unreported tickets (any pointer may be NULL). */
int prism_server_stats(const prism_server* server, size_t* smatrix_bytes_used, int* queued,
                       int* in_flight);
/* Probe-step calls the server has dispatched (prism_probe_batch calls), and
 * how many of them read more than one specimen's S-matrix (queries of
 * several specimens merged into shared launches). Either pointer may be
 * NULL. */
int prism_server_call_stats(const prism_server* server, long long* probe_calls,
                            long long* multi_specimen_calls);

/* Launch shapes of a plan, none of which changes any result (the same
 * operations run in the same order; only their distribution over
 * workgroups and launches changes), chosen per grid by a tuning sweep on
 * the target GPU. A zero field means the library default (shown).
 *   row_iters, col_iters: most row groups / column tiles one workgroup of
 *     the four-step slice passes walks (powers of two up to 64; 16, 8);
 *   row_min_groups, col_min_groups: fewest workgroups a slice-pass launch
 *     keeps when choosing those counts (512, 256);
 *   wave_chunk_mib: wave state per slice-pass launch, which sets the
 *     preferred build and multislice workspaces (16 .. 65536; 256);
 *   probe_group: probes per window-sum group (16, 32, 64; 0: 64 for
 *     W >= 128, 32 for W >= 64, else 16), which also sets the tile shape
 *     prism_probe_group reports;
 *   window_tile_div: window-sum workgroups per probe group are the 128-pixel
 *     tiles of one window divided by this (1 .. 64; 4).
 * Query workspace sizes after setting it. PRISM_EINVAL for values outside
 * these ranges (nothing is changed then). */
typedef struct {
  int row_iters;
  int row_min_groups;
  int col_iters;
  int col_min_groups;
  int wave_chunk_mib;
  int probe_group;
  int window_tile_div;
} prism_tuning;
int prism_set_tuning(prism_plan* plan, const prism_tuning* tuning);
/* The plan's effective launch shapes (probe_group 0: chosen by W). */
int prism_get_tuning(const prism_plan* plan, prism_tuning* tuning);

/* Per-kernel timing: while enabled, every kernel launch of this plan is
 * bracketed by HIP events recorded on its stream. prism_profile_report
 * waits for the recorded events, writes one line per kernel name
 * "name launches total_ms min_ms max_ms\n" into buf (NUL-terminated;
 * PRISM_ENOSPACE if buf_len is too small) and clears the records. */
int prism_profile_enable(prism_plan* plan, int enable);
int prism_profile_report(prism_plan* plan, char* buf, size_t buf_len);

/* Thread-local description of the last non-zero status ("" if none). */
const char* prism_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* PRISM_H */
