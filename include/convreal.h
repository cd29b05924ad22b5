/*
 * convreal.h - C ABI of libconvreal, the real-space half of a split spherical
 * convolution on one AMD Instinct MI355X (gfx950).
 *
 * The operation (Sutter, Wandelt & Elsner, "Using hybrid GPU/CPU kernel
 * splitting to accelerate spherical convolutions", Estimating Errors
 * section, Eq. 1): a radially symmetric kernel is split into a band-limited
 * harmonic part (l <= l_cut, applied elsewhere by spherical-harmonic
 * transforms) and a compact real-space part truncated at theta_cut. This
 * library applies the real-space part to maps on the equal-area iso-latitude
 * ring grid the paper assumes (HEALPix, ring order, Results section):
 *
 *     y_p = Omega * sum_{q : d_pq <= d_cut} Ktilde(d_pq) * x_q
 *
 *   Omega  = 4 pi / Npix, Npix = 12 nside^2 (pixel area; equal for all pixels)
 *   d_pq   = |v_p - v_q|, chord between pixel-centre unit vectors
 *   d_cut  = 2 sin(theta_cut / 2); pairs with d_pq == d_cut are included
 *   Ktilde = K interpolated from a table on a uniform chord grid (the paper's
 *            real-space convolver interpolates its kernel from tabulated
 *            nodes; discussion of Fig. 4).
 *
 * Pixel layout: ring order as in the HEALPix library. Ring i = 1..4N-1 from
 * the north pole; caps (i < N or i > 3N) hold 4k pixels (k = distance in
 * rings from the nearer pole) at phi = (pi/2k)(a + 1/2); belt rings hold 4N
 * pixels at phi = (pi/2N)(a + s/2), s = (i - N + 1) mod 2.
 *
 * Kernel table convention: n_tab values T[k] = K(d_k), d_k = k * h,
 * h = d_cut / (n_tab - 3), k = 0..n_tab-1 (the last two nodes lie beyond
 * d_cut). Ktilde(d) is the 4-point Lagrange interpolant on nodes
 * k-1..k+2 of segment k = floor(d/h) (k clamped to n_tab-3), with ghost
 * node T[-1] = T[1] (K is even in d). K is in continuous normalisation;
 * the library multiplies by Omega.
 *
 * Error behaviour: every entry point returns CONV_REAL_OK (0) or a
 * negative code. Arguments are validated on the host before any device call;
 * an invalid argument leaves all outputs untouched. conv_real_last_error()
 * returns a message for the calling thread's most recent failure.
 */
#ifndef CONVREAL_H
#define CONVREAL_H

#ifdef __cplusplus
extern "C" {
#endif

typedef struct conv_real_plan conv_real_plan;

/* Precision modes. */
#define CONV_REAL_F64   0  /* maps FP64 in/out; every pixel pair evaluated and accumulated in FP64 */
#define CONV_REAL_F32   1  /* maps FP32 in/out; every pixel pair evaluated and accumulated in FP64 */
#define CONV_REAL_MIXED 2  /* maps FP32 in/out; ring-pair weight blocks in split hi/lo FP16 on the
                              matrix cores, FP32 products summed per ring pair, FP64 across ring pairs */

/* Error codes. */
#define CONV_REAL_OK           0
#define CONV_REAL_EINVAL      -1  /* bad argument value (nside, n_tab, theta_cut, precision, nmaps, NULL) */
#define CONV_REAL_ENOMEM      -2  /* device or host allocation failed */
#define CONV_REAL_EHIP        -3  /* a HIP runtime call failed; see conv_real_last_error() */
#define CONV_REAL_EALIAS      -4  /* maps_in and maps_out overlap */
#define CONV_REAL_ENODEV      -5  /* no usable gfx950 device */

/* Limits. */
#define CONV_REAL_MAX_NSIDE  8192
#define CONV_REAL_MAX_NTAB   8192
#define CONV_REAL_MAX_LMAX   32768

/*
 * conv_real_tabulate - sample a radial kernel given by its harmonic
 * coefficients on the chord grid used by conv_real_init.
 *
 *   K(theta) = sum_{l=0}^{lmax} (2l+1)/(4 pi) * k_ell[l] * P_l(cos theta)
 *
 * (the Legendre transformation operator that links l-space and real-space
 * kernels, Eq. 1), summed in FP64 on the device with the three-term Legendre
 * recurrence written in u = 1 - cos(theta) = d^2/2, so that no cancellation
 * occurs near theta = 0.
 *
 *   k_ell      host pointer, lmax+1 doubles (read only, caller-owned)
 *   lmax       0 <= lmax <= CONV_REAL_MAX_LMAX
 *   theta_cut  truncation radius in radians, 0 < theta_cut <= pi
 *   n_tab      4 <= n_tab <= CONV_REAL_MAX_NTAB
 *   table      host pointer, n_tab doubles written (caller-owned)
 *
 * Synchronous: returns after the table has been copied back.
 */
int conv_real_tabulate(const double* k_ell, int lmax, double theta_cut, int n_tab, double* table);

/*
 * conv_real_init - build a plan for one (nside, kernel table, theta_cut, precision).
 *
 *   plan       out: opaque handle, owned by the caller until conv_real_destroy
 *   nside      1 <= nside <= CONV_REAL_MAX_NSIDE
 *   table      host pointer, n_tab doubles in the convention above (copied)
 *   n_tab      4 <= n_tab <= CONV_REAL_MAX_NTAB
 *   theta_cut  0 < theta_cut <= pi
 *   precision  CONV_REAL_F64, CONV_REAL_F32 or CONV_REAL_MIXED
 *
 * Binds the plan to the current HIP device. Computes the ring-pair windows
 * (ring_window pass), the exact pair count and the device tables; for
 * CONV_REAL_MIXED also the split-FP16 weight blocks. Synchronous.
 */
int conv_real_init(conv_real_plan** plan, int nside, const double* table, int n_tab,
                   double theta_cut, int precision);

/*
 * conv_real_apply - y = A x for nmaps maps.
 *
 *   maps_in    device pointer, [nmaps][12 nside^2] contiguous, FP64 for
 *              CONV_REAL_F64, FP32 otherwise (read only)
 *   maps_out   device pointer, same shape and type (written); must not
 *              overlap maps_in (CONV_REAL_EALIAS)
 *   nmaps      >= 1
 *   stream     hipStream_t to launch on (NULL = default stream)
 *
 * Asynchronous on stream; no host synchronisation, no allocation. Applies of one plan must not run
 * at the same time on different streams: the plan's work-queue counters and (ring-FFT method) its
 * spectrum workspaces are per plan.
 */
int conv_real_apply(conv_real_plan* plan, const void* maps_in, void* maps_out, int nmaps,
                    void* stream);

/*
 * conv_real_apply_noalloc - conv_real_apply for callers that cannot allocate device memory or call
 * the allocator at apply time (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc). Same arguments, result and errors as conv_real_apply, which stays as it is.
 *
 * The per-launch scratch of mixed plans (the per-map max |x| that sets the FP16 split scale, and the
 * work-queue counters: (64 + 8) x 4 bytes) is taken from a fixed 1 KiB array in device memory
 * instead of the plan's own buffers. Each device the library runs on holds one such array until the
 * process ends; its address is located once per device by conv_real_init. The kernels clear what
 * must start at zero at the start of every launch, so the contents a previous call left do not
 * matter; but every call on one device shares that device's array, so calls of this entry point that
 * may overlap in time on one device (other streams, other threads, other plans) race and give
 * wrong results: serialise them. Direct-method F64 and F32 plans use no scratch at all. Plans on the
 * ring-FFT method (conv_real_set_method) need spectrum workspaces of (n/2 + 1) x 32 bytes per belt
 * ring, beyond the fixed maximum: EINVAL. Calls no allocating routine.
 */
int conv_real_apply_noalloc(conv_real_plan* plan, const void* maps_in, void* maps_out, int nmaps,
                            void* stream);

/*
 * conv_real_pairs - exact number of ordered pixel pairs (p, q) with
 * d_pq <= d_cut over the whole map (counted on the device at init).
 */
int conv_real_pairs(const conv_real_plan* plan, long long* pairs);

/*
 * conv_real_profile - run conv_real_apply once with HIP events recorded on `stream` between the
 * library's kernels, wait for it, and report per kernel (tracing and benchmarks).
 *
 *   names      out: up to *nstages static kernel names (caller-owned array of pointers)
 *   ms         out: up to *nstages durations in milliseconds (launches of the same kernel in a
 *              row are merged)
 *   work       out: up to *nstages pixel pairs summed by the kernel (0 for auxiliary kernels)
 *   nstages    in: capacity of the three arrays; out: number of entries written
 *
 * Same arguments and errors as conv_real_apply; synchronous.
 */
int conv_real_profile(conv_real_plan* plan, const void* maps_in, void* maps_out, int nmaps,
                      void* stream, const char** names, float* ms, long long* work, int* nstages);

/*
 * Launch configuration of the mixed path (CONV_REAL_MIXED). All of a mixed apply's pair sums run
 * in one persistent kernel that drains a work queue of belt items (a band of 16 output rings x
 * `seg` output pixels, bound by LDS traffic) and cap items (64 output pixels with their 16 symmetric
 * images each, bound by on-the-fly weight evaluation or by the weight store's stream).
 *   seg        belt output pixels per work item: 256 or 512
 *   wg_per_cu  workgroups per compute unit (persistent grid = CUs x wg_per_cu): 1..4; at most 2
 *              are resident at once, 3 where seg is 256 and the plan holds a cap weight store
 *   order      0: items by decreasing estimated cost; 1: belt and cap items alternating; 2: one
 *              queue per XCD holding neighbouring belt bands and cap rings (whose input rings overlap,
 *              so they share that XCD's L2), alternating as in 1, with workgroups taking from
 *              other XCDs' queues once their own is empty; 3: roles: one queue of belt items and
 *              two of cap items (each by decreasing cost), the first workgroup of every compute
 *              unit starting on the belt queue and the other two on the cap queues (belt items
 *              use the matrix cores and LDS, cap items the vector memory path, so each CU runs
 *              both), every workgroup taking from the other queues once its own is empty;
 *              4: roles as in 3, with the cap items split into one queue of neighbouring rings per
 *              XCD (each XCD's cap workgroups start on rings whose input rings overlap, so that their
 *              re-reads share that XCD's L2)
 */
typedef struct conv_real_tuning {
  int seg;
  int wg_per_cu;
  int order;
} conv_real_tuning;

/* conv_real_set_tuning / conv_real_get_tuning - set or read a mixed plan's launch configuration
 * (EINVAL for other precisions or out-of-range fields). Synchronous; not while an apply on the
 * plan may still be running. */
int conv_real_set_tuning(conv_real_plan* plan, const conv_real_tuning* t);
int conv_real_get_tuning(const conv_real_plan* plan, conv_real_tuning* t);

/*
 * Cap weight store of a mixed plan. The cap-touching ring pairs' weights (one per output pixel of
 * the symmetry group's fundamental domain and input pixel inside that pixel's window: about the
 * cap-touching pixel pairs divided by 16) are either evaluated on the fly by every apply, or
 * computed once into device memory and streamed by every apply, which moves that part of the kernel
 * from arithmetic to memory bandwidth. The store keeps each weight as the FP16 pair the matrix cores
 * take, in 16-byte groups of 4 inputs that meet the output pixel's window (about 4.5 bytes per
 * weight). Both evaluate the same interpolated kernel; their results differ only by the rounding
 * of the weights' two evaluation forms, far within the mixed path's tolerance.
 *   CONV_REAL_STORE_OFF   evaluate on the fly; frees a store the plan holds
 *   CONV_REAL_STORE_ON    build the store (ENOMEM if the device cannot hold it)
 *   CONV_REAL_STORE_AUTO  build it if it needs at most 64 GiB and 40% of the free device memory
 * A new mixed plan takes CONV_REAL_STORE_AUTO. Unless the plan's launch configuration was set by
 * conv_real_set_tuning or conv_real_autotune, changing the store also picks its default: seg 256,
 * 3 workgroups per compute unit and order 3 with or without a store (the kernel is then built for
 * three waves per SIMD; without a store the cap items' coefficient table shares the LDS of the belt
 * stage).
 * conv_real_set_weight_store is synchronous (not while an apply on the plan may still run) and
 * allocates; applies never allocate. conv_real_get_weight_store reports whether a store is held
 * and its size in bytes. Mixed plans only (EINVAL otherwise).
 */
#define CONV_REAL_STORE_OFF  0
#define CONV_REAL_STORE_ON   1
#define CONV_REAL_STORE_AUTO 2
int conv_real_set_weight_store(conv_real_plan* plan, int mode);
int conv_real_get_weight_store(const conv_real_plan* plan, int* active, long long* bytes);

/*
 * Method of an FP64 or mixed plan. The paper's real-space convolver costs time linear in
 * theta_cut (Eq. 7; Results section), which a per-pair sum (quadratic) cannot match at the wide cuts
 * its optimal splits choose (Table 1). For two rings of the equatorial belt (4 Nside pixels each)
 * the pair sum is a circular convolution along the ring, so it can run in Fourier space:
 *   CONV_REAL_METHOD_DIRECT    every pixel pair summed directly (the default)
 *   CONV_REAL_METHOD_RING_FFT  belt ring pairs as a product per frequency of the input ring's
 *                              spectrum and the pair's kernel spectrum (computed once here, FP64,
 *                              (n/2 + 1) x 8 bytes per belt ring pair of a north output ring, n =
 *                              4 Nside; plus two spectrum workspaces of (n/2 + 1) x 16 bytes per belt
 *                              ring), inverse FFTs per output ring; ring pairs touching a polar cap summed per
 *                              pair, each weight once for the 16 images of its symmetry orbit (FP64
 *                              matrix cores). Same pairs and kernel values as DIRECT; results differ
 *                              by FP64 rounding only. Requires a power-of-two nside <= 2048 (EINVAL
 *                              otherwise) and a device that can hold the spectra (ENOMEM).
 *                              Mixed plans (FP32 maps): the belt ring pairs the same way (FP64
 *                              spectra and transforms), the cap-touching ring pairs on the plan's
 *                              split-FP16 cap tiles (weight store or on the fly) added to the belt
 *                              rings; within the mixed path's bound of the direct method (the belt
 *                              part is FP64 instead of split FP16). EINVAL for a mixed plan whose
 *                              belt windows cover whole rings or whose table has over 4098 nodes.
 * Synchronous and allocating (not while an apply on the plan may run); conv_real_apply then uses the
 * method, one map at a time for the belt part. FP64 and mixed plans (EINVAL for F32 plans). A plan
 * on the ring-FFT method takes no part in batches (conv_real_batch_create: EINVAL) and in
 * conv_real_apply_noalloc (EINVAL).
 */
#define CONV_REAL_METHOD_DIRECT   0
#define CONV_REAL_METHOD_RING_FFT 1
int conv_real_set_method(conv_real_plan* plan, int method);
int conv_real_get_method(const conv_real_plan* plan, int* method);

/*
 * conv_real_autotune - time every launch configuration on the caller's maps (each configuration
 * once warm, then three timed applies with HIP events on `stream`), keep the fastest on the plan
 * and return it in *best. Same map arguments as conv_real_apply; maps_out is overwritten.
 * Synchronous. Mixed plans only.
 */
int conv_real_autotune(conv_real_plan* plan, const void* maps_in, void* maps_out, int nmaps, void* stream,
                       conv_real_tuning* best);

/*
 * Batches: maps of different grids and kernels (each with its own mixed plan) in one persistent
 * launch, so that small maps fill the GPU alongside large ones.
 *
 * conv_real_batch_create - count (1..64) mixed plans on the current device; the batch keeps the
 *   plan pointers (the plans must outlive it) and builds one cost-sorted work queue.
 * conv_real_batch_apply - maps_in[k], maps_out[k]: host arrays of device pointers, one FP32 map of
 *   plan k each (12 nside_k^2 values); no overlaps between any input and output. Asynchronous on
 *   stream, no allocation, no host synchronisation (capturable in a HIP graph).
 * conv_real_batch_set_tuning / conv_real_batch_autotune - as for plans.
 * conv_real_batch_pairs - total pixel pairs of one batch apply.
 * conv_real_batch_destroy - free the batch (not its plans). NULL is accepted.
 */
typedef struct conv_real_batch conv_real_batch;
int conv_real_batch_create(conv_real_batch** batch, conv_real_plan* const* plans, int count);
int conv_real_batch_apply(conv_real_batch* batch, const float* const* maps_in, float* const* maps_out,
                          void* stream);
int conv_real_batch_set_tuning(conv_real_batch* batch, const conv_real_tuning* t);
int conv_real_batch_autotune(conv_real_batch* batch, const float* const* maps_in, float* const* maps_out,
                             void* stream, conv_real_tuning* best);
int conv_real_batch_pairs(const conv_real_batch* batch, long long* pairs);
int conv_real_batch_destroy(conv_real_batch* batch);

/* conv_real_destroy - free a plan and its device memory. NULL is accepted. */
int conv_real_destroy(conv_real_plan* plan);

/* conv_real_strerror - static description of an error code. */
const char* conv_real_strerror(int code);

/* conv_real_last_error - message for this thread's most recent failure ("" if none). */
const char* conv_real_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* CONVREAL_H */
