/*
 * tsl.h -- C ABI of the MI355X online PARAFAC subspace-tracking step.
 *
 * Method: Mardani, Giannakis, Ugurbil, "Tracking Tensor Subspaces with
 * Informative Random Sampling for Real-Time MR Imaging" (arXiv 1609.04104).
 * One sequence ("scan") is a stream of N1 x N2 k-space frames acquired with a
 * single coil.  Its state is a pair of image-domain factors A (N1 x R) and
 * B (N2 x R) plus the step-size accumulator alpha_bar and the frame counter t.
 * Each pushed frame runs one pass of Algorithm 3 with one coil (Sec. IV-B):
 * the ridge solve for gamma_t (Sec. III-A, S1), the residual of the sampled
 * k-space against F(A diag(gamma_t) B^T), its back-projection F^{-1}(Xi) and the
 * majorization-minimization factor updates (eq. 6, Algorithm 3 S2); it returns
 * X_t = A[t] diag(gamma_t) B[t]^T (Sec. IV-A).  tsl_sample_lines draws the
 * next frame's phase-encode rows by Algorithm 4 with the row score of Sec. VI-C.
 *
 * Conventions
 *   - Every array argument is a DEVICE pointer (e.g. torch.Tensor.data_ptr()),
 *     unless its comment says "host".  Complex numbers are interleaved
 *     (re, im) float32 pairs, i.e. torch.complex64.  Arrays are row-major:
 *     a frame is [n1][n2] (row = phase-encode line, column = readout sample),
 *     a factor is [n][r].
 *   - k-space is in natural FFT order (DC at index 0); the 2-D transform is
 *     unitary, F(X) = F_l X F_r with [F_N]_{km} = N^{-1/2} exp(-2 pi i k m / N).
 *   - `stream` is a hipStream_t (torch.cuda.current_stream().cuda_stream;
 *     NULL = the null stream).  Calls are stream-ordered and asynchronous:
 *     the caller keeps every buffer valid until the stream has passed the call.
 *   - Supported transform lengths: see tsl_size_supported (products of
 *     2, 3 and 5 between 8 and 512 from a fixed list).  1 <= r <= TSL_MAX_R.
 *
 * Ownership
 *   - The caller owns every buffer it passes; the library never frees them.
 *   - The library owns a tsl_seq (its device state and workspace); tsl_close
 *     releases it.  One handle is used by one host thread at a time.
 *
 * Errors
 *   - Argument errors are detected before anything is enqueued and return a
 *     negative code; the state is untouched and tsl_last_error() (thread-local)
 *     says why.
 *   - Errors the device detects (a non-positive-definite ridge Gram, NaN/Inf in
 *     a sample or in a result, rows out of range / not ascending) latch into the
 *     sequence's status word.  The frame that raised it is not committed (A, B,
 *     alpha_bar and t keep their values) and later frames of that sequence are
 *     skipped on the device until the status is cleared; tsl_status reports it.
 *   - HIP runtime failures return TSL_EDEVICE.
 */
#ifndef TSL_H
#define TSL_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define TSL_MAX_R 128
#define TSL_MAX_COILS 32       /* coils of a several-coil sequence (tsl_open_coils) */
#define TSL_MAX_COIL_R 64      /* rank of a several-coil sequence                   */

typedef struct tsl_seq tsl_seq;
typedef struct tsl_pool tsl_pool;
typedef struct tsl_batch tsl_batch;
typedef struct { float re, im; } tsl_c32;

enum {
    TSL_OK = 0,
    TSL_EINVAL = -1,         /* bad argument, or (device) bad row list            */
    TSL_ENOMEM = -2,         /* device allocation failed                          */
    TSL_EDEVICE = -3,        /* HIP runtime error                                 */
    TSL_ENOTPD = -4,         /* (device) ridge Gram not positive definite         */
    TSL_ENONFINITE = -5,     /* (device) NaN or Inf in a sample or a result       */
    TSL_EBUSY = -6,          /* pool budget exhausted                             */
    TSL_EUNSUPPORTED = -7    /* transform length not in the supported list        */
};

enum { TSL_STEP_MM = 0, TSL_STEP_CONST = 1 };

/* How a line-mask frame evaluates the residual and the back-projected
   gradients (Sec. IV-B; point masks always take the frame route).
   TSL_ROUTE_KSPACE: on the sampled rows only.  With the separable transform
   F(X) = F_l X F_r^T, the k-space prediction at the samples is
   Ahat_S diag(gamma) Bhat^T (Ahat = F_l A, Bhat = F_r B), and Theta =
   F^{-1}(Xi) = sum over samples of e_l times the conjugate sampling matrix,
   so Theta conj(B) = F_l^H [rows S: E conj(Bhat)] and Theta^T conj(A) =
   F_r^H (E^T conj(Ahat_S)), E the |S| x n2 residual.  Same quantities as the
   frame route up to rounding, without frame-sized intermediates.
   TSL_ROUTE_FRAME: synthesis A diag(gamma) B^T, the 2-D transform, the masked
   residual, the inverse 2-D transform Theta, and Theta's contractions with
   conj(B) and conj(A), all frame-sized. */
enum { TSL_ROUTE_KSPACE = 0, TSL_ROUTE_FRAME = 1 };

typedef struct {
    int      step_mode;      /* TSL_STEP_MM: mu_t = 1/alpha_bar_t, the recursion of
                                eq. (6) (default).  TSL_STEP_CONST: mu_t = mu.       */
    double   mu;             /* constant step, used iff step_mode == TSL_STEP_CONST   */
    int      allow_lambda0;  /* accept lambda == 0 (tests of exact recovery)          */
    uint64_t seed;           /* sampler key word 0 (Philox4x64-10)                    */
    uint64_t stream_id;      /* sampler key word 1                                    */
    int      line_route;     /* TSL_ROUTE_KSPACE (default) or TSL_ROUTE_FRAME          */
    int      synth_bf16;     /* operands of the rank-R syntheses A diag(gamma) B^T (the
                                frame route's X- and the output X_t, eq. 2) on the
                                matrix cores: TSL_SYNTH_FP32 (default), TSL_SYNTH_BF16
                                (BF16 operands, FP32 sums: relative error of X near
                                3e-3, outside the 1e-4 parity bar) or TSL_SYNTH_BF16X3
                                (each FP32 operand split into two BF16 numbers and
                                three products summed: near 1e-5)                    */
} tsl_opts;

enum { TSL_SYNTH_FP32 = 0, TSL_SYNTH_BF16 = 1, TSL_SYNTH_BF16X3 = 2 };

/* Number of timed phases reported by tsl_step_many_timed. */
#define TSL_N_PHASES 7

/* One frame of one sequence, for tsl_push_frame and tsl_step_many.  `mask`
   non-NULL selects a point mask (see tsl_push_points); otherwise the sample
   set is the rows `rows` (see tsl_push_lines).  Zero-initialise the struct
   and fill what is used. */
typedef struct {
    int            n_rows;     /* host: number of rows, 0..n1; with n_rows_dev, the
                                  capacity of `rows` (and of y's rows), 0..n1           */
    const int32_t* rows;       /* [n_rows] strictly ascending row indices, or NULL      */
    const uint8_t* mask;       /* [n1][n2] 0/1 point mask, or NULL                      */
    const tsl_c32* y;          /* [n_rows][n2] rows' samples; [n1][n2] if y_full or a
                                  point mask                                            */
    tsl_c32*       X_out;      /* [n1][n2] or NULL                                      */
    tsl_c32*       A_out;      /* [n1][r] or NULL                                       */
    tsl_c32*       B_out;      /* [n2][r] or NULL                                       */
    tsl_c32*       gamma_out;  /* [r] or NULL                                           */
    const int32_t* n_rows_dev; /* device word holding the row count, so that a row set
                                  drawn on the device needs no host round trip; it must
                                  lie in [0, n_rows] (checked on the device: TSL_EINVAL
                                  latches and the frame is not committed otherwise); or
                                  NULL to use n_rows                                    */
    int            y_full;     /* line masks: y is a whole [n1][n2] frame of which only
                                  the listed rows are read                              */
    int            K_next;     /* > 0: after the update, draw the rows of frame t+1 as
                                  tsl_sample_lines does, into rows_next / n_next        */
    int32_t*       rows_next;  /* [K_next] device, or NULL if K_next == 0               */
    int32_t*       n_next;     /* [1] device, or NULL if K_next == 0                    */
    double*        info_out;   /* [4] device float64, or NULL: the frame's step size
                                  alpha_t, alpha_bar_t, mu_t (eq. 6, Sec. III-A) and
                                  the conditioning of the ridge Gram G_t = Phi^H Phi +
                                  lambda I as max(D)/min(D) over the pivots of its
                                  L D L^H factorisation (a lower bound on kappa_2(G_t),
                                  equal to it for a diagonal G_t).  Written when the
                                  ridge solve succeeds                                 */
} tsl_frame;

/* Fills *o with the defaults: MM step, lambda > 0 required, seed 0, stream 0. */
void tsl_opts_default(tsl_opts* o);

/* 1 if n is a supported transform length, else 0.  Host only. */
int tsl_size_supported(int n);

/* Device bytes one sequence of this shape holds (state plus workspace); the
   unit of the pool's admission.  Host only; returns TSL_OK or TSL_EINVAL. */
int tsl_footprint(int n1, int n2, int r, size_t* bytes);

/* Opens a sequence: validates, allocates, copies A0 [n1][r] and B0 [n2][r]
   (device) into the resident state, sets alpha_bar = 0 and t = 0 (Algorithm 3's
   initialisation; the caller draws the start, e.g. at random or from a warm
   start), and computes the k-space factors F_l A0, F_r B0.  lambda >= 0 is the
   Tikhonov weight of (P2); lambda == 0 needs opts->allow_lambda0.  opts may be
   NULL (defaults). */
int tsl_open(tsl_seq** out, int n1, int n2, int r, double lambda, const tsl_opts* opts,
             const tsl_c32* A0, const tsl_c32* B0, void* stream);

/* Opens a sequence imaged by C coils (Algorithm 3 with C coils, Sec. IV-B):
   as tsl_open, plus H [C][n1][n2] (device, complex64, copied into the
   sequence), H[c] the sensitivity map of coil c; coil c sees the frame
   H_c .* X and samples F(H_c .* X).  1 <= C <= TSL_MAX_COILS, r <= TSL_MAX_COIL_R.
   Frames go through tsl_push_coils (the single-coil pushes, batched steps and
   tsl_epochs refuse such a sequence with TSL_EINVAL).  The step size uses
   g = max over pixels of sum_c |H_c|^2 (1 for maps normalised to unit sum of
   squares): alpha_t = lambda/t + g max(Gersh(G^H B^H B G), Gersh(G^H A^H A G)),
   which bounds the factor-block Lipschitz constant of the several-coil cost. */
int tsl_open_coils(tsl_seq** out, int n1, int n2, int r, int C, double lambda, const tsl_opts* opts,
                   const tsl_c32* A0, const tsl_c32* B0, const tsl_c32* H, void* stream);

/* Pushes frame t = t+1 of a several-coil sequence, sampled at the full
   k-space rows `rows` (strictly ascending, in [0, n1); checked on the device)
   of every coil: y [C][n_rows][n2], y[c][s][j] coil c's sample at
   (rows[s], j), i.e. [F(H_c .* X_t)]_{rows[s], j} plus noise (Sec. IV-B).  One
   step of Algorithm 3: Phi with entries [F(H_c .* (a_r b_r^T))]_{ij} over every
   coil's samples, gamma_t = (Phi^H Phi + lambda I)^{-1} Phi^H y (FP64), the
   residual per coil, Theta = sum_c conj(H_c) .* F^{-1}(Xi_c), and the updates
   of A and B from the factors at t-1.  n_rows == 0 is a pure shrink.  Outputs
   as tsl_push_lines (each may be NULL); device errors latch as there. */
int tsl_push_coils(tsl_seq* s, int n_rows, const int32_t* rows, const tsl_c32* y, tsl_c32* X_out, tsl_c32* A_out,
                   tsl_c32* B_out, tsl_c32* gamma_out, void* stream);

/* Releases the sequence after synchronising its last stream.  NULL is a no-op. */
int tsl_close(tsl_seq* s);

/* Pushes frame t = t+1 whose sample set is the full k-space rows `rows`
   (Sec. VI: Cartesian phase-encode lines), per Algorithm 3 with one coil:
     gamma_t = (Phi^H Phi + lambda I)^{-1} Phi^H y   (S1, Sec. III-A),
     Xi      = M .* (Y - F(A diag(gamma_t) B^T)),     Theta = F^{-1}(Xi),
     A <- (1 - lambda mu_t / t) A + mu_t Theta conj(B) conj(diag(gamma_t)),
     B <- (1 - lambda mu_t / t) B + mu_t Theta^T conj(A) conj(diag(gamma_t)),
   with mu_t from the MM recursion (eq. 6) or constant, both updates reading the
   factors of frame t-1.  rows: [n_rows] int32, strictly ascending, in [0, n1)
   (checked on the device: TSL_EINVAL latches otherwise); y: [n_rows][n2]
   complex64, y[s][j] the sample at (rows[s], j).  n_rows == 0 is allowed
   (gamma = 0, pure shrink).  Outputs (each may be NULL): X_out [n1][n2] =
   A[t] diag(gamma_t) B[t]^T, A_out [n1][r], B_out [n2][r], gamma_out [r]. */
int tsl_push_lines(tsl_seq* s, int n_rows, const int32_t* rows, const tsl_c32* y,
                   tsl_c32* X_out, tsl_c32* A_out, tsl_c32* B_out, tsl_c32* gamma_out,
                   void* stream);

/* As tsl_push_lines for an arbitrary sample set: mask [n1][n2] uint8 (nonzero =
   sampled), y [n1][n2] complex64 read only where mask is set (eq. 10). */
int tsl_push_points(tsl_seq* s, const uint8_t* mask, const tsl_c32* y,
                    tsl_c32* X_out, tsl_c32* A_out, tsl_c32* B_out, tsl_c32* gamma_out,
                    void* stream);

/* Draws the row set of frame t+1 by Algorithm 4 on rows (Sec. VI-C): row score
   s(i) proportional to N2 ||abar_i||^2 + R with abar the column-normalised
   k-space factor F_l A[t]; K >= 1 draws with replacement from Philox4x64-10 at
   counter (t+1, k, 0, 0) and key (seed, stream_id); every weight and sum in
   float64 without fused multiply-add, each sum of n terms in a fixed blocked
   order (sequential inside consecutive blocks of 16 terms, then the block sums
   in block order; the inclusive prefix is the matching blocked scan), so equal
   inputs give equal rows on any IEEE machine that keeps that order.  rows_out [K] receives the distinct rows ascending,
   n_out [1] their count (<= K).  Optional (may be NULL): draws_out [K] int32,
   the row of each trial; prefix_out [n1] float64, the inclusive prefix of the
   unnormalised weights. */
int tsl_sample_lines(tsl_seq* s, int K, int32_t* rows_out, int32_t* n_out,
                     int32_t* draws_out, double* prefix_out, void* stream);

/* Batch processing of a stored scan in several passes (Sec. VI-D): E passes
   over the T frames frames[0..T-1], pass e visiting them in the order
   order[e*T] .. order[e*T + T - 1] (host int32; each pass a permutation of
   0..T-1 -- the paper may reorder the frames at random between passes, so the
   caller draws the permutations, e.g. the time order for the first pass).  The
   state carries over from pass to pass (the subspace learnt in one pass starts
   the next, and t counts every visit, as the recursion of eq. (6) does).  Each
   visit is one step of Algorithm 3 exactly as tsl_push_frame; a frame's outputs
   are rewritten at every visit, so after the call they hold those of its last
   visit.  The frames of a stored scan draw no rows (K_next must be 0).
   TSL_EINVAL, with nothing enqueued, for bad arguments or an order that is not
   a permutation. */
int tsl_epochs(tsl_seq* s, int T, const tsl_frame* frames, int E, const int32_t* order, void* stream);

/* Draws the sample set of frame t+1 as single k-space entries by Algorithm 4
   with the score of eq. (13): s(n1, n2) = (||abar_n1||^2 + ||bbar_n2||^2) /
   (R (N1 + N2)), abar and bbar the rows of the column-normalised k-space
   factors F_l A[t] and F_r B[t] (a zero column left out), drawn as the exact
   two-component mixture of eq. (13) (probability N2/(N1+N2): row from
   ||abar||^2, column uniform; else column from ||bbar||^2, row uniform).  K >= 1
   trials with replacement; trial k takes the first three words w0..w2 of
   Philox4x64-10 at counter (t+1, k, 1, 0), key (seed, stream_id), u = (w >> 11)
   2^-53: component A iff u0 (N1+N2) < N2, the weighted index the first whose
   inclusive prefix (float64, blocked order as tsl_sample_lines) exceeds u1 W,
   the uniform one floor(u2 N) (clamped).  mask_out [n1][n2] uint8 receives 1
   at the distinct points drawn and 0 elsewhere (the form tsl_push_points
   takes), n_out [1] their count (<= K); draws_out [K] int32 (may be NULL) the
   entry n1 * N2 + n2 of each trial. */
int tsl_sample_points(tsl_seq* s, int K, uint8_t* mask_out, int32_t* n_out, int32_t* draws_out, void* stream);

/* Pushes one frame described by a tsl_frame (the general form of
   tsl_push_lines / tsl_push_points, with device-side row counts, full-frame
   sample arrays and the next frame's row draw in the same call). */
int tsl_push_frame(tsl_seq* s, const tsl_frame* frame, void* stream);

/* Batched push: frame frames[i] for sequence seqs[i], i < n, as n independent
   tsl_push_frame calls would, in one stream-ordered step.  Sequences of equal
   shape share launches; the launch sequence of a batch composition (which
   sequences, which outputs, which mask kinds, whether rows are drawn) is
   captured once in a HIP graph and replayed while the composition repeats.
   The sequences must be distinct.  Calls may go to different streams: each
   call's descriptors live in one of three slots that the library reuses only
   after the call that last used it has finished on the device (the host waits
   for it), so the host runs at most three calls ahead of the GPU. */
int tsl_step_many(tsl_seq* const* seqs, int n, const tsl_frame* frames, void* stream);

/* Allocation-free form of tsl_step_many, for callers that cannot allocate
   device memory (code under HIP graph capture, tight serving loops, harnesses
   that forbid hipMalloc): same arguments, same kernels and results as
   tsl_step_many.  It calls no hipMalloc, hipFree, hipHostMalloc or graph
   instantiation: the frame descriptors go into one fixed device array of
   2 x TSL_STATIC_MAX_FRAMES descriptors compiled into the library (each GPU it
   runs on holds its own copy, about 148 KiB, until the process ends), written by small
   kernels on `stream`, and the phases are launched directly on `stream`.
   n > TSL_STATIC_MAX_FRAMES returns TSL_EINVAL before anything is enqueued;
   every sequence must be on the current device.  All calls on one GPU share
   that array and each overwrites it: calls that can overlap on one GPU (on
   different streams with nothing ordering them) race and must not be made;
   calls on one stream are ordered.  The first call on a device looks up the
   array's device address (make it outside a stream capture). */
#define TSL_STATIC_MAX_FRAMES 256
int tsl_step_many_noalloc(tsl_seq* const* seqs, int n, const tsl_frame* frames, void* stream);

/* Profiling form of tsl_step_many: runs the same kernels without a graph,
   brackets each of the TSL_N_PHASES phases (partial Grams; solve and step
   size; synthesis + row transform; column transform + residual + column
   inverse; row inverse + A gradient [these three: frame route]; factor
   updates with F_l A and F_r B of the new factors [on the k-space route also
   the residual's gradient contractions]; output synthesis beside the row draw)
   with HIP events on `stream`, waits, and
   ADDS each phase's elapsed milliseconds to phase_ms[TSL_N_PHASES] (host). */
int tsl_step_many_timed(tsl_seq* const* seqs, int n, const tsl_frame* frames, double* phase_ms,
                        void* stream);

/* A batched step fixed once and replayed: the same work as
   tsl_step_many(seqs, n, frames, stream) (one step of Algorithm 3 per frame,
   with Algorithm 4's draw where K_next > 0), with the validation and the
   frame descriptors (uploaded once to device memory owned by the batch) done
   at creation, so that tsl_batch_launch only launches kernels.  Made for loops
   that cycle through a fixed set of steps (steady-state serving of a fixed
   batch; each step's device buffers -- rows, row counts, y, outputs -- are
   fixed at creation, their contents are read at launch).  flags:
   0 -- each launch issues the kernels on the stream directly (one launch per
        phase and shape group; the cheaper form for a few groups);
   TSL_BATCH_GRAPH -- the launches are captured once in a HIP graph and each
        launch replays it (one call whatever the number of groups).
   The sequences must be distinct and on the current device; every pointer in
   `frames` must stay valid while the batch lives.  *out receives the handle,
   or NULL on error (TSL_EINVAL on bad arguments, TSL_EDEVICE on a HIP
   failure; tsl_last_error tells which).  Closing one of the sequences
   invalidates the batch: launching it then returns TSL_EINVAL. */
enum { TSL_BATCH_GRAPH = 1 };
int tsl_batch_create(tsl_seq* const* seqs, int n, const tsl_frame* frames, int flags, tsl_batch** out);

/* Enqueues the batch's step on `stream` (NULL: the default stream).  Stream
   order is the only ordering: launches of batches that share a sequence must
   go to one stream.  Returns TSL_EINVAL for a NULL or invalidated batch or a
   current device other than the batch's. */
int tsl_batch_launch(tsl_batch* b, void* stream);

/* Waits for the batch's last launch and frees its descriptors and graph
   (NULL: no-op). */
int tsl_batch_destroy(tsl_batch* b);

/* Synchronises the sequence's last stream and returns its latched device
   status (TSL_OK or a negative code); clears it if clear != 0. */
int tsl_status(tsl_seq* s, int clear);

/* Copies the current factors (device): A [n1][r], B [n2][r] and the k-space
   factors F_l A [n1][r], F_r B [n2][r]; any pointer may be NULL. */
int tsl_get_factors(tsl_seq* s, tsl_c32* A, tsl_c32* B, tsl_c32* Ahat, tsl_c32* Bhat,
                    void* stream);

/* Host-blob checkpoint of the whole state (A, B, alpha_bar, t, options).
   tsl_get_state with blob == NULL stores the size in *nbytes.  Both
   synchronise the sequence's stream.  tsl_set_state needs a blob of the same
   shape whose lambda and options pass tsl_open's checks and whose alpha_bar
   and t are finite and >= 0 (TSL_EINVAL otherwise, nothing changed), and
   clears the status.  If the blob's lambda or options differ from the
   sequence's, every prepared batch that holds the sequence is invalidated. */
int tsl_get_state(tsl_seq* s, void* host_blob, size_t* nbytes);
int tsl_set_state(tsl_seq* s, const void* host_blob, size_t nbytes);

/* Output-synthesis tile tuner.  The output launch of a batched step (X_t =
   A[t] diag(gamma_t) B[t]^T, FP32 synthesis) has three block tiles that give
   identical results: 128 x 64 (0, the default), 64 x 64 (1) and 128 x 128 (2).
   tsl_batch_create times the three on each of the batch's output launches
   whose (largest n1, largest n2, r <= 32 or not, frame count rounded up to a
   power of two) has no choice yet -- into scratch frames and scratch row
   lists, so nothing the caller owns is written -- and keeps the fastest for every later
   launch of that kind in the process (tsl_step_many included).  TSL_TUNE=0
   turns the timing off; TSL_TUNE_CACHE names a text file of earlier choices
   ("n1 n2 one_pass count tile" per line), read at first use and appended to.
   tsl_output_tile (host) returns the tile such a launch uses now, or TSL_EINVAL. */
int tsl_output_tile(int n1, int n2, int r, int count);
/* Fixes the tile of such launches (0, 1 or 2) for the rest of the process, in
   place of timing (a deployment that wants a known launch shape). */
int tsl_set_output_tile(int n1, int n2, int r, int count, int tile);

/* Shape queries (host). */
int tsl_shape(const tsl_seq* s, int* n1, int* n2, int* r);

/* Standalone batched unitary 2-D transform of `batch` frames [n1][n2]
   (forward exp(-2 pi i k n / N) if inverse == 0, else its inverse), the
   transform the step applies to full frames (Sec. IV).  in and out may alias. */
int tsl_fft2(int n1, int n2, int batch, const tsl_c32* in, tsl_c32* out, int inverse,
             void* stream);

/* Serving admission: a pool with a device-byte budget.  tsl_open_in_pool is
   tsl_open that first reserves tsl_footprint bytes from the pool and returns
   TSL_EBUSY (nothing allocated) if the budget would be exceeded; closing the
   sequence returns its bytes. */
int tsl_pool_create(tsl_pool** out, size_t budget_bytes);
int tsl_pool_destroy(tsl_pool* p);
int tsl_pool_used(const tsl_pool* p, size_t* used, size_t* budget);
int tsl_open_in_pool(tsl_pool* p, tsl_seq** out, int n1, int n2, int r, double lambda,
                     const tsl_opts* opts, const tsl_c32* A0, const tsl_c32* B0, void* stream);

/* Text of the last failing call on this thread ("" if none). */
const char* tsl_last_error(void);

/* Host-side self-test of the in-register DFT codelets against a direct DFT in
   double precision; returns the largest relative error.  No device use. */
double tsl_selftest_codelets(void);

#ifdef __cplusplus
}
#endif

#endif /* TSL_H */
