/*
 * pbp.h -- C-ABI of the MI355X polar-code belief-propagation decoder.
 *
 * Method: Abbas, Fan, Chen, Tsui, "Low Complexity Belief Propagation Polar
 * Code Decoder".  An (n,k) polar code carries k information bits in the
 * reliable positions of the source word u and zeros in the n-k frozen ones;
 * the codeword is x = u F^{(x)m}, F = [[1,0],[1,1]], n = 2^m (Section II).
 * Decoding runs BP on the m-stage factor graph with the scaled min-sum PE
 * update of eq. (1), optionally stopping early on the G-matrix criterion
 * and freezing converged connected sub-factor-graphs (CSFGs, Section III,
 * eqs. (2)-(4)).
 *
 * Conventions used by every call:
 *  - N is a power of two, 2 <= N <= 16384 (the code length n); K is the
 *    number of information bits, 0 <= K <= N.
 *  - Bits are uint8 values 0/1.  Information bits are ordered by increasing
 *    source-word position.  LLRs are FP32, ln P(bit=0)/P(bit=1): positive
 *    favours 0.  Batches are row-major: frame f occupies [f*N, (f+1)*N).
 *  - "device" pointers are HIP device memory of the current device; "host"
 *    pointers are ordinary host memory.  The caller owns every buffer it
 *    passes; the library owns pbp_code handles, mixed plans and the
 *    per-stream decoder workspaces (see pbp_workspace_release).
 *  - `stream` is a hipStream_t (NULL: the default stream).  Device calls are
 *    asynchronous: they return after enqueuing, and results are valid once
 *    the stream has been synchronised.
 *  - A pbp_code handle is immutable once created: any number of threads and
 *    streams may use one handle at once.  Scratch that a decoder needs
 *    between launches lives in a workspace the library keeps per (device,
 *    stream), created by the first call on that stream that needs it (that
 *    call allocates device memory and synchronises the device; later calls
 *    on the stream do neither, unless a longer code needs more state).
 *  - Every call returns a pbp_status.  Arguments are checked on the host
 *    before anything is enqueued; a rejected call enqueues nothing.  No
 *    exception crosses the boundary.
 */
#ifndef PBP_H
#define PBP_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    PBP_OK = 0,
    PBP_EINVAL = -1,        /* an argument is out of range or inconsistent */
    PBP_ENOMEM = -2,        /* a host or device allocation failed          */
    PBP_EDEVICE = -3,       /* a HIP runtime call failed                   */
    PBP_EUNSUPPORTED = -4   /* valid request this build does not handle    */
} pbp_status;

/* Opaque, immutable code handle: N, K, the frozen set, its device copy and
 * the launch geometry derived from them. */
typedef struct pbp_code pbp_code;

/* Decoder options.
 *  max_iter      >= 1; the paper's experiments use 40 (Section IV).
 *  early_stop    0: none (the baseline decoder always runs max_iter
 *                iterations); 1: G-matrix criterion, checked after every
 *                iteration: stop when uhat G equals the hard decision of the
 *                total belief R + L at the channel column.
 *  freezing      0/1: CSFG freezing of Section III.
 *  freeze_input  the messages eq. (2) hard-decides: 0 = R at column j+1 as
 *                printed; 1 = the total belief R + L at column j+1.
 *  freeze_walk   what follows a successful freeze within one iteration:
 *                0 = no further check this iteration; 1 = continue at the
 *                next stage; 2 = keep checking the next CSFG of the stage.
 *  alpha         min-sum scale of eq. (1) (0.9375 in Section IV), > 0.
 */
typedef struct {
    int32_t max_iter;
    int32_t early_stop;
    int32_t freezing;
    int32_t freeze_input;
    int32_t freeze_walk;
    float alpha;
} pbp_decode_opts;

/* Human-readable text of a status code (static storage). */
const char *pbp_status_string(int32_t status);

/* Code construction (Section II: information bits go to the K most reliable
 * positions; the paper gives no construction method).  Positions are ranked
 * by the Bhattacharyya parameter of the recursion z_{2i} = 2z_i - z_i^2,
 * z_{2i+1} = z_i^2 from z_0 = exp(-(K/N) 10^(design_ebn0_db/10)), evaluated
 * in the log domain; the N-K largest are frozen, ties freezing the lower
 * index.  Host only.  frozen_out: host, N bytes, 1 = frozen.
 * Errors: PBP_EINVAL for a bad N or K or a NULL pointer. */
int32_t pbp_construct(int32_t N, int32_t K, double design_ebn0_db,
                      uint8_t *frozen_out);

/* Create a code handle from a frozen mask (host, N bytes, nonzero =
 * frozen).  The number of frozen positions must be N-K.  Allocates device
 * memory on the current device; the handle is then used on that device.
 * Errors: PBP_EINVAL, PBP_ENOMEM, PBP_EDEVICE. */
int32_t pbp_code_create(int32_t N, int32_t K, const uint8_t *frozen,
                        pbp_code **out);

/* Release a handle (NULL is ignored).  Synchronises the device first, so
 * no enqueued call may still use it. */
void pbp_code_destroy(pbp_code *code);

/* N and K of a handle; either out pointer may be NULL. */
int32_t pbp_code_dims(const pbp_code *code, int32_t *N, int32_t *K);

/* Encoding (Section II, Fig. 1): place the K information bits of each frame
 * at the information positions, zeros at the frozen ones, and compute
 * x = u F^{(x)m}.
 *   info      device, B x K uint8 (0/1)
 *   codeword  device, B x N uint8 (0/1), written
 * B >= 0 (0 enqueues nothing).  Errors: PBP_EINVAL, PBP_EDEVICE. */
int32_t pbp_encode(const pbp_code *code, const uint8_t *info, int64_t B,
                   uint8_t *codeword, void *stream);

/* BP decoding of a batch (Section II-A eq. (1), Section III, Section IV).
 * One iteration activates the PEs stage by stage from the channel column to
 * the source-word column; stage j computes L at column j from the previous
 * iteration's L at column j+1 and R at column j+1 from R at column j.  The
 * initial messages are the channel LLRs for R at column 1, +inf (frozen) /
 * 0 (information) for L at column m+1, and 0 elsewhere.
 *   llr       device, B x N FP32 channel LLRs (finite)
 *   opts      host, see pbp_decode_opts
 *   info_out  device, B x K uint8, the decided information bits
 *   iters_out device, B int32, iterations executed per frame
 *   pe_out    device, B int64, PE activations per frame (Section IV's
 *             computation count), or NULL
 *   soft_out  device, B x N FP32, or NULL: the posterior LLR of each source
 *             bit at exit (R + L at column m+1; +-inf inside frozen CSFGs)
 * Codes up to N = 4096 keep every message on chip (N <= 64: one wavefront
 * per frame, a row per lane, registers only; N = 128..512: one workgroup per
 * frame in LDS; N = 1024: one wavefront per frame, registers and LDS;
 * N = 2048, 4096: one workgroup of N/4 threads per frame, half the L
 * columns in VGPRs, the rest in LDS).  Longer
 * codes keep L in device memory.  The frame counter of the persistent
 * kernels and the message state of codes longer than 4096 come from the
 * stream's workspace (see the conventions above), so calls on different
 * streams may overlap, on one handle or several.  The message state takes
 * (m + 1) N floats per resident workgroup: 503 MB on 256 compute units at
 * N = 16384.
 * Errors: PBP_EINVAL (bad options, B < 0, NULL required pointer; checked
 * before any allocation), PBP_ENOMEM (the workspace cannot be allocated),
 * PBP_EDEVICE (launch failure). */
int32_t pbp_decode(const pbp_code *code, const float *llr, int64_t B,
                   const pbp_decode_opts *opts, uint8_t *info_out,
                   int32_t *iters_out, int64_t *pe_out, float *soft_out,
                   void *stream);

/* Free the decoder workspace of `stream` on the current device, after
 * synchronising that stream (a no-op when it has none).  The next decode on
 * the stream creates a new one.  Call it before destroying a stream that
 * decoded, so that a later stream created at the same address starts clean.
 * Errors: PBP_EDEVICE. */
int32_t pbp_workspace_release(void *stream);

/* pbp_decode for callers that cannot allocate device memory (code under
 * graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same decoding, arguments and results bit for bit, with the scratch of
 * the persistent kernels (the frame counter of the N = 1024, 2048 and 4096
 * kernels, the message state of longer codes) taken from a static 64 MiB
 * device array instead of the stream's workspace, and no allocation of any
 * kind.  Each GPU holds one such array until the process ends; codes longer
 * than 4096 run at most as many resident workgroups as state slots fit in
 * it (146 at N = 8192, 68 at N = 16384).  Every call on a GPU shares
 * that array, so calls that overlap on one GPU (two streams, or two
 * threads) race; order them on one stream.  B must be at most 2^30.
 * Errors: as pbp_decode; PBP_EINVAL also for B > 2^30, PBP_EDEVICE when the
 * array's address cannot be obtained. */
int32_t pbp_decode_noalloc(const pbp_code *code, const float *llr, int64_t B,
                           const pbp_decode_opts *opts, uint8_t *info_out,
                           int32_t *iters_out, int64_t *pe_out,
                           float *soft_out, void *stream);

/* The round-trip schedule, the other common reading of Section II-A's
 * schedule (pbp_decode runs the single left-to-right sweep): each iteration
 * computes every L output of eq. (1) for stages m, m-1, ..., 1 (from the L
 * just computed at column j+1 and the previous pass's R at column j), then
 * every R output for stages 1, ..., m (from the R just computed at column j
 * and this pass's L at column j+1).  Arguments, layouts, ownership and the
 * stop test as for pbp_decode (its frame counter also comes from the
 * stream's workspace); pe_out counts both passes, m N PE activations per
 * iteration.  opts->freezing must be 0 and N <= 2048.
 * Errors: as pbp_decode; PBP_EUNSUPPORTED for freezing or N > 2048. */
int32_t pbp_decode_round_trip(const pbp_code *code, const float *llr,
                              int64_t B, const pbp_decode_opts *opts,
                              uint8_t *info_out, int32_t *iters_out,
                              int64_t *pe_out, float *soft_out, void *stream);

/* pbp_decode with saturating b-bit fixed-point messages, the integer
 * arithmetic of a hardware decoder in which the paper counts a PE's cost
 * (Sections I and V; the paper fixes no format).  Every message lies in
 * [-Q, Q], Q = 2^(bits-1) - 1: the channel is clamp(round(LLR 2^frac))
 * (halves away from zero); eq. (1)'s scaled minimum is
 * sign sign ((a min(|x|, |y|) + 8) >> 4), a = round(16 alpha); its sums
 * saturate; +-Q replaces the +-inf of the frozen prior and of frozen CSFGs;
 * hard decisions take the exact sum's sign.  Same schedule, stop test,
 * freezing walk, iteration and PE counts as pbp_decode.  The scaled minimum
 * itself is not saturated (above 1, alpha can lift it past Q).
 *   bits      2..8 (the posteriors are returned as bytes); frac 0..16
 *   soft_out  device, B x N int8, or NULL: sat(R + L) at column m+1 (+-Q
 *             inside frozen CSFGs)
 * Every length runs the on-chip decoder pbp_decode uses for it, with the
 * integers held exactly in FP32 registers and LDS words (N >= 1024 take
 * frames from the stream's workspace counter: calls on one stream are
 * ordered, as for pbp_decode).
 * Other arguments as pbp_decode.  N <= 4096.
 * Errors: as pbp_decode; PBP_EUNSUPPORTED for N > 4096. */
int32_t pbp_decode_quant(const pbp_code *code, const float *llr, int64_t B,
                         const pbp_decode_opts *opts, int32_t bits,
                         int32_t frac, uint8_t *info_out, int32_t *iters_out,
                         int64_t *pe_out, int8_t *soft_out, void *stream);

/* Successive-cancellation decoding (the decoder whose scheduling tree
 * Section III maps onto the factor graph; its ML comparison with a frozen
 * CSFG is the argument of Lemma 1's use).  Source bits are decided in
 * increasing position order: a node over n positions with LLRs L decodes its
 * first half from f(L[i], L[i + n/2]) = sign * sign * min (exact, unscaled
 * min-sum), then its second half from L[i + n/2] + (1 - 2c) L[i] (one
 * rounding), c the first half's re-encoded bits; a leaf takes 0 at a frozen
 * position and [LLR < 0] otherwise.
 *   llr       device, B x N FP32 channel LLRs
 *   info_out  device, B x K uint8, the decided information bits
 *   leaf_out  device, B x N FP32, or NULL: the LLR reaching each leaf
 * B >= 0.  Errors: PBP_EINVAL, PBP_EDEVICE. */
int32_t pbp_decode_sc(const pbp_code *code, const float *llr, int64_t B,
                      uint8_t *info_out, float *leaf_out, void *stream);

/* ---- Mixed-code persistent decoding ----------------------------------
 * One batch may mix codes of different lengths and rates (each frame names
 * its code).  Persistent wavefronts drain a device work queue, each taking
 * the next frame when it finishes one.  Decoding per frame is that of
 * pbp_decode (same results bit for bit); only the schedule differs. */

/* Plan: the codes of a mixed batch, device buffers of the work queue and of
 * long codes' message state, and the launch configuration.  Calls on one
 * plan must be ordered on one stream (they share the queue). */
typedef struct pbp_mixed_plan pbp_mixed_plan;

/* Launch configuration.
 *  order         0: one launch for the whole batch: the queue takes frames
 *                   in the caller's order, and one kernel dispatches on
 *                   each frame's code length (every frame on one
 *                   wavefront; N >= 2048 with L in the wavefront's slot);
 *                1: frames grouped by code, longest code first: a device
 *                   counting sort (four small kernels), then one persistent
 *                   kernel per code, specialised for its length (N >= 2048
 *                   on 256-thread groups)
 *  waves_per_cu  resident wavefronts per compute unit, 1..16 (each decodes
 *                one frame at a time); under order 1, codes with
 *                N >= 2048 run waves_per_cu / 2 256-thread groups (at least
 *                1, at most 4) per compute unit.  No kernel is given more
 *                groups than its occupancy allows. */
typedef struct {
    int32_t order;
    int32_t waves_per_cu;
} pbp_mixed_config;

/* Create a plan for up to max_frames frames (1 .. 2^30) over ncodes code
 * handles (1..16, all on one device; they must outlive the plan).  Device
 * memory: the queue (4 B per frame) and, when a code has N >= 2048, one
 * message slot per resident wavefront ((m+1) 2^m floats for the longest
 * such code, 16 per compute unit).
 * Default configuration: {0, 16}.  Errors: PBP_EINVAL, PBP_ENOMEM,
 * PBP_EDEVICE. */
int32_t pbp_mixed_plan_create(const pbp_code *const *codes, int32_t ncodes,
                              int64_t max_frames, pbp_mixed_plan **out);

/* Release a plan (NULL is ignored); synchronises its device first. */
void pbp_mixed_plan_destroy(pbp_mixed_plan *plan);

int32_t pbp_mixed_plan_get_config(const pbp_mixed_plan *plan,
                                  pbp_mixed_config *cfg);
/* Errors: PBP_EINVAL for a configuration out of range. */
int32_t pbp_mixed_plan_set_config(pbp_mixed_plan *plan,
                                  const pbp_mixed_config *cfg);

/* Decode a mixed batch of B frames (B <= the plan's max_frames).
 *   code_of_frame  device, B int32: index into the plan's codes.  A frame
 *                  naming no code of the plan is not decoded: its iteration
 *                  (and PE) count is set to 0 and its bits are not written.
 *   llr_off        device, B int64: element offset of the frame's N FP32
 *                  LLRs in llr (any offset)
 *   info_off       device, B int64: byte offset of the frame's K decided
 *                  information bits in info_out
 *   llr            device FP32 LLR buffer (finite)
 *   opts           host, as for pbp_decode
 *   iters_out      device, B int32; pe_out device, B int64, or NULL
 * Ranges given by the offsets must lie inside the caller's buffers; output
 * ranges of different frames must not overlap.  Enqueues one persistent
 * kernel (order 0), or the four kernels of the sort and one persistent
 * kernel per code (order 1); no allocation, no memset, no host
 * synchronisation, so the call can be captured in a HIP graph and replayed
 * (the queue rewinds itself at the end of every launch).
 * Errors: PBP_EINVAL, PBP_EDEVICE. */
int32_t pbp_decode_mixed(pbp_mixed_plan *plan, const int32_t *code_of_frame,
                         const int64_t *llr_off, const int64_t *info_off,
                         int64_t B, const float *llr,
                         const pbp_decode_opts *opts, uint8_t *info_out,
                         int32_t *iters_out, int64_t *pe_out, void *stream);

/* Autotuner: time every candidate configuration (order 0/1 x 4, 8, 12 or
 * 16 wavefronts per compute unit) on the given batch, one untimed and `reps`
 * timed launches each, and keep the fastest in the plan (also written to
 * *best if not NULL).  Results are cached for the life of the process per
 * (device, the plan's (N, K) list, early_stop, freezing): a later call with
 * the same key launches nothing.  The batch's outputs are overwritten.
 * Synchronous.  Errors: as pbp_decode_mixed, PBP_EINVAL for reps < 1. */
int32_t pbp_mixed_plan_tune(pbp_mixed_plan *plan, const int32_t *code_of_frame,
                            const int64_t *llr_off, const int64_t *info_off,
                            int64_t B, const float *llr,
                            const pbp_decode_opts *opts, uint8_t *info_out,
                            int32_t *iters_out, int64_t *pe_out, int32_t reps,
                            void *stream, pbp_mixed_config *best);

/* Fill efficiency of the plan's last pbp_decode_mixed call: the resident
 * wavefronts' time spent decoding over (the largest launch's resident
 * wavefronts x the call's whole span, from the first wavefront's start to
 * the last one's end), from device timestamps; kernel tails and the gaps
 * between the per-code launches of order 1 count as idle.  Synchronises
 * `stream` first.  Errors: PBP_EINVAL, PBP_EDEVICE. */
int32_t pbp_mixed_plan_fill(pbp_mixed_plan *plan, void *stream, double *fill);

/* Unrolled BP with trainable scales (the decoder of eq. (1) unrolled over T
 * iterations, single sweep, no early stop and no freezing), for learning the
 * min-sum scale per iteration, stage and direction.  Iteration t, stage j:
 *   L^t_{a,j}   = aL g(L_a, L_b + R_b),   L^t_{b,j}   = L_b + aL g(L_a, R_a),
 *   R^t_{a,j+1} = aR g(R_a, L_b + R_b),   R^t_{b,j+1} = R_b + aR g(L_a, R_a),
 * g(x,y) = sign(x) sign(y) min(|x|,|y|), L = L^{t-1} at column j+1,
 * aL = alpha[t][j][0], aR = alpha[t][j][1].  With every scale equal this is
 * pbp_decode's iteration without early stop or freezing.  N <= 1024
 * (PBP_EUNSUPPORTED above).
 *   llr    device, B x N FP32 channel LLRs (finite)
 *   T      iterations, 1 <= T <= 65536
 *   alpha  device, T x m x 2 FP32 scales (finite and nonzero)
 *   out    device, B x N FP32, written: R^T at column m+1 (the posterior
 *          LLR of each source bit, without the prior)
 *   ckpt   device, T x B x (m-1) x N FP32, or NULL (inference): written with
 *          L at columns 2..m at the start of each iteration, for the
 *          backward pass.  Unused when N = 2.
 * Errors: PBP_EINVAL (B < 0, T out of range, NULL required pointer),
 * PBP_EUNSUPPORTED (N > 1024), PBP_EDEVICE. */
int32_t pbp_unrolled_forward(const pbp_code *code, const float *llr, int64_t B,
                             int32_t T, const float *alpha, float *out,
                             float *ckpt, void *stream);

/* Adjoint of pbp_unrolled_forward: gradients of sum(dout * out) with respect
 * to the scales and the channel LLRs.  d g(x,y)/dx = sign(y) when
 * |x| <= |y| (ties to x) and d g/dy = sign(x) otherwise; infinite messages
 * (the frozen prior and what it produces) are constants and take no
 * gradient.
 *   llr, alpha, T  as given to the forward call
 *   ckpt           device, the forward call's checkpoints (NULL if N = 2);
 *                  read only (the adjoint state stays on chip)
 *   dout           device, B x N FP32, the gradient at the output
 *   dalpha_frame   device, B x T x m x 2 FP32, written: each frame's
 *                  contribution to the scale gradient (workspace owned by
 *                  the caller; may be NULL only when B = 0)
 *   dalpha         device, T x m x 2 FP32, written: the sum over frames,
 *                  accumulated in FP64 in frame order (deterministic)
 *   dllr           device, B x N FP32, or NULL: gradient at the channel LLRs
 * Errors: as pbp_unrolled_forward. */
int32_t pbp_unrolled_backward(const pbp_code *code, const float *llr,
                              int64_t B, int32_t T, const float *alpha,
                              const float *ckpt, const float *dout,
                              float *dalpha_frame, float *dalpha, float *dllr,
                              void *stream);

#ifdef __cplusplus
}
#endif

#endif /* PBP_H */
