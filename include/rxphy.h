/*
 * librxphy: OFDM massive-MIMO uplink receiver on one MI355X (gfx950).
 *
 * The four forward calls are the DSP stages whose names (fft, csi, equal,
 * demod) open the paper's preamble.  The paper defines the segment FFT
 * (Section III-A1: a non-overlapping N_FFT-point FFT over consecutive I/Q
 * segments, F = N_FFT bins per segment; Section IV-D: 32-bit floating-point
 * I/Q, time-parallel across segments) and gives the other three stages only
 * their names; they follow the textbook per-subcarrier uplink model
 * y = H x + n (comb-pilot least squares, ZF / MMSE linear detection,
 * max-log soft demapping).
 *
 * Conventions shared by every call
 *  - All tensor pointers are DEVICE pointers to densely packed row-major
 *    arrays; complex values are interleaved (re, im) float32 pairs ("c64").
 *  - n_frames frames of the same shape are stacked on a leading [F] axis.
 *  - The used-subcarrier index i in [0, n_sc) is the fastest-varying index of
 *    every frequency-domain tensor.  Used subcarrier i sits on FFT bin
 *    (i - n_sc/2) mod n_fft (a centred block, DC kept).
 *  - Symbol 0 of every frame carries comb pilots: used subcarrier i carries
 *    user (i mod K)'s pilot.  Symbols 1 .. n_sym-1 carry data (D = n_sym-1).
 *  - Every call is asynchronous on `stream`, never synchronises and never
 *    allocates device memory; the caller owns every buffer.  The first call
 *    on a device uploads a 32 KiB twiddle table to it (a blocking copy).
 *  - Shape, range and pointer errors return a status before any launch and
 *    write nothing.  A failed launch returns RXPHY_EHIP.  Numerical trouble
 *    never fails a call: it is reported per subcarrier in `flags`.
 *  - Calls are thread-safe; calls that write the same buffers race.
 */
#ifndef RXPHY_H
#define RXPHY_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  RXPHY_OK = 0,
  RXPHY_EINVAL = 1,        /* bad pointer, size or shape                        */
  RXPHY_EUNSUPPORTED = 2,  /* shape outside the supported range (see below)     */
  RXPHY_EWORKSPACE = 3,    /* workspace missing or smaller than required        */
  RXPHY_EHIP = 4           /* a HIP runtime call or kernel launch failed        */
} rxphy_status;

typedef enum { RXPHY_ZF = 0, RXPHY_MMSE = 1 } rxphy_detector;

/* Calls take the precision as an int32_t holding one of these values; any
 * other value is rejected with RXPHY_EINVAL (rxphy_workspace_bytes returns 0). */
typedef enum { RXPHY_FP32 = 0, RXPHY_BF16 = 1, RXPHY_FP16 = 2 } rxphy_precision;

/* per-subcarrier flags written by rxphy_detect */
enum {
  RXPHY_FLAG_REFINED = 1u,    /* re-solved in FP64 (condition estimate above threshold)     */
  RXPHY_FLAG_BREAKDOWN = 2u,  /* Cholesky pivot <= 0 or not finite, or MMSE gain mu <= 0    */
  RXPHY_FLAG_NONFINITE = 4u   /* a channel or data input of this subcarrier was not finite  */
};

/* Shape of one frame.  Supported: 1 <= K <= 16, K <= M <= 64;
 * n_fft in {512, 1024, 2048, 4096}; K <= n_sc <= n_fft; 2 <= n_sym <= 17;
 * 0 <= cp_len <= n_fft; qam_bits in {2, 4, 6}; detector a rxphy_detector;
 * n0 > 0 and finite: noise variance per resource element per antenna after
 * the unscaled FFT. */
typedef struct {
  int32_t M;          /* base-station antennas                                   */
  int32_t K;          /* users                                                   */
  int32_t n_fft;      /* FFT size                                                */
  int32_t n_sc;       /* used subcarriers                                        */
  int32_t n_sym;      /* OFDM symbols per frame, symbol 0 = comb pilots          */
  int32_t cp_len;     /* cyclic-prefix samples skipped before each symbol        */
  int32_t qam_bits;   /* bits per QAM symbol: 2 (QPSK), 4 (16QAM), 6 (64QAM)      */
  int32_t detector;   /* RXPHY_ZF or RXPHY_MMSE                                  */
  float n0;           /* noise variance N0                                       */
} rxphy_frame;

/* fft stage (Section III-A1 segment FFT; `fft` macro of the preamble).
 * For each frame f, antenna m, symbol s: skip cp_len samples, take the
 * unscaled forward DFT X[k] = sum_n x[n] exp(-j 2 pi k n / n_fft) and keep
 * the used bins:  yf[f][m][s][i] = X[(i - n_sc/2) mod n_fft].
 *   x  : c64 [F][M][n_sym][cp_len + n_fft]   (read)
 *   yf : c64 [F][M][n_sym][n_sc]             (written)                       */
rxphy_status rxphy_fft(const rxphy_frame* frame, int32_t n_frames,
                       const void* x, void* yf, hipStream_t stream);

/* rxphy_fft from 16-bit fixed-point I/Q samples, the fronthaul format of
 * Section IV-D (processing stays FP32): sample = (x[..][0] + j x[..][1]) *
 * scale, converted exactly to FP32 when scale is a power of two (then the
 * result equals rxphy_fft of the converted samples bit for bit).
 *   x     : i16 [F][M][n_sym][cp_len + n_fft][2] (I, Q interleaved; read)
 *   scale : finite, > 0
 *   yf    : c64 [F][M][n_sym][n_sc] (written)                                */
rxphy_status rxphy_fft_sc16(const rxphy_frame* frame, int32_t n_frames, const int16_t* x, float scale,
                            void* yf, hipStream_t stream);

/* csi stage (`csi` macro): least-squares channel estimate from the comb
 * pilots of symbol 0, held over each pilot group.  G = n_sc / K groups;
 * subcarrier i belongs to group g(i) = min(i / K, G - 1) and
 *   h[f][m][u][i] = yf[f][m][0][q] * conj(p[f][q]) / |p[f][q]|^2,  q = g(i) K + u.
 * A zero pilot yields non-finite estimates (flagged later by rxphy_detect).
 *   yf     : c64 [F][M][n_sym][n_sc]  (only symbol 0 is read)
 *   pilots : c64 [F][n_sc]
 *   h      : c64 [F][M][K][n_sc]      (written)                              */
rxphy_status rxphy_csi(const rxphy_frame* frame, int32_t n_frames,
                       const void* yf, const void* pilots, void* h, hipStream_t stream);

/* equal stage (`equal` macro): per subcarrier, A = H^H H (ZF) or
 * H^H H + n0 I (MMSE); A = L L^H (Cholesky); z_s = H^H y_s and
 * x_hat_s = A^{-1} z_s for every data symbol s; d_u = [A^{-1}]_uu.
 *   ZF  : xt = x_hat,            nu_u = n0 d_u
 *   MMSE: mu_u = 1 - n0 d_u,     xt_u = x_hat_u / mu_u,   nu_u = (1 - mu_u) / mu_u
 * (unbiased symbol estimates and their post-detection noise variances).
 * Broken-down or non-finite subcarriers are erased: xt = 0, nu = +inf.
 * precision RXPHY_FP32: FP32 products on MFMA and an FP32 factorisation.
 * precision RXPHY_BF16 / RXPHY_FP16: the Gram and matched-filter products
 * take BF16 / FP16 operands (rounded to nearest even from FP32) with FP32
 * accumulation, the Cholesky runs in FP32, and every subcarrier whose
 * condition estimate ||A||_F tr(A^{-1}) exceeds cond_threshold (an upper
 * bound on kappa_2(A), at most K^1.5 times it), or whose low-precision
 * factorisation breaks down, is re-solved in FP64 from the FP32 inputs:
 * A = L L^H in FP64 and two steps of iterative refinement
 * x <- x + A^{-1} (b - A x), b = H^H y, from the low-precision solution
 * (from 0 where that is not finite); flag RXPHY_FLAG_REFINED.  A refined
 * subcarrier with a non-finite input is erased and flagged NONFINITE.
 * cond_threshold is ignored for FP32.
 *   h     : c64 [F][M][K][n_sc]
 *   yf    : c64 [F][M][n_sym][n_sc]   (symbols 1 .. n_sym-1 are read)
 *   xt    : c64 [F][K][n_sym-1][n_sc] (written)
 *   nu    : f32 [F][K][n_sc]          (written)
 *   flags : u8  [F][n_sc]             (written; may be NULL)
 *   ws    : workspace of rxphy_workspace_bytes(frame, n_frames, RXPHY_WS_DETECT,
 *           precision) bytes (NULL when that is 0)                            */
rxphy_status rxphy_detect(const rxphy_frame* frame, int32_t n_frames,
                          const void* h, const void* yf, void* xt, float* nu, uint8_t* flags,
                          int32_t precision, float cond_threshold,
                          void* ws, size_t ws_bytes, hipStream_t stream);

/* csi and equal stages fused: rxphy_csi followed by rxphy_detect on the same
 * frames, with the channel estimate formed on the fly from symbol 0 of yf and
 * the pilots instead of being written to and read back from an H tensor.
 * In FP32, and in BF16 / FP16 with fewer than 16 users, every output (xt, nu,
 * flags, and the refinement of the low-precision forms) is bit-identical to
 * the two-call sequence; the CSI stage's H is simply never stored.  With 16
 * users each 16-subcarrier tile is one pilot group and the call factors each
 * tile once (its A^{-1} in a 2304-byte record, applied to the matched filter
 * in FP32); in BF16 / FP16 that path forms the Gram matrix and the matched
 * filter from BF16 / FP16 operands on the 16x16x32 matrix products, its
 * condition estimate and FP64 refinement act per pilot group, and its results
 * agree with rxphy_detect's within the precision's error (bit-identical only
 * in FP32).  Arguments as rxphy_csi and rxphy_detect; the workspace is
 * rxphy_workspace_bytes(frame, n_frames, RXPHY_WS_CSI_DETECT, precision)
 * bytes, 8-byte aligned (the 16-user path's records, plus for BF16 / FP16 the
 * list of refined subcarriers: 4 bytes per subcarrier and 256 more), written
 * and read back within the call; the caller owns it and may reuse it once the
 * stream has passed the call.                                               */
rxphy_status rxphy_csi_detect(const rxphy_frame* frame, int32_t n_frames,
                              const void* yf, const void* pilots, void* xt, float* nu,
                              uint8_t* flags, int32_t precision, float cond_threshold,
                              void* ws, size_t ws_bytes, hipStream_t stream);

/* csi, equal and demod stages fused: rxphy_csi_detect followed by
 * rxphy_demod on its x_tilde and nu.  llr, nu and flags are bit-identical to
 * that sequence; x_tilde is written only if xt is not NULL.  With 16 users
 * the whole chain after the FFT is two kernels (the per-tile factorisation,
 * then the detector with the max-log demapping of each equalised symbol as it
 * is formed, so x_tilde need not round-trip through memory), plus in BF16 /
 * FP16 the FP64 refinement of the listed pilot groups, which demaps its own
 * symbols; otherwise the stages run one after the other.
 *   xt  : c64 [F][K][n_sym-1][n_sc] (written if not NULL)
 *   llr : f32 [F][K][n_sym-1][n_sc][qam_bits] (written)
 *   ws  : rxphy_workspace_bytes(frame, n_frames, RXPHY_WS_CSI_DETECT_DEMOD,
 *         precision) bytes, 8-byte aligned (caller-owned, reusable once the
 *         stream has passed the call)
 * Other arguments as rxphy_csi_detect.                                        */
rxphy_status rxphy_csi_detect_demod(const rxphy_frame* frame, int32_t n_frames,
                                    const void* yf, const void* pilots, void* xt, float* nu,
                                    uint8_t* flags, float* llr, int32_t precision,
                                    float cond_threshold, void* ws, size_t ws_bytes,
                                    hipStream_t stream);

/* rxphy_csi_detect_demod without a workspace argument, for callers that
 * cannot allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc).  It calls no allocating routine:
 * the workspace is a scratch array of RXPHY_NOALLOC_SCRATCH_BYTES (32 MiB)
 * inside the library, one per GPU, held until the process ends; its device
 * address is looked up on the first call on each device.  Arguments, outputs
 * and results are those of rxphy_csi_detect_demod (the same kernels run).
 * Returns RXPHY_EWORKSPACE, with nothing launched, when that call would need
 * more than RXPHY_NOALLOC_SCRATCH_BYTES of workspace (the 16-user FP32 path
 * needs 2304 bytes per 16-subcarrier tile: up to 194 frames of 64 x 16
 * antennas/users with 1200 subcarriers).  Every call on one GPU shares that
 * GPU's scratch, so calls that overlap in time on one GPU (on different
 * streams, or from different threads) race; calls ordered on one stream do
 * not.  Nothing in the scratch needs to start at zero: the kernels write every
 * byte they read within the call.                                           */
#define RXPHY_NOALLOC_SCRATCH_BYTES (32u << 20)
rxphy_status rxphy_csi_detect_demod_noalloc(const rxphy_frame* frame, int32_t n_frames,
                                            const void* yf, const void* pilots, void* xt, float* nu,
                                            uint8_t* flags, float* llr, int32_t precision,
                                            float cond_threshold, hipStream_t stream);

/* demod stage (`demod` macro): max-log LLRs over the Gray square-QAM set
 * with unit average energy (bits b0 .. b_{Q-1}; b0, b2, b4 select the
 * in-phase level, b1, b3, b5 the quadrature level):
 *   llr_j = (min_{c: b_j = 1} |xt - c|^2 - min_{c: b_j = 0} |xt - c|^2) / nu,
 * i.e. ln P(b_j = 0) / P(b_j = 1) under max-log; an erased stream (nu = +inf)
 * gives 0, and a non-finite coordinate of xt (nu finite) non-finite LLRs for
 * the bits of that axis.  Each minimum is
 * found in closed form per axis (the nearest level of the bit's set), so a
 * large |xt| keeps its large, finite LLR.
 *   xt  : c64 [F][K][n_sym-1][n_sc]
 *   nu  : f32 [F][K][n_sc]
 *   llr : f32 [F][K][n_sym-1][n_sc][qam_bits]  (written)                      */
rxphy_status rxphy_demod(const rxphy_frame* frame, int32_t n_frames,
                         const void* xt, const float* nu, float* llr, hipStream_t stream);

/* ---------------------------------------------------------------------------
 * Downlink (the transmit direction: the preamble's `modul`, `precode` and
 * `ifft` macros, beside the uplink stages).
 *
 * rxphy_modulate: Gray square-QAM mapping, the inverse of rxphy_demod's
 * labelling: bits b0 .. b_{Q-1} of each point (one byte per bit, b0 first,
 * any non-zero byte is a one) -> the unit-energy point with that label.
 *   bits : u8  [F][K][n_sym-1][n_sc][qam_bits]
 *   sym  : c64 [F][K][n_sym-1][n_sc] (written)                                 */
rxphy_status rxphy_modulate(const rxphy_frame* frame, int32_t n_frames, const uint8_t* bits, void* sym,
                            hipStream_t stream);

/* rxphy_precode: zero-forcing precoding with the uplink estimate
 * (reciprocity): for every subcarrier X = H A^-1 S, A = H^H H (detector ZF)
 * or H^H H + N0 I (MMSE: the regularised precoder), H the LS estimate of
 * rxphy_csi from symbol 0 of yf and the pilots, so that a downlink channel
 * H^H delivers S for ZF.  No power normalisation.  Every pilot group of K
 * subcarriers shares one H and one A, factored once: for K = 16 by the fused
 * detector's factor kernel (its records, in the workspace), for K < 16 by a
 * wave per group (no workspace).  A subcarrier whose
 * factorisation breaks down or whose estimate is not finite transmits zeros
 * and is flagged (RXPHY_FLAG_BREAKDOWN / _NONFINITE).
 *   yf     : c64 [F][M][n_sym][n_sc] (symbol 0 read)   pilots: c64 [F][n_sc]
 *   sym    : c64 [F][K][n_sym-1][n_sc]
 *   xf     : c64 [F][M][n_sym-1][n_sc] (written)
 *   flags  : u8  [F][n_sc] (written; may be NULL)
 *   ws     : rxphy_workspace_bytes(frame, n_frames, RXPHY_WS_PRECODE,
 *            RXPHY_FP32) bytes, 8-byte aligned (0 bytes, may be NULL, for
 *            K < 16)
 *   options: RXPHY_PRECODE_REUSE_FACTORS (K = 16): ws already holds the
 *            factor records that rxphy_csi_detect or rxphy_csi_detect_demod
 *            (FP32) left in its workspace for the same frames, yf, pilots and
 *            detector, the same Gram and Cholesky as the uplink (reciprocity);
 *            the factorisation is then skipped.  0: factor here.            */
enum { RXPHY_PRECODE_REUSE_FACTORS = 1u };   /* options of rxphy_precode */
rxphy_status rxphy_precode(const rxphy_frame* frame, int32_t n_frames, const void* yf, const void* pilots,
                           const void* sym, void* xf, uint8_t* flags, void* ws, size_t ws_bytes,
                           uint32_t options, hipStream_t stream);

/* rxphy_modulate_precode: rxphy_modulate then rxphy_precode in one call,
 * the symbols never stored: each point is mapped from its bit bytes where
 * the precoder reads it, so xf and flags equal those of the two calls bit
 * for bit.  Arguments as rxphy_precode, with
 *   bits : u8 [F][K][n_sym-1][n_sc][qam_bits] in place of sym               */
rxphy_status rxphy_modulate_precode(const rxphy_frame* frame, int32_t n_frames, const void* yf, const void* pilots,
                                    const uint8_t* bits, void* xf, uint8_t* flags, void* ws, size_t ws_bytes,
                                    uint32_t options, hipStream_t stream);

/* rxphy_ifft: inverse of rxphy_fft's used-bin transform, unscaled, with a
 * cyclic prefix: row r of xf (n_sc used subcarriers) becomes
 * x[r][cp_len + n] = sum_i xf[r][i] exp(+j 2 pi bin(i) n / N), n = 0..N-1,
 * and x[r][0 .. cp_len-1] repeats its last cp_len samples; so rxphy_fft of
 * the result returns N xf.  Rows are independent (frame->n_sym is not used).
 *   xf : c64 [n_rows][n_sc]     x : c64 [n_rows][cp_len + n_fft] (written)    */
rxphy_status rxphy_ifft(const rxphy_frame* frame, int64_t n_rows, const void* xf, void* x, hipStream_t stream);

/* rxphy_ifft with the time samples as 16-bit I/Q for the radio (the
 * fronthaul format of Section IV-D): each component of a sample becomes
 * round(value * (1 / scale)) to nearest even in FP32, saturated to
 * [-32768, 32767]; that is the FP32 sample rxphy_ifft writes, quantised.
 *   xf : c64 [n_rows][n_sc]   x : i16 [n_rows][cp_len + n_fft][2] (written)
 *   scale : finite, > 0 (the value of one integer step)                      */
rxphy_status rxphy_ifft_sc16(const rxphy_frame* frame, int64_t n_rows, const void* xf, float scale, int16_t* x,
                            hipStream_t stream);

/* Intermediate results of the forward stages that rxphy_backward may reuse;
 * any member may be NULL, in which case it is recomputed into the workspace
 * (xt and nu are used only as a pair: if either is NULL both are recomputed
 * with the FP32 detector).  Each must be the output of the FP32 forward call
 * on the same x and pilots (rxphy_fft, rxphy_csi, rxphy_detect); the
 * Cholesky factors are never saved (always recomputed from h).             */
typedef struct {
  const void* yf;    /* c64 [F][M][n_sym][n_sc]    */
  const void* h;     /* c64 [F][M][K][n_sc]        */
  const void* xt;    /* c64 [F][K][n_sym-1][n_sc]  */
  const float* nu;   /* f32 [F][K][n_sc]           */
} rxphy_saved;

/* Adjoint of the whole forward map x -> llr (FP32 forward), for gradients
 * with PyTorch's complex convention grad = dL/dRe + j dL/dIm.  The paper
 * differentiates nothing: this call is the exact derivative of the forward
 * map the four stage calls above define (wherever no argmin of the max-log
 * demapper switches), the differentiable form of the receiver through
 * demod -> equalise -> ZF / MMSE -> CSI -> FFT.  Given
 * dllr = dL/dllr it runs the demod adjoint (through the argmin points, ties
 * to the lowest point index, and through nu), the detector adjoint
 *   dL/dY = H V,  dL/dH = Y V^H - H (X_hat V^H + V X_hat^H + 2 A^{-1} diag(e) A^{-1})
 * (V = A^{-1} dL/dx_hat; e the weights of d_u), the CSI adjoint (pilot-group
 * sums times p / |p|^2 into symbol 0) and the inverse-direction unscaled DFT
 * of the used-bin gradient into the samples (cyclic-prefix samples get 0).
 * The Cholesky factors are always recomputed, never stored.
 *   x      : c64 [F][M][n_sym][cp_len + n_fft]   pilots: c64 [F][n_sc]
 *   saved  : may be NULL
 *   dllr   : f32 [F][K][n_sym-1][n_sc][qam_bits]
 *   dx     : c64 like x (written)
 *   dh     : c64 [F][M][K][n_sc] gradient w.r.t. the channel estimate (written; may be NULL)
 *   ws     : rxphy_workspace_bytes(frame, n_frames, RXPHY_WS_BACKWARD, RXPHY_FP32) bytes */
rxphy_status rxphy_backward(const rxphy_frame* frame, int32_t n_frames,
                            const void* x, const void* pilots, const rxphy_saved* saved,
                            const float* dllr, void* dx, void* dh,
                            void* ws, size_t ws_bytes, hipStream_t stream);

enum {
  RXPHY_WS_DETECT = 0,
  RXPHY_WS_BACKWARD = 1,
  RXPHY_WS_CSI_DETECT = 2,
  RXPHY_WS_CSI_DETECT_DEMOD = 3,
  RXPHY_WS_PRECODE = 4
};

/* Workspace bytes needed by rxphy_detect (which = RXPHY_WS_DETECT),
 * rxphy_backward (RXPHY_WS_BACKWARD), rxphy_csi_detect (RXPHY_WS_CSI_DETECT),
 * rxphy_csi_detect_demod (RXPHY_WS_CSI_DETECT_DEMOD) or rxphy_precode
 * (RXPHY_WS_PRECODE); 0 if none, or if the shape or the precision is invalid.  */
size_t rxphy_workspace_bytes(const rxphy_frame* frame, int32_t n_frames, int32_t which,
                             int32_t precision);

/* ---------------------------------------------------------------------------
 * Batched uneven frames.  The paper batches nothing across frames (its
 * Section IV-D spreads one stream's FFT segments over threads); this is the
 * batched form of the four stage calls above, defined frame by frame as
 * their results, for frames of differing shape.  A plan holds such frames
 * (each one a valid rxphy_frame) and runs all four forward stages of all of
 * them in ONE persistent launch: a fixed grid of workgroups pulls work items (a group of
 * FFT segments, of CSI tiles, of detector subcarrier tiles or of demod
 * elements of one frame) from a device queue in stage-major order, and an
 * item of stage s of frame f starts once every item of stage s-1 of frame f
 * has finished (per-frame stage counters).  Each frame's results are those of
 * the four single-frame calls (FP32 detector) on that frame, bit for bit when
 * the frame's detector uses the same K padding as rxphy_detect.
 *
 * Buffers are packed: frame f's tensor T (laid out as in the single-frame
 * calls with F = 1) starts at byte offset offsets[f].T of the one buffer for
 * T; every offset is a multiple of 256.  rxphy_plan_layout gives the offsets
 * and the buffer sizes.  Plans own a small device allocation (descriptor
 * table, work list, counters) made by rxphy_plan_create; running a plan
 * allocates nothing.  Two runs of one plan must not overlap in time (they
 * share the counters); different plans are independent.
 * ------------------------------------------------------------------------- */

typedef struct rxphy_plan rxphy_plan;   /* opaque */

/* Work-item sizes of one frame (0 = default).  Any values >= 1 give the same
 * results except det_kp, which changes the detector's arithmetic padding. */
typedef struct {
  int32_t fft_iters;   /* FFT item = fft_iters rounds of max(1, 2048 / n_fft) segments                 */
  int32_t csi_tiles;   /* CSI item = csi_tiles consecutive (antenna, 512-subcarrier) tiles              */
  int32_t det_tiles;   /* detector item = det_tiles consecutive 16-subcarrier tiles                     */
  int32_t det_kp;      /* K padding of the detector: 0 = smallest of {4, 8, 16} >= K, else 4, 8 or 16   */
  int32_t dem_groups;  /* demod item = dem_groups x 256 consecutive (user, subcarrier) columns          */
} rxphy_tiles;

enum {
  RXPHY_STAGE_FFT = 1, RXPHY_STAGE_CSI = 2, RXPHY_STAGE_DETECT = 4, RXPHY_STAGE_DEMOD = 8,
  RXPHY_STAGE_ALL = 15
};

typedef struct {
  int32_t stages;      /* RXPHY_STAGE_* mask of the stages to run (0 = all); a stage left out is
                          not waited for, so its outputs must already be in the buffers          */
  int32_t grid;        /* workgroups of the persistent launch (0 = every resident slot)       */
  uint32_t spin_limit; /* polls of a stage counter (about 0.1 us apart) before a wait gives up
                          (0 = 2^22, about half a second)                                   */
  int32_t fuse_csi;    /* 1: the CSI stage runs inside the detector items, which form the LS
                          estimate from the pilot symbol of yf and the pilots (as
                          rxphy_csi_detect does) and wait for the frame's FFT items; H is
                          never written (buffers.h may be NULL) and the CSI stage has no
                          items.  Every other output is bit-identical to the staged plan's.
                          0: four stages, H written.                                       */
  int32_t fuse_demod;  /* 1: the demod stage runs inside the detector items, which demap each
                          tile from x_tilde and nu held in LDS (the demod stage's arithmetic,
                          so the LLRs are bit-identical); x_tilde is never written
                          (buffers.xt may be NULL) and the demod stage has no items.
                          0: x_tilde written and demapped by demod items.                  */
} rxphy_plan_options;

/* Byte offsets of one frame's tensors in the packed buffers (or, for the
 * totals, the byte size of each buffer). */
typedef struct {
  int64_t x, pilots, yf, h, xt, nu, flags, llr;
} rxphy_offsets;

/* Device pointers of the packed buffers (flags may be NULL). */
typedef struct {
  const void* x;
  const void* pilots;
  void* yf;
  void* h;
  void* xt;
  float* nu;
  uint8_t* flags;
  float* llr;
} rxphy_batch;

/* Status bits of rxphy_plan_device_status */
enum { RXPHY_PLAN_WAIT_TIMEOUT = 1u };

/* Validates every frame (1 <= n_frames <= 16384), sizes the work items
 * (tiles: n_frames entries or NULL for defaults; options may be NULL) and
 * uploads the descriptor table and work list to the current device.        */
rxphy_status rxphy_plan_create(const rxphy_frame* frames, int32_t n_frames, const rxphy_tiles* tiles,
                               const rxphy_plan_options* options, rxphy_plan** plan);
/* per_frame: n_frames entries (may be NULL); totals: buffer sizes (may be NULL) */
rxphy_status rxphy_plan_layout(const rxphy_plan* plan, rxphy_offsets* per_frame, rxphy_offsets* totals);
/* Number of work items per stage (counts[4], FFT .. demod) and the grid. */
rxphy_status rxphy_plan_info(const rxphy_plan* plan, int64_t* counts, int32_t* grid);
/* Runs the plan on `stream` (a counter-reset kernel, then the persistent
 * kernel; no memset and no allocation, so the call may be stream-captured). */
rxphy_status rxphy_plan_forward(rxphy_plan* plan, const rxphy_batch* buffers, hipStream_t stream);
/* Builds (or rebuilds) a hipGraph of the same two launches bound to
 * `buffers`, owned by the plan; rxphy_plan_replay launches it on `stream`. */
rxphy_status rxphy_plan_graph(rxphy_plan* plan, const rxphy_batch* buffers);
rxphy_status rxphy_plan_replay(rxphy_plan* plan, hipStream_t stream);
/* Reads the device status word of the last run with a blocking copy; call it
 * after that run has completed (e.g. after synchronising its stream).
 * 0 = clean; RXPHY_PLAN_WAIT_TIMEOUT = a dependency wait hit spin_limit and
 * the results of that run are not to be trusted. */
rxphy_status rxphy_plan_device_status(rxphy_plan* plan, uint32_t* status);
void rxphy_plan_destroy(rxphy_plan* plan);

/* ---------------------------------------------------------------------------
 * Real-time streaming (Section III-B: a task must finish before the next one
 * becomes available, for at least 99 % of tasks; Section IV-D: a ping-pong
 * buffer between the arriving samples and their processing, whose depth sets
 * the latency budget).  A stream holds `depth` slots (2 = ping-pong); each
 * slot owns a HIP stream (default priority), a completion event and the
 * device buffers of one task of n_frames frames.  A task is rxphy_fft
 * followed by rxphy_csi_detect_demod (FP32) on its frames.
 *
 * Host I/O streams (host_io = 1) also own pinned host buffers per slot: the
 * producer writes the task's samples and pilots there, submit copies them in,
 * runs the task and copies llr, nu and flags back into the slot's pinned
 * outputs.  Device-resident streams (host_io = 0) take the task's input and
 * output device pointers at submit (samples already in HBM).
 *
 * The slots are handed out in turn: acquire waits until the next slot's
 * previous task has completed (back-pressure), the producer fills it and
 * submits it.  A completion thread owned by the stream polls the slots'
 * events and records each task's latency = completion time - arrival time
 * (steady clock, rxphy_clock_ns), in submission order.  The outputs of a host
 * I/O slot stay valid until that slot is submitted again.  One producer
 * thread per stream.
 * ------------------------------------------------------------------------- */

typedef struct rxphy_stream rxphy_stream;   /* opaque */

/* Pinned host buffers of one slot of a host I/O stream (layouts as in the
 * single-frame calls, F = n_frames). */
typedef struct {
  void* x;          /* c64 (or i16 pairs) [F][M][n_sym][cp_len + n_fft]  input */
  void* pilots;     /* c64 [F][n_sc]                      input  */
  float* llr;       /* f32 [F][K][n_sym-1][n_sc][qam_bits] output */
  float* nu;        /* f32 [F][K][n_sc]                   output */
  uint8_t* flags;   /* u8  [F][n_sc]                      output */
} rxphy_stream_host;

/* Latency summary.  Percentiles are nearest-rank: p-th = the ceil(p n / 100)-th
 * smallest value, so p99_us <= bound_us exactly when at least 99 % of the
 * tasks met the bound (meets_99 = 1). */
typedef struct {
  int64_t count;      /* tasks summarised                                 */
  int64_t on_time;    /* tasks with latency <= bound_us                   */
  int32_t meets_99;   /* 100 * on_time >= 99 * count (and count > 0)      */
  double p50_us, p99_us, max_us, mean_us;
} rxphy_latency_summary;

/* Creates a stream on the current device: 1 <= n_frames <= 65535,
 * 1 <= depth <= 8, host_io 0 or 1.  sc16_scale = 0: the samples x are
 * complex64; sc16_scale > 0: they are 16-bit I/Q pairs (rxphy_fft_sc16's
 * layout and scale), half the bytes to move.  Arguments are validated before
 * any HIP call; allocation failures return RXPHY_EHIP with nothing left
 * allocated. */
rxphy_status rxphy_stream_create(const rxphy_frame* frame, int32_t n_frames, int32_t depth, int32_t host_io,
                                 float sc16_scale, rxphy_stream** stream);
/* Pinned host buffers of `slot` (host I/O streams only). */
rxphy_status rxphy_stream_host_buffers(rxphy_stream* stream, int32_t slot, rxphy_stream_host* host);
/* Waits until the next slot in turn is free and hands it to the caller. */
rxphy_status rxphy_stream_acquire(rxphy_stream* stream, int32_t* slot);
/* Enqueues the task of an acquired slot.  arrival_ns: the time the task's
 * samples became available (rxphy_clock_ns; 0 = now).  Device-resident
 * streams pass x, pilots, llr and nu (flags may be NULL) as device pointers
 * in the single-frame layouts; host I/O streams pass NULL for all five.  A
 * rejected submit leaves the slot acquired. */
rxphy_status rxphy_stream_submit(rxphy_stream* stream, int32_t slot, int64_t arrival_ns, const void* x,
                                 const void* pilots, float* llr, float* nu, uint8_t* flags);
/* Waits for every submitted task; returns RXPHY_EHIP if a task failed on
 * the device. */
rxphy_status rxphy_stream_drain(rxphy_stream* stream);
/* Latencies (microseconds) of the submitted tasks in submission order, NaN
 * for tasks not yet completed: copies min(cap, n) values, *n = tasks so far. */
rxphy_status rxphy_stream_latencies(rxphy_stream* stream, double* lat_us, int64_t cap, int64_t* n);
/* Forgets the recorded latencies (no task may be outstanding). */
rxphy_status rxphy_stream_reset_latencies(rxphy_stream* stream);
/* Drains, stops the completion thread and frees every buffer. */
void rxphy_stream_destroy(rxphy_stream* stream);
/* The steady clock the stream stamps completions with, in nanoseconds. */
int64_t rxphy_clock_ns(void);
/* Summary of n latencies against bound_us (host only; NaN entries are
 * rejected with RXPHY_EINVAL; n = 0 gives a zero summary). */
rxphy_status rxphy_latency_summarize(const double* lat_us, int64_t n, double bound_us, rxphy_latency_summary* out);

/* ---------------------------------------------------------------------------
 * Spectrum sensing (the paper's own pipeline, Sections III-A1 and IV-B):
 * a capture of T consecutive non-overlapping F-sample segments becomes a TF
 * plot of FFT magnitudes (row = segment, column c = bin (c - F/2) mod F, no
 * normalisation); its column sums are the PSD, smoothed by a Savitzky-Golay
 * filter (mirror-reflected edges); the lowest local minimum of the smoothed
 * PSD (interior points no larger than both neighbours; the global minimum if
 * there is none) is the noise floor N0 and theta_PSD = psd_factor * N0;
 * columns whose PSD is below theta_PSD are pruned; each retained column is
 * binarised at Otsu's threshold (the bin that maximises the between-class
 * variance of a `bins`-bin histogram over the column's [min, max], ties to
 * the lower bin, decided exactly in integers; a value's bin is
 * min(bins-1, floor((v - min) * (bins / (max - min)))) in FP32); the mask
 * then gets one 3x3 closing, one 3x3 opening and one 1x3 opening along
 * frequency, in that order (all-ones elements, neighbours inside the plot
 * only; the last one leaves a 3x3 opening unchanged); its
 * 4-connected components give one inclusive box (t0, f0, t1, f1) each,
 * listed in raster order of each component's first pixel.
 * ------------------------------------------------------------------------- */

typedef struct {
  int32_t n_fft;       /* F: plot width, 512, 1024, 2048 or 4096             */
  int32_t n_rows;      /* T: segments per plot, 3 .. 4096                    */
  int32_t sg_window;   /* Savitzky-Golay window: odd, 3 .. 63, <= F           */
  int32_t sg_order;    /* polynomial order: 0 .. min(6, sg_window - 1)        */
  float psd_factor;    /* theta_PSD = psd_factor * N0, > 0                    */
  int32_t bins;        /* Otsu histogram bins, 2 .. 256                       */
} rxphy_sense_config;

/* Intermediate results, each optional (NULL = kept in the workspace). */
typedef struct {
  float* tf;           /* f32 [P][T][F] magnitudes                            */
  float* psd;          /* f32 [P][F] column sums                              */
  float* psd_smooth;   /* f32 [P][F]                                          */
  float* floor;        /* f32 [P][2]: N0, theta_PSD                           */
  int32_t* otsu_bin;   /* i32 [P][F]: the threshold bin; -1 for a pruned column
                          or one whose values all fall into one bin          */
  uint8_t* mask;       /* u8 [P][T][F] after binarisation (0 / 1)             */
  uint8_t* mask_mo;    /* u8 [P][T][F] after the morphological operations    */
} rxphy_sense_outputs;

/* Workspace bytes of rxphy_sense for n_plots plots (0 if cfg is invalid). */
size_t rxphy_sense_workspace_bytes(const rxphy_sense_config* cfg, int32_t n_plots);

/* The whole pipeline over n_plots captures (1 .. 65535).
 *   x        : c64 [P][T][F] samples (device)
 *   out      : optional intermediates (may be NULL)
 *   n_boxes  : i32 [P] number of components of each plot (device; may exceed
 *              max_boxes, in which case only the first max_boxes are written)
 *   boxes    : i32 [P][max_boxes][4] (t0, f0, t1, f1) (device)
 *   ws       : rxphy_sense_workspace_bytes bytes, 256-byte aligned (device)
 * Asynchronous on `stream`; no allocation, no synchronisation. */
rxphy_status rxphy_sense(const rxphy_sense_config* cfg, int32_t n_plots, const void* x,
                         const rxphy_sense_outputs* out, int32_t* n_boxes, int32_t* boxes, int32_t max_boxes,
                         void* ws, size_t ws_bytes, hipStream_t stream);

/* The Savitzky-Golay smoothing weights rxphy_sense applies to the PSD
 * (Section IV-B names the filter; window and order are the config's):
 * weights[k + window/2], k = -window/2 .. window/2, is the value at 0 of the
 * least-squares polynomial of degree `order` through unit samples at offset
 * k, i.e. the smoothed value is sum_k weights[k + window/2] psd[i + k].
 * Computed on the host in FP64 and rounded to FP32 (the same routine the
 * pipeline uses).  window odd in 3 .. 63, 0 <= order <= 6, order < window;
 * weights: `window` floats (host).  Host only; no GPU needed. */
rxphy_status rxphy_savgol_weights(int32_t window, int32_t order, float* weights);

/* Detection metrics of Section III-A on the host: the IoU matrix of ground
 * truth boxes against detections (inclusive pixel boxes), N_t = ground
 * truths whose best IoU exceeds theta_iou, N_f = detections whose best IoU
 * is below it, P_d = N_t / N_gt and P_fa = N_f / N_d (NaN when the
 * denominator is 0), mean_iou = mean over ground truths of their best IoU
 * (0 when either list is empty).  iou may be NULL (else n_gt x n_det). */
typedef struct {
  int32_t n_t, n_f;
  double p_d, p_fa, mean_iou;
} rxphy_detection_metrics;
rxphy_status rxphy_box_metrics(const int32_t* gt, int32_t n_gt, const int32_t* det, int32_t n_det,
                               double theta_iou, double* iou, rxphy_detection_metrics* out);

/* Human-readable name of a status, and thread-local detail of the last
 * non-OK status returned on the calling thread (empty string if none). */
/* ---------------------------------------------------------------------------
 * Channel decoding (the preamble's `dec` stage, with its LDPC notation:
 * lifting size Z_c, code-block size K_cb, code rate R).  The paper defines
 * no decoder; this is layered belief propagation with the normalised
 * min-sum check rule over a quasi-cyclic code given by its base matrix.
 *
 * Code: base matrix B [mb][nb] (host, row-major int16): entry -1 is a
 * z x z zero block, entry s in [0, z) the z x z identity with its columns
 * cyclically shifted by s (row r has its one in column (r + s) mod z).
 * Codeword length N = nb z; check i z + r involves bit c z + (r + B[i][c]) mod z
 * of every block column c with B[i][c] >= 0.  Supported: 1 <= z <= 384,
 * 1 <= mb <= 64, mb < nb, N <= 38400, every block row with 2 to 27 non-zero
 * blocks.  rxphy_ldpc_code_create validates B (RXPHY_EINVAL /
 * RXPHY_EUNSUPPORTED before any HIP call) and uploads its edge table (a
 * small device allocation owned by the code, freed by destroy); B is copied.
 *
 * Decoding (rxphy_ldpc_decode), per codeword independently: L starts at the
 * channel LLRs (ln P(0) / P(1)), every check-to-bit message R at 0; one
 * iteration visits the block rows in order 0 .. mb-1 (one layer each, its z
 * checks in parallel) and for each check and each of its bits v (block
 * columns in increasing order) sets Q = L_v - R,
 *   R_new = alpha * (product of the signs of the check's other Q)
 *                 * (smallest |Q| among the check's other bits)   (sgn 0 = +1),
 *   L_v = Q + R_new,
 * every operation rounded once in FP32.  The syndrome of the hard decisions
 * (bit 1 iff L < 0) is tested before the first iteration and after each one,
 * and decoding stops at the first zero syndrome or after max_iter iterations.
 * Inputs must be finite (a non-finite LLR propagates).
 *   llr   : f32 [n_cw][N] (device)      post  : f32 [n_cw][N] posterior LLRs (written)
 *   bits  : u8 [n_cw][N] hard decisions (written; may be NULL)
 *   iters : i32 [n_cw] iterations run, 0 if the channel word was a codeword
 *           (written; may be NULL)
 *   ws    : rxphy_ldpc_workspace_bytes(code, n_cw) bytes, 4-byte aligned:
 *           the compressed messages (two scaled minima and one word of signs
 *           and argmin per check), written and read within the call
 * max_iter >= 0; alpha finite and > 0 (1 = plain min-sum).                  */
typedef struct rxphy_ldpc_code rxphy_ldpc_code;   /* opaque */
rxphy_status rxphy_ldpc_code_create(const int16_t* base, int32_t mb, int32_t nb, int32_t z,
                                    rxphy_ldpc_code** code);
void rxphy_ldpc_code_destroy(rxphy_ldpc_code* code);
size_t rxphy_ldpc_workspace_bytes(const rxphy_ldpc_code* code, int32_t n_cw);
rxphy_status rxphy_ldpc_decode(const rxphy_ldpc_code* code, int32_t n_cw, const float* llr, int32_t max_iter,
                               float alpha, float* post, uint8_t* bits, int32_t* iters, void* ws,
                               size_t ws_bytes, hipStream_t stream);

const char* rxphy_status_string(rxphy_status status);
const char* rxphy_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* RXPHY_H */
