// Internal helpers shared by the librxphy translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stddef.h>

#include "../../include/rxphy.h"

namespace rxphy {

// ------------------------------------------------------------------ host side
// Records a message for rxphy_last_error() and returns `st`.
rxphy_status fail(rxphy_status st, const char* fmt, ...);
void clear_error();

// Shape validation shared by every entry point.
rxphy_status check_frame(const rxphy_frame* fr, int32_t n_frames);
rxphy_status check_ptr(const void* p, const char* name);

// Per-device one-time set-up (twiddle table upload).  Returns the table.
rxphy_status ensure_device_tables(const float2** tw4096);

inline rxphy_status launch_status(const char* what) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(RXPHY_EHIP, "%s: %s", what, hipGetErrorString(e));
  return RXPHY_OK;
}

// Launchers implemented per stage (device pointers, validated shapes).
rxphy_status launch_fft(const rxphy_frame& fr, int64_t n_tr, const float2* x, float2* out,
                        bool inverse, hipStream_t s);
rxphy_status launch_csi(const rxphy_frame& fr, int32_t nf, const float2* yf, const float2* pil,
                        float2* h, hipStream_t s);
// pil != nullptr: fused CSI (h unused; the channel is the LS estimate from
// the pilot symbol of yf and the pilots, bit-identical to the CSI stage's).
rxphy_status launch_detect(const rxphy_frame& fr, int32_t nf, const float2* h, const float2* yf,
                           const float2* pil, float2* xt, float* nu, uint8_t* flags,
                           rxphy_precision prec, float thr, void* ws, hipStream_t s);
// Fused CSI + detector for K = 16 (one pilot group per tile); ws holds
// group_workspace_bytes() of per-tile factor records (and, for BF16 / FP16,
// the list of subcarriers handed to the FP64 refinement).
// llr != nullptr: the demod stage fused in (xt may then be nullptr).
rxphy_status launch_detect_group(const rxphy_frame& fr, int32_t nf, const float2* yf, const float2* pil,
                                 float2* xt, float* nu, uint8_t* flags, float* llr, rxphy_precision prec,
                                 float thr, void* ws, hipStream_t s);
size_t group_workspace_bytes(const rxphy_frame& fr, int32_t nf, rxphy_precision prec = RXPHY_FP32);
// FP64 refinement of the listed subcarriers (rl[0] = count, then the entries
// f * n_sc + i): x0 the low-precision start (nullptr: start from 0), xt / llr
// written when not nullptr; with pil the channel is the LS estimate.
// FP64 refinement of the 16-user group path: one workgroup per listed tile.
rxphy_status launch_refine_group(const rxphy_frame& fr, int32_t nf, const float2* yf, const float2* pil,
                                 float2* xt, float* nu, uint8_t* flags, float* llr, const uint32_t* rl,
                                 hipStream_t s);
rxphy_status launch_refine(const rxphy_frame& fr, int32_t nf, const float2* h, const float2* yf,
                           const float2* pil, const float2* x0, float2* xt, float* nu, uint8_t* flags,
                           float* llr, const uint32_t* rl, hipStream_t s);
// Downlink: ZF precoder of 16 users from the uplink pilots (factor records in
// ws, as the fused detector's); QAM mapping; inverse transform with a prefix.
rxphy_status launch_precode(const rxphy_frame& fr, int32_t nf, const float2* yf, const float2* pil,
                            const void* src, int src_bits, float2* xf, uint8_t* flags, void* ws, bool reuse,
                            hipStream_t s);
rxphy_status launch_modulate(const rxphy_frame& fr, int64_t n_points, const uint8_t* bits, float2* sym,
                             hipStream_t s);
// the forward FFT of 16-bit I/Q samples (value = integer * scale)
rxphy_status launch_fft_sc16(const rxphy_frame& fr, int64_t n_tr, const short2* in, float scale, float2* out,
                             hipStream_t s);
// the inverse rows with prefix as 16-bit I/Q: round(sample * out_scale), saturated
rxphy_status launch_ifft_rows_sc16(const rxphy_frame& fr, int64_t n_rows, const float2* in, float out_scale,
                                   short2* out, hipStream_t s);
// |FFT| of n_rows F-point rows into float rows of F centred bins (TF plot)
rxphy_status launch_fft_mag(int n_fft, int64_t n_rows, const float2* in, float* out, hipStream_t s);
rxphy_status launch_ifft_rows(const rxphy_frame& fr, int64_t n_rows, const float2* in, float2* out,
                              hipStream_t s);
// Workspace of rxphy_csi_detect (the group path's records, else as detect).
size_t csi_detect_workspace_bytes(const rxphy_frame& fr, int32_t nf, rxphy_precision prec);
// Workspace of rxphy_csi_detect_demod: as rxphy_csi_detect, plus x_tilde
// (for a caller that does not want it) where the demod runs as its own stage.
size_t csi_detect_demod_workspace_bytes(const rxphy_frame& fr, int32_t nf, rxphy_precision prec);
bool group_path(const rxphy_frame& fr, rxphy_precision prec);
size_t detect_workspace_bytes(const rxphy_frame& fr, int32_t nf, rxphy_precision prec);
rxphy_status launch_demod(const rxphy_frame& fr, int32_t nf, const float2* xt, const float* nu,
                          float* llr, hipStream_t s);

inline int64_t sym_len(const rxphy_frame& f) { return (int64_t)f.cp_len + f.n_fft; }

// ---------------------------------------------------------------- device side
// threadIdx.x behind an empty asm: the tile bodies read it through this so that
// nothing derived from it is hoisted out of the persistent kernel's item loop
// (where it would stay live, and spill, across every stage's body).
__device__ __forceinline__ int tid_x() {
  int t = (int)threadIdx.x;
  asm volatile("" : "+v"(t));
  return t;
}

__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ float2 cmulc(float2 a, float2 b) {  // a * conj(b)
  return make_float2(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y);
}
__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 cscale(float2 a, float s) { return make_float2(a.x * s, a.y * s); }

// Least-squares channel estimate from one pilot subcarrier: y conj(p) / |p|^2
// (a zero pilot gives 0/0 = NaN, flagged downstream).  The CSI stage and the
// fused CSI + detector path both call this one expression, so they round alike.
__device__ __forceinline__ float2 ls_estimate(float2 y, float2 p) {
  const float pp = p.x * p.x + p.y * p.y;
  return make_float2((y.x * p.x + y.y * p.y) / pp, (y.y * p.x - y.x * p.y) / pp);
}


// Store that is not expected to be read again soon (global_store with the
// non-temporal hint): for outputs streamed once, such as the LLRs.
typedef float f32x2v __attribute__((ext_vector_type(2)));
__device__ __forceinline__ void store_stream2(float2* p, float2 v) {
  __builtin_nontemporal_store(f32x2v{v.x, v.y}, reinterpret_cast<f32x2v*>(p));
}

}  // namespace rxphy
