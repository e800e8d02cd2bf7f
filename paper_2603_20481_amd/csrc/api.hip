// Host side of the C ABI: validation, error reporting, per-device tables and
// the public entry points that dispatch to the stage launchers.
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <vector>

#include "abi_checks.h"
#include "common.h"

namespace rxphy {

// precode.hip: the precoder for K < 16 (one wave per pilot group)
rxphy_status launch_precode_general(const rxphy_frame& fr, int32_t nf, const float2* yf, const float2* pil,
                                    const void* src, int src_bits, float2* xf, uint8_t* flags, hipStream_t s);

static thread_local char g_err[512];

rxphy_status fail(rxphy_status st, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
  return st;
}

void clear_error() { g_err[0] = 0; }

rxphy_status check_ptr(const void* p, const char* name) {
  if (!p) return fail(RXPHY_EINVAL, "%s is NULL", name);
  return RXPHY_OK;
}

rxphy_status check_frame(const rxphy_frame* fr, int32_t n_frames) {
  if (!fr) return fail(RXPHY_EINVAL, "frame is NULL");
  if (n_frames < 0) return fail(RXPHY_EINVAL, "n_frames = %d < 0", n_frames);
  const rxphy_frame& f = *fr;
  if (f.K < 1 || f.M < 1) return fail(RXPHY_EINVAL, "M = %d, K = %d must be >= 1", f.M, f.K);
  if (f.K > 16) return fail(RXPHY_EUNSUPPORTED, "K = %d > 16", f.K);
  if (f.M > 64) return fail(RXPHY_EUNSUPPORTED, "M = %d > 64", f.M);
  if (f.K > f.M) return fail(RXPHY_EINVAL, "K = %d > M = %d", f.K, f.M);
  if (f.n_fft != 512 && f.n_fft != 1024 && f.n_fft != 2048 && f.n_fft != 4096)
    return fail(f.n_fft > 0 && (f.n_fft & (f.n_fft - 1)) == 0 ? RXPHY_EUNSUPPORTED : RXPHY_EINVAL,
                "n_fft = %d not in {512, 1024, 2048, 4096}", f.n_fft);
  if (f.n_sc < f.K || f.n_sc > f.n_fft)
    return fail(RXPHY_EINVAL, "n_sc = %d outside [K, n_fft] = [%d, %d]", f.n_sc, f.K, f.n_fft);
  if (f.n_sym < 2) return fail(RXPHY_EINVAL, "n_sym = %d < 2", f.n_sym);
  if (f.n_sym > 17) return fail(RXPHY_EUNSUPPORTED, "n_sym = %d > 17", f.n_sym);
  if (f.cp_len < 0 || f.cp_len > f.n_fft)
    return fail(RXPHY_EINVAL, "cp_len = %d outside [0, n_fft]", f.cp_len);
  if (f.qam_bits != 2 && f.qam_bits != 4 && f.qam_bits != 6)
    return fail(RXPHY_EINVAL, "qam_bits = %d not in {2, 4, 6}", f.qam_bits);
  if (f.detector != RXPHY_ZF && f.detector != RXPHY_MMSE)
    return fail(RXPHY_EINVAL, "detector = %d", f.detector);
  if (!(std::isfinite(f.n0) && f.n0 > 0.0f)) return fail(RXPHY_EINVAL, "n0 = %g must be finite and > 0", f.n0);
  return RXPHY_OK;
}

// Twiddle table exp(-j 2 pi t / 4096), t = 0..4095, computed in FP64 and
// rounded once to FP32; every FFT size indexes it with a stride.
static __device__ float2 g_tw4096[4096];

rxphy_status ensure_device_tables(const float2** tw) {
  static std::mutex mu;
  static std::vector<const float2*> done;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return fail(RXPHY_EHIP, "hipGetDevice failed");
  std::lock_guard<std::mutex> lk(mu);
  if ((int)done.size() <= dev) done.resize(dev + 1, nullptr);
  if (!done[dev]) {
    std::vector<float2> h(4096);
    const double two_pi = 6.283185307179586476925286766559;
    for (int t = 0; t < 4096; ++t) {
      double a = -two_pi * (double)t / 4096.0;
      h[t] = make_float2((float)std::cos(a), (float)std::sin(a));
    }
    hipError_t e = hipMemcpyToSymbol(HIP_SYMBOL(g_tw4096), h.data(), sizeof(float2) * 4096, 0,
                                     hipMemcpyHostToDevice);
    if (e != hipSuccess) return fail(RXPHY_EHIP, "twiddle upload: %s", hipGetErrorString(e));
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(g_tw4096));
    if (e != hipSuccess) return fail(RXPHY_EHIP, "twiddle address: %s", hipGetErrorString(e));
    done[dev] = (const float2*)p;
  }
  *tw = done[dev];
  return RXPHY_OK;
}

}  // namespace rxphy

using namespace rxphy;

extern "C" {

const char* rxphy_status_string(rxphy_status st) {
  switch (st) {
    case RXPHY_OK: return "RXPHY_OK";
    case RXPHY_EINVAL: return "RXPHY_EINVAL";
    case RXPHY_EUNSUPPORTED: return "RXPHY_EUNSUPPORTED";
    case RXPHY_EWORKSPACE: return "RXPHY_EWORKSPACE";
    case RXPHY_EHIP: return "RXPHY_EHIP";
  }
  return "RXPHY_UNKNOWN";
}

const char* rxphy_last_error(void) { return g_err; }

rxphy_status rxphy_fft(const rxphy_frame* frame, int32_t n_frames, const void* x, void* yf,
                       hipStream_t stream) {
  clear_error();
  rxphy_status st = check_frame(frame, n_frames);
  if (st) return st;
  if (n_frames == 0) return RXPHY_OK;
  if ((st = check_ptr(x, "x")) || (st = check_ptr(yf, "yf"))) return st;
  int64_t n_tr = (int64_t)n_frames * frame->M * frame->n_sym;
  return launch_fft(*frame, n_tr, (const float2*)x, (float2*)yf, false, stream);
}

rxphy_status rxphy_csi(const rxphy_frame* frame, int32_t n_frames, const void* yf,
                       const void* pilots, void* h, hipStream_t stream) {
  clear_error();
  rxphy_status st = check_frame(frame, n_frames);
  if (st) return st;
  if (n_frames == 0) return RXPHY_OK;
  if ((st = check_ptr(yf, "yf")) || (st = check_ptr(pilots, "pilots")) || (st = check_ptr(h, "h")))
    return st;
  return launch_csi(*frame, n_frames, (const float2*)yf, (const float2*)pilots, (float2*)h, stream);
}

rxphy_status rxphy_detect(const rxphy_frame* frame, int32_t n_frames, const void* h,
                          const void* yf, void* xt, float* nu, uint8_t* flags,
                          int32_t precision_in, float cond_threshold, void* ws,
                          size_t ws_bytes, hipStream_t stream) {
  clear_error();
  rxphy_status st = check_frame(frame, n_frames);
  if (st) return st;
  if (!valid_precision(precision_in)) return fail(RXPHY_EINVAL, "precision = %d", (int)precision_in);
  const rxphy_precision precision = (rxphy_precision)precision_in;
  if (precision != RXPHY_FP32 && !(cond_threshold >= 0.0f))
    return fail(RXPHY_EINVAL, "cond_threshold = %g must be >= 0", cond_threshold);
  size_t need = rxphy_workspace_bytes(frame, n_frames, RXPHY_WS_DETECT, precision);
  if (need && (!ws || ws_bytes < need))
    return fail(RXPHY_EWORKSPACE, "detect needs %zu workspace bytes, got %zu", need, ws_bytes);
  if (n_frames == 0) return RXPHY_OK;
  if ((st = check_ptr(h, "h")) || (st = check_ptr(yf, "yf")) || (st = check_ptr(xt, "xt")) ||
      (st = check_ptr(nu, "nu")))
    return st;
  return launch_detect(*frame, n_frames, (const float2*)h, (const float2*)yf, nullptr, (float2*)xt, nu,
                       flags, precision, cond_threshold, ws, stream);
}

rxphy_status rxphy_csi_detect(const rxphy_frame* frame, int32_t n_frames, const void* yf,
                              const void* pilots, void* xt, float* nu, uint8_t* flags,
                              int32_t precision_in, float cond_threshold, void* ws,
                              size_t ws_bytes, hipStream_t stream) {
  clear_error();
  rxphy_status st = check_frame(frame, n_frames);
  if (st) return st;
  if (!valid_precision(precision_in)) return fail(RXPHY_EINVAL, "precision = %d", (int)precision_in);
  const rxphy_precision precision = (rxphy_precision)precision_in;
  if (precision != RXPHY_FP32 && !(cond_threshold >= 0.0f))
    return fail(RXPHY_EINVAL, "cond_threshold = %g must be >= 0", cond_threshold);
  size_t need = rxphy_workspace_bytes(frame, n_frames, RXPHY_WS_CSI_DETECT, precision);
  if (need && (!ws || ws_bytes < need))
    return fail(RXPHY_EWORKSPACE, "csi_detect needs %zu workspace bytes, got %zu", need, ws_bytes);
  if (n_frames == 0) return RXPHY_OK;
  if ((st = check_ptr(yf, "yf")) || (st = check_ptr(pilots, "pilots")) || (st = check_ptr(xt, "xt")) ||
      (st = check_ptr(nu, "nu")))
    return st;
  return launch_detect(*frame, n_frames, nullptr, (const float2*)yf, (const float2*)pilots, (float2*)xt,
                       nu, flags, precision, cond_threshold, ws, stream);
}

rxphy_status rxphy_fft_sc16(const rxphy_frame* frame, int32_t n_frames, const int16_t* x, float scale,
                            void* yf, hipStream_t stream) {
  clear_error();
  rxphy_status st = check_frame(frame, n_frames);
  if (st) return st;
  if (!(scale > 0.0f) || !std::isfinite(scale)) return fail(RXPHY_EINVAL, "scale = %g must be finite and > 0", scale);
  if (n_frames == 0) return RXPHY_OK;
  if ((st = check_ptr(x, "x")) || (st = check_ptr(yf, "yf"))) return st;
  int64_t n_tr = (int64_t)n_frames * frame->M * frame->n_sym;
  return launch_fft_sc16(*frame, n_tr, (const short2*)x, scale, (float2*)yf, stream);
}

rxphy_status rxphy_csi_detect_demod(const rxphy_frame* frame, int32_t n_frames, const void* yf,
                                    const void* pilots, void* xt, float* nu, uint8_t* flags, float* llr,
                                    int32_t precision_in, float cond_threshold, void* ws,
                                    size_t ws_bytes, hipStream_t stream) {
  clear_error();
  rxphy_status st = check_frame(frame, n_frames);
  if (st) return st;
  if (!valid_precision(precision_in)) return fail(RXPHY_EINVAL, "precision = %d", (int)precision_in);
  const rxphy_precision precision = (rxphy_precision)precision_in;
  if (precision != RXPHY_FP32 && !(cond_threshold >= 0.0f))
    return fail(RXPHY_EINVAL, "cond_threshold = %g must be >= 0", cond_threshold);
  size_t need = rxphy_workspace_bytes(frame, n_frames, RXPHY_WS_CSI_DETECT_DEMOD, precision);
  if (need && (!ws || ws_bytes < need))
    return fail(RXPHY_EWORKSPACE, "csi_detect_demod needs %zu workspace bytes, got %zu", need, ws_bytes);
  if (n_frames == 0) return RXPHY_OK;
  if ((st = check_ptr(yf, "yf")) || (st = check_ptr(pilots, "pilots")) || (st = check_ptr(nu, "nu")) ||
      (st = check_ptr(llr, "llr")))
    return st;
  const rxphy_frame& fr = *frame;
  if (group_path(fr, precision))
    return launch_detect_group(fr, n_frames, (const float2*)yf, (const float2*)pilots, (float2*)xt, nu, flags,
                               llr, precision, cond_threshold, ws, stream);
  // the stages one after the other; x_tilde in the caller's buffer or after
  // the detector's part of the workspace
  float2* x = (float2*)xt;
  if (!x) x = (float2*)((char*)ws + ((detect_workspace_bytes(fr, n_frames, precision) + 255) & ~(size_t)255));
  if ((st = launch_detect(fr, n_frames, nullptr, (const float2*)yf, (const float2*)pilots, x, nu, flags,
                          precision, cond_threshold, ws, stream)))
    return st;
  return launch_demod(fr, n_frames, x, nu, llr, stream);
}

// Scratch memory of the allocation-free entry point: one copy per GPU the
// library runs on, held until the process ends.  Host code never passes the
// array's name to a kernel (on the host it is a stand-in, not a device
// address); it passes the address hipGetSymbolAddress returns for the
// current device, looked up once per device.
static __device__ __align__(256) unsigned char scratch[RXPHY_NOALLOC_SCRATCH_BYTES];

static rxphy_status scratch_address(void** out) {
  static std::mutex mu;
  static std::vector<void*> addr;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return fail(RXPHY_EHIP, "hipGetDevice failed");
  std::lock_guard<std::mutex> lk(mu);
  if ((int)addr.size() <= dev) addr.resize(dev + 1, nullptr);
  if (!addr[dev]) {
    void* ptr = nullptr;
    hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) return fail(RXPHY_EHIP, "scratch address: %s", hipGetErrorString(e));
    addr[dev] = ptr;
  }
  *out = addr[dev];
  return RXPHY_OK;
}

rxphy_status rxphy_csi_detect_demod_noalloc(const rxphy_frame* frame, int32_t n_frames, const void* yf,
                                            const void* pilots, void* xt, float* nu, uint8_t* flags,
                                            float* llr, int32_t precision_in, float cond_threshold,
                                            hipStream_t stream) {
  clear_error();
  rxphy_status st = check_frame(frame, n_frames);
  if (st) return st;
  if (!valid_precision(precision_in)) return fail(RXPHY_EINVAL, "precision = %d", (int)precision_in);
  const rxphy_precision precision = (rxphy_precision)precision_in;
  const size_t need = rxphy_workspace_bytes(frame, n_frames, RXPHY_WS_CSI_DETECT_DEMOD, precision);
  if (need > (size_t)RXPHY_NOALLOC_SCRATCH_BYTES)
    return fail(RXPHY_EWORKSPACE,
                "csi_detect_demod_noalloc needs %zu scratch bytes for %d frames; its scratch holds %zu",
                need, n_frames, (size_t)RXPHY_NOALLOC_SCRATCH_BYTES);
  if (n_frames == 0) return RXPHY_OK;
  void* ws = nullptr;
  if ((st = scratch_address(&ws))) return st;
  return rxphy_csi_detect_demod(frame, n_frames, yf, pilots, xt, nu, flags, llr, precision, cond_threshold, ws,
                                (size_t)RXPHY_NOALLOC_SCRATCH_BYTES, stream);
}

rxphy_status rxphy_modulate(const rxphy_frame* frame, int32_t n_frames, const uint8_t* bits, void* sym,
                            hipStream_t stream) {
  clear_error();
  rxphy_status st = check_frame(frame, n_frames);
  if (st) return st;
  if (n_frames == 0) return RXPHY_OK;
  if ((st = check_ptr(bits, "bits")) || (st = check_ptr(sym, "sym"))) return st;
  const int64_t n = (int64_t)n_frames * frame->K * (frame->n_sym - 1) * frame->n_sc;
  return launch_modulate(*frame, n, bits, (float2*)sym, stream);
}

// rxphy_precode and rxphy_modulate_precode: the points come as complex64
// symbols (src_bits = 0) or as bit bytes mapped on the fly (src_bits = Q).
static rxphy_status precode_common(const rxphy_frame* frame, int32_t n_frames, const void* yf, const void* pilots,
                                   const void* src, int src_bits, void* xf, uint8_t* flags, void* ws,
                                   size_t ws_bytes, uint32_t options, hipStream_t stream) {
  clear_error();
  rxphy_status st = check_frame(frame, n_frames);
  if (st) return st;
  if (options & ~(uint32_t)RXPHY_PRECODE_REUSE_FACTORS) return fail(RXPHY_EINVAL, "precode options = %#x", options);
  const bool reuse = (options & RXPHY_PRECODE_REUSE_FACTORS) != 0;
  if (reuse && frame->K != 16)
    return fail(RXPHY_EINVAL, "precode: reusing the uplink factors needs K = 16 (the group records), K = %d", frame->K);
  size_t need = rxphy_workspace_bytes(frame, n_frames, RXPHY_WS_PRECODE, RXPHY_FP32);
  if (need && (!ws || ws_bytes < need))
    return fail(RXPHY_EWORKSPACE, "precode needs %zu workspace bytes, got %zu", need, ws_bytes);
  if (n_frames == 0) return RXPHY_OK;
  if ((st = check_ptr(yf, "yf")) || (st = check_ptr(pilots, "pilots")) ||
      (st = check_ptr(src, src_bits ? "bits" : "sym")) || (st = check_ptr(xf, "xf")))
    return st;
  if (frame->K == 16)
    return launch_precode(*frame, n_frames, (const float2*)yf, (const float2*)pilots, src, src_bits, (float2*)xf,
                          flags, ws, reuse, stream);
  return launch_precode_general(*frame, n_frames, (const float2*)yf, (const float2*)pilots, src, src_bits,
                                (float2*)xf, flags, stream);
}

rxphy_status rxphy_precode(const rxphy_frame* frame, int32_t n_frames, const void* yf, const void* pilots,
                           const void* sym, void* xf, uint8_t* flags, void* ws, size_t ws_bytes,
                           uint32_t options, hipStream_t stream) {
  return precode_common(frame, n_frames, yf, pilots, sym, 0, xf, flags, ws, ws_bytes, options, stream);
}

rxphy_status rxphy_modulate_precode(const rxphy_frame* frame, int32_t n_frames, const void* yf, const void* pilots,
                                    const uint8_t* bits, void* xf, uint8_t* flags, void* ws, size_t ws_bytes,
                                    uint32_t options, hipStream_t stream) {
  if (frame && (frame->qam_bits != 2 && frame->qam_bits != 4 && frame->qam_bits != 6)) {
    clear_error();
    return fail(RXPHY_EINVAL, "qam_bits = %d", frame->qam_bits);
  }
  return precode_common(frame, n_frames, yf, pilots, bits, frame ? frame->qam_bits : 0, xf, flags, ws, ws_bytes,
                        options, stream);
}

rxphy_status rxphy_ifft_sc16(const rxphy_frame* frame, int64_t n_rows, const void* xf, float scale, int16_t* x,
                            hipStream_t stream) {
  clear_error();
  rxphy_status st = check_frame(frame, 0);
  if (st) return st;
  if (!(scale > 0.0f) || !std::isfinite(scale)) return fail(RXPHY_EINVAL, "scale = %g must be finite and > 0", scale);
  if (n_rows < 0) return fail(RXPHY_EINVAL, "n_rows = %lld < 0", (long long)n_rows);
  if (n_rows == 0) return RXPHY_OK;
  if ((st = check_ptr(xf, "xf")) || (st = check_ptr(x, "x"))) return st;
  return launch_ifft_rows_sc16(*frame, n_rows, (const float2*)xf, 1.0f / scale, (short2*)x, stream);
}

rxphy_status rxphy_ifft(const rxphy_frame* frame, int64_t n_rows, const void* xf, void* x, hipStream_t stream) {
  clear_error();
  rxphy_status st = check_frame(frame, 0);
  if (st) return st;
  if (n_rows < 0) return fail(RXPHY_EINVAL, "n_rows = %lld < 0", (long long)n_rows);
  if (n_rows == 0) return RXPHY_OK;
  if ((st = check_ptr(xf, "xf")) || (st = check_ptr(x, "x"))) return st;
  return launch_ifft_rows(*frame, n_rows, (const float2*)xf, (float2*)x, stream);
}

rxphy_status rxphy_demod(const rxphy_frame* frame, int32_t n_frames, const void* xt,
                         const float* nu, float* llr, hipStream_t stream) {
  clear_error();
  rxphy_status st = check_frame(frame, n_frames);
  if (st) return st;
  if (n_frames == 0) return RXPHY_OK;
  if ((st = check_ptr(xt, "xt")) || (st = check_ptr(nu, "nu")) || (st = check_ptr(llr, "llr")))
    return st;
  return launch_demod(*frame, n_frames, (const float2*)xt, nu, llr, stream);
}

}  // extern "C"
