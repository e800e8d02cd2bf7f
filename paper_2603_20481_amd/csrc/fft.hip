// Batched segment FFT stage: one launch over every (frame, antenna, symbol)
// segment; the transform itself is fftk::fft_tile.
#include "fft_core.h"

namespace rxphy {
namespace {

using namespace fftk;

// Each workgroup runs PER_WG transforms per transform slot.
constexpr int PER_WG = 8;

template <int N, bool INV, bool MAG = false, typename IN_T = float2, bool OUT16 = false>
__global__ void __launch_bounds__(WG)
fft_kernel(const IN_T* __restrict__ in, float2* __restrict__ out, const float2* __restrict__ tw,
           int64_t n_tr, int sym_len, int cp, int n_sc, int cp_tail, float in_scale, float out_scale) {
  __shared__ float2 lds[Geom<N>::LDS];
  fft_tile<N, INV, MAG, IN_T, OUT16>(in, out, tw, n_tr, (int64_t)blockIdx.x * Geom<N>::TPW * PER_WG, PER_WG,
                                     sym_len, cp, n_sc, lds, cp_tail != 0, in_scale, out_scale);
}

template <int N, bool INV, bool MAG = false, typename IN_T = float2, bool OUT16 = false>
rxphy_status run(int64_t n_tr, const IN_T* in, float2* out, const float2* tw, int sym_len,
                 int cp, int n_sc, int cp_tail, hipStream_t s, float in_scale = 1.f, float out_scale = 1.f) {
  using G = Geom<N>;
  const int64_t per = (int64_t)G::TPW * PER_WG;
  int64_t blocks = (n_tr + per - 1) / per;
  if (blocks > 0x7fffffff) return fail(RXPHY_EUNSUPPORTED, "too many transforms (%lld)", (long long)n_tr);
  if (blocks == 0) return RXPHY_OK;
  hipLaunchKernelGGL((fft_kernel<N, INV, MAG, IN_T, OUT16>), dim3((unsigned)blocks), dim3(WG), 0, s, in, out, tw,
                     n_tr, sym_len, cp, n_sc, cp_tail, in_scale, out_scale);
  return launch_status("fft kernel");
}

}  // namespace

static rxphy_status dispatch(const rxphy_frame& fr, int64_t n_tr, const float2* in, float2* out, bool inverse,
                             int cp_tail, hipStream_t s) {
  const float2* tw = nullptr;
  rxphy_status st = ensure_device_tables(&tw);
  if (st) return st;
  const int L = (int)sym_len(fr);
#define RXPHY_FFT_CASE(NN)                                                                  \
  case NN:                                                                                  \
    return inverse ? run<NN, true>(n_tr, in, out, tw, L, fr.cp_len, fr.n_sc, cp_tail, s)     \
                   : run<NN, false>(n_tr, in, out, tw, L, fr.cp_len, fr.n_sc, cp_tail, s);
  switch (fr.n_fft) {
    RXPHY_FFT_CASE(512)
    RXPHY_FFT_CASE(1024)
    RXPHY_FFT_CASE(2048)
    RXPHY_FFT_CASE(4096)
  }
#undef RXPHY_FFT_CASE
  return fail(RXPHY_EUNSUPPORTED, "n_fft = %d", fr.n_fft);
}

rxphy_status launch_fft(const rxphy_frame& fr, int64_t n_tr, const float2* in, float2* out,
                        bool inverse, hipStream_t s) {
  return dispatch(fr, n_tr, in, out, inverse, 0, s);
}

rxphy_status launch_fft_sc16(const rxphy_frame& fr, int64_t n_tr, const short2* in, float scale, float2* out,
                             hipStream_t s) {
  const float2* tw = nullptr;
  rxphy_status st = ensure_device_tables(&tw);
  if (st) return st;
  const int L = (int)sym_len(fr);
  switch (fr.n_fft) {
    case 512: return run<512, false, false, short2>(n_tr, in, out, tw, L, fr.cp_len, fr.n_sc, 0, s, scale);
    case 1024: return run<1024, false, false, short2>(n_tr, in, out, tw, L, fr.cp_len, fr.n_sc, 0, s, scale);
    case 2048: return run<2048, false, false, short2>(n_tr, in, out, tw, L, fr.cp_len, fr.n_sc, 0, s, scale);
    case 4096: return run<4096, false, false, short2>(n_tr, in, out, tw, L, fr.cp_len, fr.n_sc, 0, s, scale);
  }
  return fail(RXPHY_EUNSUPPORTED, "n_fft = %d", fr.n_fft);
}

rxphy_status launch_ifft_rows_sc16(const rxphy_frame& fr, int64_t n_rows, const float2* in, float out_scale,
                                   short2* out, hipStream_t s) {
  const float2* tw = nullptr;
  rxphy_status st = ensure_device_tables(&tw);
  if (st) return st;
  const int L = (int)sym_len(fr);
  float2* o = reinterpret_cast<float2*>(out);
  switch (fr.n_fft) {
    case 512: return run<512, true, false, float2, true>(n_rows, in, o, tw, L, fr.cp_len, fr.n_sc, 1, s, 1.f, out_scale);
    case 1024: return run<1024, true, false, float2, true>(n_rows, in, o, tw, L, fr.cp_len, fr.n_sc, 1, s, 1.f, out_scale);
    case 2048: return run<2048, true, false, float2, true>(n_rows, in, o, tw, L, fr.cp_len, fr.n_sc, 1, s, 1.f, out_scale);
    case 4096: return run<4096, true, false, float2, true>(n_rows, in, o, tw, L, fr.cp_len, fr.n_sc, 1, s, 1.f, out_scale);
  }
  return fail(RXPHY_EUNSUPPORTED, "n_fft = %d", fr.n_fft);
}

rxphy_status launch_fft_mag(int n_fft, int64_t n_rows, const float2* in, float* out, hipStream_t s) {
  const float2* tw = nullptr;
  rxphy_status st = ensure_device_tables(&tw);
  if (st) return st;
  float2* o = reinterpret_cast<float2*>(out);
  switch (n_fft) {
    case 512: return run<512, false, true>(n_rows, in, o, tw, 512, 0, 512, 0, s);
    case 1024: return run<1024, false, true>(n_rows, in, o, tw, 1024, 0, 1024, 0, s);
    case 2048: return run<2048, false, true>(n_rows, in, o, tw, 2048, 0, 2048, 0, s);
    case 4096: return run<4096, false, true>(n_rows, in, o, tw, 4096, 0, 4096, 0, s);
  }
  return fail(RXPHY_EUNSUPPORTED, "n_fft = %d", n_fft);
}

rxphy_status launch_ifft_rows(const rxphy_frame& fr, int64_t n_rows, const float2* in, float2* out,
                              hipStream_t s) {
  return dispatch(fr, n_rows, in, out, true, 1, s);
}

}  // namespace rxphy
