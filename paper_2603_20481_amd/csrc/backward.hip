// Adjoint of the forward receiver map and workspace sizing.
#include "common.h"

using namespace rxphy;

extern "C" {

size_t rxphy_workspace_bytes(const rxphy_frame* frame, int32_t n_frames, int32_t which,
                             rxphy_precision precision) {
  (void)precision;
  if (check_frame(frame, n_frames) != RXPHY_OK) return 0;
  if (which == RXPHY_WS_DETECT) return 0;
  return 0;
}

rxphy_status rxphy_backward(const rxphy_frame* frame, int32_t n_frames, const void* x,
                            const void* pilots, const rxphy_saved* saved, const float* dllr,
                            void* dx, void* dh, void* ws, size_t ws_bytes, hipStream_t stream) {
  (void)frame; (void)n_frames; (void)x; (void)pilots; (void)saved; (void)dllr; (void)dx;
  (void)dh; (void)ws; (void)ws_bytes; (void)stream;
  clear_error();
  return fail(RXPHY_EUNSUPPORTED, "rxphy_backward is not built yet");
}

}  // extern "C"
