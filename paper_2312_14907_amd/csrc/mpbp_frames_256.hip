// mpbp_frames_256.hip - frame kernel instances for 256 x 256 detector windows
// (footprint bounds 48, 64, 256).
#include "mpbp_frame.hpp"

namespace mpbp {

hipError_t frames_d256(int op, int fb, const FrameArgs* a, int lds_bytes, hipStream_t s) {
  return frame_dispatch<256, 48, 64, 256>(op, fb, a, lds_bytes, s);
}

}  // namespace mpbp
