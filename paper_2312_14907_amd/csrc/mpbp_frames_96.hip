// mpbp_frames_96.hip - frame kernel instances for 96 x 96 detector windows
// (footprint bounds 48, 64, 96).
#include "mpbp_frame.hpp"

namespace mpbp {

hipError_t frames_d96(int op, int fb, const FrameArgs* a, int lds_bytes, hipStream_t s) {
  return frame_dispatch<96, 48, 64, 96>(op, fb, a, lds_bytes, s);
}

}  // namespace mpbp
