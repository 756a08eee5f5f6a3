// mpbp_frames_64.hip - frame kernel instances for 64 x 64 detector windows
// (footprint bounds 48, 64).
#include "mpbp_frame.hpp"

namespace mpbp {

hipError_t frames_d64(int op, int fb, const FrameArgs* a, int lds_bytes, hipStream_t s) {
  return frame_dispatch<64, 48, 64>(op, fb, a, lds_bytes, s);
}

}  // namespace mpbp
