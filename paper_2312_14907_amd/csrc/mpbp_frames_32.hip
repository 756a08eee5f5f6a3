// mpbp_frames_32.hip - frame kernel instances for 32 x 32 detector windows
// (footprint bounds 32).
#include "mpbp_frame.hpp"

namespace mpbp {

hipError_t frames_d32(int op, int fb, const FrameArgs* a, int lds_bytes, hipStream_t s) {
  return frame_dispatch<32, 32>(op, fb, a, lds_bytes, s);
}

}  // namespace mpbp
