// mpbp_frames_192.hip - frame kernel instances for 192 x 192 detector windows
// (footprint bounds 48, 64, 192).
#include "mpbp_frame.hpp"

namespace mpbp {

hipError_t frames_d192(int op, int fb, const FrameArgs* a, int lds_bytes, hipStream_t s) {
  return frame_dispatch<192, 48, 64, 192>(op, fb, a, lds_bytes, s);
}

}  // namespace mpbp
