// mpbp_frames_128.hip - frame kernel instances for 128 x 128 detector windows
// (footprint bounds 48, 64, 128).
#include "mpbp_frame.hpp"

namespace mpbp {

hipError_t frames_d128(int op, int fb, const FrameArgs* a, int lds_bytes, hipStream_t s) {
  return frame_dispatch<128, 48, 64, 128>(op, fb, a, lds_bytes, s);
}

}  // namespace mpbp
