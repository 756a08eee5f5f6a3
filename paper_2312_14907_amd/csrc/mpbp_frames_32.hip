// mpbp_frames_32.hip - frame kernel instances for 32 x 32 detector windows
// (footprint bounds 32; every compiled slab depth).
#include "mpbp_frame.hpp"

namespace mpbp {

hipError_t frames_d32(int op, int fb, int g, const FrameArgs* a, int lds_bytes, hipStream_t s) {
  return frame_dispatch<32, 32>(op, fb, g, a, lds_bytes, s);
}

}  // namespace mpbp
