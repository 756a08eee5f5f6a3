// mpbp_frames_150.hip - frame kernel instances for 150 x 150 detector windows (the
// paper's detector, 150 = 2 * 3 * 5^2: rows as 10 x 15, columns in chunks of 50 = 10 x 5;
// footprint bounds 48, 64, 150).
#include "mpbp_frame.hpp"

namespace mpbp {

hipError_t frames_d150(int op, int fb, const FrameArgs* a, int lds_bytes, hipStream_t s) {
  return frame_dispatch<150, 48, 64, 150>(op, fb, a, lds_bytes, s);
}

}  // namespace mpbp
