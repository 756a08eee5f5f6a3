// mpbp_launch.hpp - host-callable launchers of the device kernels.
#pragma once
#include <hip/hip_runtime.h>

#include <vector>

#include "mpbp_kernels.hpp"

namespace mpbp {

// Allow the frame and gradient kernels the full 160 KB of LDS on the current device.
// Called once per plan, before any launch (and before any graph capture).
hipError_t prepare_kernels();
// True if the frame kernel is compiled for detector size D, footprint bound FB and
// projection slab depth G.
bool frame_instance(int D, int FB, int G);

// tied = ny * nx for fields given per lateral pixel (the z-tied parameterisation), else 0.
hipError_t launch_object(const float* u, const float* chi, const float* alpha, const PeakDev* peaks,
                         int n_peaks, long long nvox, long long tied, float* obj, hipStream_t s);
// Frames of one detector size D whose footprints fit FB x FB (a.list holds only such
// frames; frame_bound(D, largest footprint side) is the smallest such FB), with G object
// slices staged per projection step.
hipError_t launch_frames(int D, int FB, int G, const FrameArgs& a, int lds_bytes, hipStream_t s);
int frame_bound(int D, int footprint);
// Gradient kernel reading `batch` frames per step of its frame walk (1, 2 or 4), over
// tiles `tile_x` voxels wide (16: 16 x 4, 8: 8 x 8).
hipError_t launch_grad(int batch, int tile_x, const GradArgs& a, int lds_bytes, hipStream_t s);
hipError_t launch_finalize(const double* floss, const int* out_list, int n_out, double* loss,
                           float* frame_loss, const double* apart, int n_part, int n_peaks,
                           float* grad_alpha, hipStream_t s);
hipError_t launch_step(float* p, const float* g, long long n, float eta, hipStream_t s);
hipError_t launch_adam(float* p, float* x, float* m, float* v, const float* g, long long n, float lr,
                       float b1, float b2, float eps, float c1, float c2, int log_mode, int project,
                       long long fixed, hipStream_t s);
hipError_t launch_exp(float* x, const float* xlog, long long n, hipStream_t s);
hipError_t launch_fill(float* p, long long n, float v, hipStream_t s);
// out (dev double) = sum of a[i]^2, using part[max_part] as scratch.
hipError_t launch_norm2(const float* a, long long n, double* part, int max_part, double* out, hipStream_t s);
hipError_t launch_mark_active(unsigned char* act, long long n_frames, const int* list, int n,
                              hipStream_t s);

// Dynamic LDS of the frame kernel for one peak and slab depth G (bytes); must match
// frame_body's layout.
int frame_lds_bytes(int D, int fy, int fx, int fxp, int np, int nz, bool grad, int G);
// Append the frame kernel's twiddle tables of one peak (complex64 as float pairs):
// row twiddles [D], column twiddles [L], residue-fold twiddles [R][fy] (footprint at
// the window origin).
bool frame_twiddles(int D, int fy, std::vector<float>& out);
// Rows per residue chunk of the detector (the column-transform length).
int frame_chunk_len(int D);
// Dynamic LDS of the gradient kernel (bytes).
int grad_lds_bytes(int np, int nz, int maxspan_y, int maxspan_x, int max_cand, bool tied);

}  // namespace mpbp
