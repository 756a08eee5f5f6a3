// mpbp_launch.hpp - host-callable launchers of the device kernels.
#pragma once
#include <hip/hip_runtime.h>

#include <vector>

#include "mpbp_kernels.hpp"

namespace mpbp {

// Allow the frame and gradient kernels the full 160 KB of LDS on the current device.
// Called once per plan, before any launch (and before any graph capture).
hipError_t prepare_kernels();
// True if the frame kernel is compiled for detector size D and footprint bound FB.
bool frame_instance(int D, int FB);

// tied = ny * nx for fields given per lateral pixel (the z-tied parameterisation), else 0.
hipError_t launch_object(const float* u, const float* chi, const float* alpha, const PeakDev* peaks,
                         int n_peaks, long long nvox, long long tied, float* obj, hipStream_t s);
// The run sums S_k = sum over the slices z of run k of O_m(z), for every peak and run:
// complex64 [sum of nruns][ny][nx] into rsum (zrun: [M][nz] run of each slice).
hipError_t launch_runsum(const float* u, const float* chi, const float* alpha, const PeakDev* peaks, int n_peaks,
                         int nz, long long nlat, int tied, const int* zrun, float* rsum, hipStream_t s);
// Frames of one detector size D whose footprints fit FB x FB (a.list holds only such
// frames; frame_bound(D, largest footprint side) is the smallest such FB).  Reads each
// frame's exit wave from its slot (written by launch_project).
hipError_t launch_frames(int D, int FB, const FrameArgs& a, int lds_bytes, hipStream_t s);
// Exit waves of the listed frames into their slots, with G object slices in flight per
// lane (G = 2, 4 or 8); lds_bytes from project_lds_bytes.  With a detector map
// (a.mapz), launch_project_map runs instead and G and lds_bytes are not used.
hipError_t launch_project(int G, const FrameArgs& a, int lds_bytes, hipStream_t s);
int project_lds_bytes(int np, int G, int nz, int acc_pix);
int frame_bound(int D, int footprint);
// Back-projection and chain rule reading `batch` frames at once (the run gather
// k_bp_gather plus k_bp_chain, where
// grad_uses_runs(a): batch clamped to [4, 16]; otherwise the per-slice walk, k_grad:
// batch clamped to at most 4), over tiles `tile_x` voxels wide (16: 16 x 4, 8: 8 x 8).
hipError_t launch_grad(int batch, int tile_x, const GradArgs& a, int lds_bytes, hipStream_t s);
bool grad_uses_runs(const GradArgs& a);
// Number of alpha partials [n][M] the gradient launch writes (per tile, or per workgroup
// of the run chain rule).
int grad_partials(const GradArgs& a);
int grad_effective_batch(int batch, bool runs);
// R with a detector-frame map (MPBP_DETECTOR_MAP, a.mapz set): the interpolating
// projection and its adjoint back-projection (mpbp_map.hip); launch_project and
// launch_grad dispatch to them.
hipError_t launch_project_map(const FrameArgs& a, hipStream_t s);
hipError_t launch_grad_map(const GradArgs& a, hipStream_t s);
hipError_t prepare_map_kernels();
// The chain rule per voxel from the frame sums per run in a.rs (k_bp_chain).
hipError_t launch_bp_chain(const GradArgs& a, hipStream_t s);
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

// Dynamic LDS of the frame kernel for one peak (bytes); must match frame_body's layout.
int frame_lds_bytes(int D, int fy, int fx, int fxp, bool grad);
// Append the frame kernel's twiddle tables of one peak (complex64 as float pairs):
// row twiddles [D], column twiddles [L], residue-fold twiddles [R][fy] (footprint at
// the window origin).
bool frame_twiddles(int D, int fy, std::vector<float>& out);
// Rows per residue chunk of the detector (the column-transform length).
int frame_chunk_len(int D);
// Dynamic LDS of the gradient kernel (bytes).
int grad_lds_bytes(int np, int nz, int maxspan_y, int maxspan_x, int max_cand, bool tied, bool runs);

}  // namespace mpbp
