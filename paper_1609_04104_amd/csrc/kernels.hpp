// Host-side launchers of the step's kernels.  A Batch describes the frames of
// one launch group: either one frame passed by value, or `count` frames of the
// same (n1, n2) read from a device table (see FrameTable for the block order).
#pragma once

#include "frame.hpp"

namespace tsl {

struct Batch {
    const FrameArgs* one;        // single frame (by value), or null
    const FrameArgs* table;      // device table of `count` frames, or null
    int count;
    int n1, n2;                  // shared by every frame of the group
    int r_max;                   // largest rank in the group
    int rows_max;                // largest n_rows (line masks)
    int mode;                    // MODE_LINES or MODE_POINTS (shared)
    bool kspace;                 // line masks on the k-space route (shared)
    bool want_x;                 // some frame asks for X_t
    bool want_sample;            // some frame draws its next rows
    int synth;                   // synthesis operands (SYN_*), shared by the frames of an output launch
    int out_tile;                // output block tile (OUT_*; FP32 synthesis), chosen by the tuner
};

// Block tiles of the output synthesis (X_t = A diag(gamma) B^T): identical results.
enum : int { OUT_128x64 = 0, OUT_64x64 = 1, OUT_128x128 = 2, OUT_TILES = 3 };

// Threads per block of the kernels that are not templated on a length.
constexpr int kBlock = 256;

// Grid of a launch with x blocks per frame (table launches pad the frame count
// to a multiple of kXcds; see FrameTable).
inline dim3 frame_grid(const Batch& b, int x) {
    return b.table ? dim3(unsigned(x) * unsigned((b.count + kXcds - 1) / kXcds * kXcds)) : dim3(unsigned(x));
}

// Row direction (length n2): K1 synthesis + row transform, K3 row inverse +
// Theta conj(B); standalone row pass of the 2-D transform.
hipError_t launch_synth_rowfft(const Batch& b, hipStream_t st);
hipError_t launch_row_inv_grad(const Batch& b, hipStream_t st);
hipError_t launch_rowfft(int n1, int n2, int batch, const float2* in, float2* out, bool inv, hipStream_t st);

// Column direction (length n1 / n2): K2 column transform + residual + column
// inverse + Z^T conj(A); K4 factor updates with the k-space factor transforms;
// standalone column pass; plain column transform of a [n][r] factor.
hipError_t launch_col_resid(const Batch& b, hipStream_t st);
hipError_t launch_update_a(const Batch& b, hipStream_t st);
hipError_t launch_update_b(const Batch& b, hipStream_t st);
hipError_t launch_colfft(int n1, int n2, int batch, const float2* in, float2* out, bool inv, hipStream_t st);
hipError_t launch_factor_fft(int n, int r, const float2* in, float2* out, bool inv, hipStream_t st);

// Length-independent kernels: partial Grams (a2), ridge solve and step size
// (a3, a8), output synthesis (a10), line sampler (a11), status clear.
hipError_t launch_stats(const Batch& b, hipStream_t st);
hipError_t launch_solve(const Batch& b, hipStream_t st);
hipError_t launch_synth_out(const Batch& b, hipStream_t st);

hipError_t launch_sample(const Batch& b, hipStream_t st);
// Algorithm 4 on entries (eq. 13) for one frame's sequence: mask [n1][n2], count, trial entries.
hipError_t launch_sample_points(const FrameArgs& a, int K, unsigned char* mask, int* n_out, int* draws,
                                hipStream_t st);

// One frame of a sequence imaged by several coils (Algorithm 3 with C coils,
// csrc/k_coils.hip): the sequence's state, its coil maps and workspace, the
// frame's rows and samples.
struct CoilArgs {
    int n1, n2, r, C, n_rows, step_mode;
    double lambda, mu_const;
    float2 *A, *B, *Ahat, *Bhat;       // state (A, B updated in place; F_l A, F_r B recomputed)
    SeqDev* dev;
    double2* gamma64;
    float2* gamma32;
    const float2* H;                   // [C][n1][n2] sensitivity maps
    float2* P;                         // [r][n1][n2] transformed rank images of one coil
    float2* Q;                         // [C][n1][n2] coil-weighted prediction, then Xi_c, then F^{-1}(Xi_c)
    float2* theta;                     // [n1][n2] Theta
    float2 *GA, *GB;                   // [n1][r] Theta conj(B), [n2][r] Theta^T conj(A)
    double2* gslot;                    // [C][n1][r][r] Gram partials per coil and sampled row (upper entries)
    double2* hslot;                    // [C][n1][r] right-hand-side partials
    double* gain;                      // [1] max over pixels of sum_c |H_c|^2
    const int* rows;                   // [n_rows] ascending
    const float2* y;                   // [C][n_rows][n2]
    float2 *A_out, *B_out, *gamma_out;
};
hipError_t launch_coil_step(const CoilArgs& a, hipStream_t st);
hipError_t launch_coil_gain(const CoilArgs& a, hipStream_t st);

// Raises the dynamic-LDS limit of the kernels that need more than the default
// (idempotent; called before any launch or graph capture).
void init_kernel_attributes();

bool size_supported(int n);
int plan_threads(int n);   // T of Plan<n>, 0 if unsupported

}  // namespace tsl
