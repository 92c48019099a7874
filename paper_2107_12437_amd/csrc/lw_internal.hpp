// lw_internal.hpp -- declarations shared by the host runtime and the kernel
// translation units of liblw.so (not part of the public ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/lw.h"

namespace lw {

struct SrcRec;

// Outputs of an oscillator run, [steps/stride + 1][n_dip] each; all but d may
// be null.  wabs: work done on the dipole by its drive field since t = 0 (the
// integral of E_d d_dot); wrad: energy radiated since t = 0 (the integral of
// the Larmor power |d_ddot|^2 / (6 pi eps0 c^3)); both by the trapezoid rule
// over steps (Sec. 2.5).
struct RunOut {
    double *d, *v, *E, *Ed, *wabs, *wrad;
    int64_t stride;
    int n_dip;
};

// Run state of an oscillator run (device FP64), enough to continue it exactly:
//   [0] steps taken n, [1] ring depth, [2] number of dipoles, [3] unused;
//   the history rings: instance (dipoles a0..a1) at state_ring_off(a0, ring) as
//     [slot][a1 - a0][3] (d, d_dot, d_ddot), slot = step & (ring - 1);
//   E_d(t_n) of every dipole (state_ecur_off);
//   the energy sums (absorbed, radiated) of every dipole (state_w_off).
constexpr int64_t STATE_HEAD = 4;
__host__ __device__ inline int64_t state_ring_off(int a0, int ring) { return STATE_HEAD + (int64_t)a0 * ring * 3; }
__host__ __device__ inline int64_t state_ecur_off(int n_dip, int ring) { return state_ring_off(n_dip, ring); }
__host__ __device__ inline int64_t state_w_off(int n_dip, int ring) { return state_ecur_off(n_dip, ring) + n_dip; }
__host__ __device__ inline int64_t state_doubles(int n_dip, int ring) { return state_w_off(n_dip, ring) + 2 * (int64_t)n_dip; }

// Launch parameters of the grid-field kernel chosen by the tuner.
struct FieldLaunch {
    int block;       // threads per workgroup (multiple of 64)
    int tchunk;      // observation times per lane, kept in registers: 1, 2 or 4
};

// Grid fields: preparation of (time, charge) records, then the fused
// retarded-solve / Lienard-Wiechert / superposition / store kernel.
hipError_t launch_prep(const lw_traj *d_ch, int nch, const double *d_times, int nt, SrcRec *d_recs,
                       uint32_t *d_flags, int64_t npts, hipStream_t s);
// d_hist non-null: the counting instance (one time per lane, 256 lanes) adds each
// pair to the iteration histogram d_hist[ITER_BINS] (see fields_kernel).
constexpr int ITER_BINS = LW_ITER_BINS, ITER_BIN_FALLBACK = LW_ITER_BIN_FALLBACK, ITER_BIN_NOCONV = LW_ITER_BIN_NOCONV;
hipError_t launch_fields(const SrcRec *d_recs, int nch, const double *d_pts, int64_t npts, int nt,
                         const lw_opts &o, double tol_rel, double mask_r, void *d_out, uint32_t *d_flags,
                         const FieldLaunch &L, hipStream_t s, unsigned long long *d_hist = nullptr);
size_t src_rec_bytes();
// Output rows of an outputs mask (0: Phi | A | E | B).
int output_mask(int outputs);
int output_rows(int outputs);
// Zero-fills n doubles with a kernel (no memset node if the stream is captured).
hipError_t launch_fill_zero(double *d, int64_t n, hipStream_t s);

// Vector-Jacobian product of the grid fields with respect to the 11 trajectory
// parameters of every charge (lw_adjoint.hip).
int vjp_params();
size_t vjp_partial_doubles(int64_t npts, int nt, int nch, int tchunk);
hipError_t launch_fields_vjp(const SrcRec *d_recs, int nch, const double *d_pts, int64_t npts, int nt,
                             const lw_opts &o, double tol_rel, double mask_r, const void *d_cot, double *d_partial,
                             int tchunk, double *d_grad, hipStream_t s);

// Lorentz-oscillator runs.
struct DipDev;     // device-side oscillator constants
size_t dip_dev_bytes(int n);   // the DipDev array and its structure-of-arrays copy
int ring_lds_bytes(int n, int ring);
hipError_t launch_dipole_prep(const lw_dipole *d_in, int n, DipDev *d_dev, hipStream_t s);
// One launch of the per-instance persistent kernel over the instances listed in
// d_list[0..n_list); max_n is the largest of them.  With ring_lds the history
// ring lives in LDS, otherwise at d_ring_global + d_ring_off[block].
// d_state (nullable): the run state, read at the start when resume is set and
// written at the end.
hipError_t launch_dipole_instances(const DipDev *d_dev, const int32_t *d_off, const int32_t *d_list, int n_list,
                                   int max_n, bool ring_lds, const int64_t *d_ring_off, double *d_ring_global,
                                   int ring, int64_t steps, double dt, double max_vel, int max_iter,
                                   const RunOut &out, bool moving, bool mixed, double *d_state, bool resume,
                                   uint32_t *d_err, hipStream_t s);
// A resumed run: checks the state's header against (ring, n_dip) and writes
// output row 0 of every dipole from it.
hipError_t launch_state_rows(const DipDev *d_dev, const int32_t *d_off, int n_inst, const double *d_state, int ring,
                             const RunOut &out, uint32_t *d_err, hipStream_t s);
// After a run: the state's header (steps taken, ring, n_dip).
hipError_t launch_state_header(double *d_state, int ring, int n_dip, int64_t steps, bool resume, hipStream_t s);

// moving: some dipole's origin moves (kernels with the moving-origin code).
// mixed: FP32 pair fields (FP64 retarded times, state and sums).
// Large instances: one launch per step (captured into a replayed graph when
// graph_chunk > 0 and a capture stream is given), one workgroup per target.
// d_W: 2 doubles per dipole of running energy sums (absorbed, radiated).
// d_step: 2 int64 (the device step base, the run's first step).  resume: the
// ring, E_d and the sums already hold step (int64)d_resume[0] (a run state)
// and the first stage is not taken; otherwise the run starts at t = 0.
hipError_t launch_dipole_steps(const DipDev *d_dev, const int32_t *d_tgt, const int32_t *d_tgt_lo, const int32_t *d_tgt_n,
                               const int64_t *d_ring_base, int n_tgt, double *d_ring, double *d_Ecur, double *d_W,
                               int64_t *d_step, int ring, int64_t steps, double dt, double max_vel, int max_iter,
                               const RunOut &out, bool moving, bool mixed, const double *d_resume, uint32_t *d_err,
                               int graph_chunk, hipStream_t s, hipStream_t cap, hipGraph_t *graph_out,
                               hipGraphExec_t *exec_out);

// Pieces of the oscillator adjoint (lw_dipole_adjoint.hip), whose sweep runs
// over segments of steps; `ring` is the depth of the history and of its
// cotangents ([ring][n_dip][3], power of two: the whole run, or windows of
// recomputed segments), whose slots are cleared as the sweep consumes them.
// d_pair_off / d_pair_off0: per-instance prefix sums of the drive pairs of a
// step (4 n (n-1)) and of E_d(0) (2 n (n-1)); d_state 8 n_dip doubles (the
// cotangent state, double-buffered by step parity); d_rbp /
// d_rbp0 three doubles per pair, d_taup one per pair; d_step a device step
// index.  launch_hist_rows: samples row0 .. row0+nrows-1 from
// a stride-1 run's outputs; launch_hist_from_state: samples lo .. hi from a run
// state of depth ring_state; launch_vjp_begin: zeroes the cotangents, the
// gradient and the pair buffers and starts the step base at steps - 1;
// launch_vjp_detector: J partials (one double per 256 lanes of npts x n_snap)
// and the detector's cotangents for the given snapshots, J's sum over
// snapshots being divided by n_norm (the run's snapshot count); launch_vjp_steps:
// `count` backward steps from the current base; launch_vjp_end: E_d(0), the
// positions and the sum of n_jpart J partials into d_J.
hipError_t launch_hist_rows(const DipDev *d_dev, const double *d_D, const double *d_V, const double *d_Ed, int n_dip,
                            int64_t nrows, int64_t row0, int ring, double *d_hist, hipStream_t s);
hipError_t launch_hist_from_state(const double *d_state, const int32_t *d_off, int n_inst, int n_dip, int ring_state,
                                  int64_t lo, int64_t hi, int ring, double *d_hist, hipStream_t s);
hipError_t launch_vjp_begin(int n_dip, int64_t n_pairs, int64_t steps, double *d_hbar, int64_t hbar_doubles,
                            double *d_grad, double *d_rbp, double *d_taup, double *d_state, int64_t *d_step,
                            hipStream_t s);
hipError_t launch_vjp_detector(const DipDev *d_dev, int n_dip, const double *d_hist, double *d_hbar, int ring,
                               int64_t steps, double dt, const double *d_pts, int64_t npts, const double *d_times,
                               int n_snap, int n_norm, double *d_grad, double *d_Jpart, uint32_t *d_err,
                               hipStream_t s);
hipError_t launch_vjp_steps(const DipDev *d_dev, const int32_t *d_off, const int64_t *d_pair_off, int n_inst,
                            int n_dip, const double *d_hist, double *d_hbar, int ring, double dt, double *d_state,
                            double *d_rbp, double *d_taup, int64_t *d_step, int64_t count, int64_t steps,
                            uint32_t *d_err, hipStream_t s);
hipError_t launch_vjp_end(const DipDev *d_dev, const int32_t *d_off, const int64_t *d_pair_off,
                          const int64_t *d_pair_off0, int n_inst, int64_t n_pairs0, int n_dip, const double *d_hist,
                          double *d_hbar, int ring, double dt, double *d_state, double *d_rbp, double *d_rbp0,
                          double *d_grad, const double *d_Jpart, int64_t n_jpart, double *d_J, uint32_t *d_err,
                          hipStream_t s);


}  // namespace lw
