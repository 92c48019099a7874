// lw_adjoint.hip -- vector-Jacobian product of the grid fields with respect to
// the trajectory parameters of every charge (FP64).
//
// For one (point x, time t, charge) the outputs O = (Phi, A, E, B) depend on the
// retarded separation R = x - r(t'), velocity v(t') and acceleration a(t') and
// on q, with t' = t - tau and tau the root of c tau = |x - r(t - tau)| (Eq.
// (ret_t)).  For a parameter theta of the trajectory,
//   dR = -r_theta dtheta + v dtau,  dv = v_theta dtheta - a dtau,
//   da = a_theta dtheta - j dtau   (j = da/dt', the jerk),
// and differentiating the retarded-time equation (implicit function theorem)
//   dtau = -(n . r_theta) / (c kappa) dtheta,  c kappa = c - n . v.
// With Rb, vb, ab the cotangents of R, v, a (the reverse of the Lienard-Wiechert
// evaluator) and s = Rb.v - vb.a - ab.j, the cotangent of the trajectory
// position is rb = -Rb - s n / (c kappa), and the gradient of a parameter is
// rb . r_theta + vb . v_theta + ab . a_theta.  Sums over points and times are
// per-wave partials reduced in a fixed order (bitwise reproducible).
#include <math.h>

#include "lw_device.hpp"
#include "lw_internal.hpp"

namespace lw {

// Parameter order of the gradient rows.
enum { P_Q = 0, P_C0 = 1, P_AMP = 4, P_OMEGA = 5, P_PHASE = 6, P_ACCEL = 7, P_V = 8, NP = 11 };
// Waves per workgroup of the VJP kernel (256 lanes): each writes its own partials.
constexpr int WAVES = 4;

// Gradient of one (point, time, charge) contribution, added into g[NP].
// EONLY: only E has a cotangent (lw_terms_vjp<true>).
template <bool EONLY>
__device__ __forceinline__ void pair_param_grad(const SrcRec &S, const Kin &k, int field_kind, const double ob[10],
                                                double g[NP])
{
    double Rb[3], vb[3], ab[3], n[3], kqb, kappa;
    lw_terms_vjp<EONLY, true>(k, S.kq, field_kind, ob, Rb, vb, ab, kqb, n, kappa);
    // jerk at t': -omega^2 v for the harmonic families, 0 otherwise
    const bool harm = (S.kind == K_CIRCULAR || S.kind == K_LINEAR_OSC);
    const double w2 = harm ? S.omega * S.omega : 0.0;
    double sres = 0.0;
    for (int i = 0; i < 3; ++i) sres += Rb[i] * k.v[i] - vb[i] * k.a[i] + ab[i] * w2 * k.v[i];
    const double fac = sres * recip<double>(C_LIGHT - (n[0] * k.v[0] + n[1] * k.v[1] + n[2] * k.v[2]));
    double rb[3];
    for (int i = 0; i < 3; ++i) rb[i] = -Rb[i] - fac * n[i];
    g[P_Q] += kqb * K_COUL;
    for (int i = 0; i < 3; ++i) g[P_C0 + i] += rb[i];
    const double A = S.amp, om = S.omega, c = k.cph, sn = k.sph, tp = k.tp;
    const double r1 = rb[0] * S.e1[0] + rb[1] * S.e1[1] + rb[2] * S.e1[2];
    const double v1 = vb[0] * S.e1[0] + vb[1] * S.e1[1] + vb[2] * S.e1[2];
    const double a1 = ab[0] * S.e1[0] + ab[1] * S.e1[1] + ab[2] * S.e1[2];
    if (S.kind == K_CIRCULAR) {
        const double r2 = rb[0] * S.e2[0] + rb[1] * S.e2[1] + rb[2] * S.e2[2];
        const double v2 = vb[0] * S.e2[0] + vb[1] * S.e2[1] + vb[2] * S.e2[2];
        const double a2 = ab[0] * S.e2[0] + ab[1] * S.e2[1] + ab[2] * S.e2[2];
        // projections on the radial (c e1 + s e2) and tangential (-s e1 + c e2) directions
        const double Pr = r1 * c + r2 * sn, Qr = r2 * c - r1 * sn;
        const double Pv = v1 * c + v2 * sn, Qv = v2 * c - v1 * sn;
        const double Pa = a1 * c + a2 * sn, Qa = a2 * c - a1 * sn;
        const double gphi = A * Qr - A * om * Pv - A * om * om * Qa;
        g[P_AMP] += Pr + om * Qv - om * om * Pa;
        g[P_PHASE] += gphi;
        g[P_OMEGA] += tp * gphi + A * Qv - 2.0 * A * om * Pa;
    } else if (S.kind == K_LINEAR_OSC) {
        const double gphi = -A * sn * r1 - A * om * c * v1 + A * om * om * sn * a1;
        g[P_AMP] += r1 * c - om * sn * v1 - om * om * c * a1;
        g[P_PHASE] += gphi;
        g[P_OMEGA] += tp * gphi - A * sn * v1 - 2.0 * A * om * c * a1;
    } else if (S.kind == K_ACCEL) {
        if (tp >= 0.0) g[P_ACCEL] += 0.5 * tp * tp * r1 + tp * v1 + a1;
    } else if (S.kind == K_UNIFORM_VELOCITY) {
        for (int i = 0; i < 3; ++i) g[P_V + i] += rb[i] * tp + vb[i];
    }
}

// The contributions of one charge of family KIND at point x over nt_here times
// (records Rc[ti * nch], cotangent rows cot[(ti * nrows + row) * npts + p]),
// added into g[NP]: per time the retarded kinematics (the FP64 correction
// solves, their fallback on a rebuilt geometry, so the geometry here needs no
// bracket) and their reverse.  The geometry is rebuilt per time: keeping it live
// across the times would take this kernel from 3 to 2 waves per SIMD.  EONLY:
// the cotangent holds the three E rows alone (outputs E), which are all it reads.
template <int KIND, bool EONLY, typename G>
__device__ __forceinline__ void charge_grad(const SrcRec *__restrict__ Rc, int nch, int nt_here, const double x[3],
                                            int64_t p, int64_t npts, int nrows, const int row[10], int field_kind,
                                            int max_iter, double tol_rel, double mask_r, const G *__restrict__ cot,
                                            double g[NP])
{
    for (int ti = 0; ti < nt_here; ++ti) {
        const SrcRec &S = Rc[(int64_t)ti * nch];
        double ob[10];
        bool fin = true;
#pragma unroll
        for (int j = 0; j < 10; ++j) {
            if (EONLY) {
                ob[j] = (j >= 4 && j < 7) ? (double)cot[((int64_t)ti * 3 + (j - 4)) * npts + p] : 0.0;
            } else {
                ob[j] = row[j] >= 0 ? (double)cot[((int64_t)ti * nrows + row[j]) * npts + p] : 0.0;
            }
            fin = fin && isfinite(ob[j]);
        }
        // the cotangent is tested after the solve, which does not depend on it,
        // so that its loads are in flight during the solve
        Geo geo;
        geo_prepare_k<KIND, false, true>(S, x, geo);
        Kin k;
        retarded_kind<true, true, KIND>(S, geo, x, max_iter, tol_rel, k);
        const double D2 = k.R[0] * k.R[0] + k.R[1] * k.R[1] + k.R[2] * k.R[2];
        if (!fin || !(D2 >= mask_r * mask_r) || D2 == 0.0) continue;
        pair_param_grad<EONLY>(S, k, field_kind, ob, g);
    }
}

template <typename G, bool EONLY>
__global__ __launch_bounds__(256) void fields_vjp_kernel(const SrcRec *__restrict__ recs, int nch,
                                                         const double *__restrict__ pts, int64_t npts, int nt,
                                                         int tchunk, int field_kind, int outputs, int nrows,
                                                         int max_iter, double tol_rel, double mask_r,
                                                         const G *__restrict__ cot, double *__restrict__ partial)
{
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int64_t p = (int64_t)blockIdx.x * 256 + tid;
    const bool live = p < npts;
    double x[3] = {0.0, 0.0, 0.0};
    if (live) {
        x[0] = pts[p];
        x[1] = pts[npts + p];
        x[2] = pts[2 * npts + p];
    }
    const int t0 = blockIdx.y * tchunk;
    const int t1 = min(t0 + tchunk, nt);
    const int64_t blk = (int64_t)blockIdx.y * gridDim.x + blockIdx.x;
    // cotangent row of each of the 10 outputs (-1: not requested, cotangent 0)
    int row[10];
    {
        int r = 0;
        row[0] = (outputs & OUT_PHI) ? r++ : -1;
        for (int q = 1; q < 4; ++q) row[q] = (outputs & OUT_A) ? r++ : -1;
        for (int q = 4; q < 7; ++q) row[q] = (outputs & OUT_E) ? r++ : -1;
        for (int q = 7; q < 10; ++q) row[q] = (outputs & OUT_B) ? r++ : -1;
    }
    for (int c = 0; c < nch; ++c) {
        double g[NP];
#pragma unroll
        for (int j = 0; j < NP; ++j) g[j] = 0.0;
        if (live) {
            // every time's record of a charge carries the charge's family, so
            // the solver is chosen once per charge
            const SrcRec *Rc = recs + (int64_t)t0 * nch + c;
            switch (Rc->kind) {
            case K_CIRCULAR:
                charge_grad<K_CIRCULAR, EONLY>(Rc, nch, t1 - t0, x, p, npts, nrows, row, field_kind, max_iter, tol_rel,
                                        mask_r, cot + (int64_t)t0 * nrows * npts, g);
                break;
            case K_LINEAR_OSC:
                charge_grad<K_LINEAR_OSC, EONLY>(Rc, nch, t1 - t0, x, p, npts, nrows, row, field_kind, max_iter, tol_rel,
                                          mask_r, cot + (int64_t)t0 * nrows * npts, g);
                break;
            case K_ACCEL:
                charge_grad<K_ACCEL, EONLY>(Rc, nch, t1 - t0, x, p, npts, nrows, row, field_kind, max_iter, tol_rel,
                                     mask_r, cot + (int64_t)t0 * nrows * npts, g);
                break;
            case K_UNIFORM_VELOCITY:
                charge_grad<K_UNIFORM_VELOCITY, EONLY>(Rc, nch, t1 - t0, x, p, npts, nrows, row, field_kind, max_iter,
                                                tol_rel, mask_r, cot + (int64_t)t0 * nrows * npts, g);
                break;
            default:
                charge_grad<K_STATIONARY, EONLY>(Rc, nch, t1 - t0, x, p, npts, nrows, row, field_kind, max_iter, tol_rel,
                                          mask_r, cot + (int64_t)t0 * nrows * npts, g);
                break;
            }
        }
        // the wave's sum by a shuffle tree (every lane ends with the totals), and
        // lane j writes parameter j's: one partial per (wave, charge), no barrier
        double mine = 0.0;
#pragma unroll
        for (int j = 0; j < NP; ++j) {
            double v = g[j];
            for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
            if (lane == j) mine = v;
        }
        if (lane < NP) partial[((blk * WAVES + wave) * nch + c) * NP + lane] = mine;
    }
}

// One workgroup per output: strided partial sums per lane, then a tree, all in
// a fixed order (bitwise reproducible).
__global__ __launch_bounds__(256) void vjp_reduce_kernel(const double *__restrict__ partial, int64_t nblk, int nout,
                                                         double *__restrict__ grad)
{
    __shared__ double red[256];
    const int o = blockIdx.x, tid = threadIdx.x;
    double s = 0.0;
    for (int64_t b = tid; b < nblk; b += 256) s += partial[b * nout + o];
    red[tid] = s;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if (tid < off) red[tid] += red[tid + off];
        __syncthreads();
    }
    if (tid == 0) grad[o] = red[0];
}

int vjp_params() { return NP; }

size_t vjp_partial_doubles(int64_t npts, int nt, int nch, int tchunk)
{
    const int64_t gx = (npts + 255) / 256, gy = (nt + tchunk - 1) / tchunk;
    return (size_t)(gx * gy * WAVES) * (size_t)nch * NP;
}

hipError_t launch_fields_vjp(const SrcRec *d_recs, int nch, const double *d_pts, int64_t npts, int nt,
                             const lw_opts &o, double tol_rel, double mask_r, const void *d_cot, double *d_partial,
                             int tchunk, double *d_grad, hipStream_t s)
{
    const dim3 grid((unsigned)((npts + 255) / 256), (unsigned)((nt + tchunk - 1) / tchunk));
    const int max_iter = o.max_iter > 0 ? o.max_iter : 100;
    const int om = output_mask(o.outputs), nrows = output_rows(o.outputs);
    // a cotangent of E alone (objectives of |E|^2) takes the kernel that reads
    // and reverses only E
    const bool eonly = om == OUT_E;
    if (o.precision == LW_MIXED) {
        if (eonly)
            hipLaunchKernelGGL((fields_vjp_kernel<float, true>), grid, dim3(256), 0, s, d_recs, nch, d_pts, npts, nt,
                               tchunk, o.field_kind, om, nrows, max_iter, tol_rel, mask_r, (const float *)d_cot,
                               d_partial);
        else
            hipLaunchKernelGGL((fields_vjp_kernel<float, false>), grid, dim3(256), 0, s, d_recs, nch, d_pts, npts,
                               nt, tchunk, o.field_kind, om, nrows, max_iter, tol_rel, mask_r, (const float *)d_cot,
                               d_partial);
    } else {
        if (eonly)
            hipLaunchKernelGGL((fields_vjp_kernel<double, true>), grid, dim3(256), 0, s, d_recs, nch, d_pts, npts,
                               nt, tchunk, o.field_kind, om, nrows, max_iter, tol_rel, mask_r, (const double *)d_cot,
                               d_partial);
        else
            hipLaunchKernelGGL((fields_vjp_kernel<double, false>), grid, dim3(256), 0, s, d_recs, nch, d_pts, npts,
                               nt, tchunk, o.field_kind, om, nrows, max_iter, tol_rel, mask_r, (const double *)d_cot,
                               d_partial);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int nout = nch * NP;
    const int64_t nblk = (int64_t)grid.x * grid.y * WAVES;      // partial rows, one per wave
    hipLaunchKernelGGL(vjp_reduce_kernel, dim3(nout), dim3(256), 0, s, d_partial, nblk, nout, d_grad);
    return hipGetLastError();
}

}  // namespace lw
