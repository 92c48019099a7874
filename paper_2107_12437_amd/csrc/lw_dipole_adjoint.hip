// lw_dipole_adjoint.hip -- gradient of a detector objective with respect to the
// oscillator positions, by a backward-in-time discrete adjoint of the run.
//
// Objective: J = (1/n_snap) sum_k sum_p |E(r_p, t_k)|^2, E the total field of all
// oscillator charges at detector points r_p and snapshot times t_k, read from
// the stored history at their retarded times (Secs. 2.1-2.3).
//
// The run (Algorithm 1) is a discrete map: per step n each dipole's
// y = (d, d_dot) advances by classic RK4, which for Eq. (LO_equation) is linear:
//   y[n+1] = M y[n] + b_c Ec[n] + b_m Em[n] + b_e Ee[n],
// with the drives Em, Ee read from the other dipoles' history samples
// h_j[k] = (d, d_dot, d_ddot)_j at the retarded times, Ec[n+1] = Ee[n] and
// d_ddot[n+1] = f Ee[n] - gamma0 d_dot[n+1] - omega0^2 d[n+1].  The adjoint runs
// the steps backwards: the RK4 transpose gives the cotangents of Em, Ee, Ec, and
// each drive pair's vector-Jacobian product scatters them onto the source's
// history samples (the adjoint history, read back once the backward sweep
// reaches that step) and onto the positions.  Every pair's retarded time is
// differentiated by the implicit-function theorem on
//   g = c tau - |Delta - cf d(t - tau) p_j| = 0,  Delta = R_i - R_j,
// with d(t') the interpolated (or extrapolated, or pre-history) stored moment.
// Either the whole history of the forward run is kept in device memory (24
// bytes per dipole per step), or the sweep runs over segments recomputed from
// run states (checkpointing): then the history and its cotangents live in a
// ring of one segment plus the retarded look-back (hist_rows_kernel,
// hist_from_state_kernel), and each cotangent slot is cleared once read.
#include <math.h>

#include "lw_device.hpp"
#include "lw_dipole.hpp"
#include "lw_internal.hpp"

namespace lw {

// Value and t'-derivative of the stored moment, its rate and acceleration at s
// steps, and where they came from (for scattering cotangents back).
struct HistEval {
    double d, v, a;        // at t'
    double sd, sv, sa;     // d/dt' of each
    int region;            // 0 before t = 0, 1 between samples k and k+1, 2 beyond the newest sample k
    int64_t k;
    double u;              // region 1: weight of sample k+1; region 2: time past sample k
};

__device__ __forceinline__ void hist_eval(const Hist &H, int j, double d0, int64_t nstep, double s, HistEval &e)
{
    if (s < 0.0) {
        e.d = d0;
        e.v = e.a = e.sd = e.sv = e.sa = 0.0;
        e.region = 0;
        e.k = 0;
        e.u = 0.0;
        return;
    }
    const double fk = floor(s);
    const int64_t k = (int64_t)fk;
    if (k >= nstep) {
        const double *h = H.ring + ((int64_t)(nstep & H.mask) * H.n + j) * 3;
        const double tt = (s - (double)nstep) * H.dt;
        e.d = h[0] + h[1] * tt + 0.5 * h[2] * tt * tt;
        e.v = h[1] + h[2] * tt;
        e.a = h[2];
        e.sd = e.v;
        e.sv = h[2];
        e.sa = 0.0;
        e.region = 2;
        e.k = nstep;
        e.u = tt;
        return;
    }
    const double u = s - fk;
    const double *h0 = H.ring + ((int64_t)(k & H.mask) * H.n + j) * 3;
    const double *h1 = H.ring + ((int64_t)((k + 1) & H.mask) * H.n + j) * 3;
    e.d = (1.0 - u) * h0[0] + u * h1[0];
    e.v = (1.0 - u) * h0[1] + u * h1[1];
    e.a = (1.0 - u) * h0[2] + u * h1[2];
    e.sd = (h1[0] - h0[0]) * H.inv_dt;
    e.sv = (h1[1] - h0[1]) * H.inv_dt;
    e.sa = (h1[2] - h0[2]) * H.inv_dt;
    e.region = 1;
    e.k = k;
    e.u = u;
}

// hist_eval at s from the segment the closed form already loaded, when s lies
// in it (the same values and operations, without reading the samples again).
__device__ __forceinline__ void seg_eval(const Hist &H, int j, const Seg &g, double d0, int64_t nstep, double s,
                                         HistEval &e)
{
    const double fk = floor(s);
    const int64_t k = (int64_t)fk;
    if (s < 0.0 || k >= nstep || k != g.k) {
        hist_eval(H, j, d0, nstep, s, e);
        return;
    }
    const double u = s - fk;
    e.d = (1.0 - u) * g.d0 + u * g.d1;
    e.v = (1.0 - u) * g.v0 + u * g.v1;
    e.a = (1.0 - u) * g.a0 + u * g.a1;
    e.sd = (g.d1 - g.d0) * H.inv_dt;
    e.sv = (g.v1 - g.v0) * H.inv_dt;
    e.sa = (g.a1 - g.a0) * H.inv_dt;
    e.region = 1;
    e.k = k;
    e.u = u;
}

// Retarded field of charge (cf, kq) of source j at point x and time base*dt
// (samples up to nstep); fills the kinematics and the history evaluation.
// tau_init (> 0) starts Newton; tau_out receives Newton's root and is left
// alone when the closed form settles the pair.
__device__ void pair_solve(const Hist &H, const double x[3], const DipLds &Sj, int j, double cf, int64_t nstep,
                           double base, int max_iter, Kin &k, HistEval &e, uint32_t &err, double tau_init = 0.0,
                           double *tau_out = nullptr)
{
    const double dx = x[0] - Sj.ox, dy = x[1] - Sj.oy, dz = x[2] - Sj.oz;
    const double L2 = dx * dx + dy * dy + dz * dz;
    const double L = sqrt(L2);
    const double sD = dx * Sj.px + dy * Sj.py + dz * Sj.pz;
    Bracket b(0.0, 2.0 * L * INV_C);
    double tau = L * INV_C;
    const double tol = 4.0 * 2.220446049250313e-16;
    bool ok = false, closed = false;
    // the closed form on the interpolated history (retarded_seg) from the
    // segment of tau = L/c (the charge sits within |rho| << L of its origin, so
    // that is the root's segment or a neighbour); Newton past the newest
    // stored step, warm-started from the same pair's retarded time one step
    // later if given (read only there)
    {
        const double s0 = base - tau * H.inv_dt;
        const int64_t k0 = s0 < 0.0 ? -1 : (int64_t)floor(s0);
        if (k0 < nstep) {
            Seg g;
            seg_load(H, j, Sj.d0, nstep, k0, g, err);
            double hh[3], tc;
            if (retarded_seg(H, j, Sj.d0, nstep, base, L2, sD, cf, g, hh, tc, err)) {
                tau = tc;
                seg_eval(H, j, g, Sj.d0, nstep, base - tau * H.inv_dt, e);
                ok = true;
                closed = true;
            }
        }
    }
    if (!ok && tau_init > 0.0 && tau_init < b.hi) tau = tau_init;
    for (int it = 0; it < max_iter && !ok; ++it) {
        const double s = base - tau * H.inv_dt;
        hist_eval(H, j, Sj.d0, nstep, s, e);
        const double rho = cf * e.d;
        const double D = sqrt(fmax(L2 - 2.0 * rho * sD + rho * rho, 0.0));
        const double r1 = cf * e.sd;                             // d rho / d t'
        const double dD = (D > 0.0) ? r1 * (sD - rho) * rcp_steer(D) : 0.0;
        bool free_step;
        const double tn = halley_step(tau, D, dD, 0.0, b, free_step);
        ok = converged(tn, tau, tol, b);
        if (ok) break;
        // within one interpolation segment (or one side of the history's ends)
        // g is smooth with |g''| <= rho'^2 / D + |rho''|: once Newton's error
        // bound from tau is below tol/4 the new iterate is accepted, and the
        // history is evaluated there once more
        const double st = tn - tau;
        const double r2 = (e.region == 2) ? cf * e.sv : 0.0;
        const double sn = base - tn * H.inv_dt;
        const bool same_seg = (e.region == 1) ? (floor(sn) == floor(s) && sn < (double)nstep)
                                              : (e.region == 2 ? sn >= (double)nstep : sn < 0.0);
        tau = tn;
        if (free_step && same_seg && D > 0.0 &&
            (r1 * r1 + fabs(r2) * D) * (st * st) <= 0.5 * tol * tn * D * (C_LIGHT - fabs(r1))) {
            hist_eval(H, j, Sj.d0, nstep, sn, e);
            ok = true;
            break;
        }
    }
    if (!ok) err |= ERR_NOCONV;
    if (tau_out && !closed) *tau_out = tau;        // Newton's root, the next step's start
    const double rho = cf * e.d;
    k.R[0] = dx - rho * Sj.px;
    k.R[1] = dy - rho * Sj.py;
    k.R[2] = dz - rho * Sj.pz;
    k.v[0] = cf * e.v * Sj.px;
    k.v[1] = cf * e.v * Sj.py;
    k.v[2] = cf * e.v * Sj.pz;
    k.a[0] = cf * e.a * Sj.px;
    k.a[1] = cf * e.a * Sj.py;
    k.a[2] = cf * e.a * Sj.pz;
    k.tp = 0.0;
    k.cph = 1.0;
    k.sph = 0.0;
    k.flags = 0u;
}

// Cotangents of the history samples one pair read: samples k and k+1
// (interpolation), sample k alone (Taylor step past the newest sample), or none
// (static pre-history).
struct HistBar {
    int region;
    int64_t k;
    double c0[3], c1[3];
};

// Reverse of pair_solve + the field: given the cotangent Eb of the pair's E,
// returns the cotangent of Delta = x - R_j and the cotangents of the samples.
__device__ void pair_vjp(const Kin &k, const HistEval &e, const DipLds &Sj, double cf, double kq, const double Eb[3],
                         double Db[3], HistBar &hb)
{
    const double ob[10] = {0.0, 0.0, 0.0, 0.0, Eb[0], Eb[1], Eb[2], 0.0, 0.0, 0.0};
    double Rb[3], vb[3], ab[3], n[3], kqb, kappa;
    lw_terms_vjp(k, kq, F_TOTAL, ob, Rb, vb, ab, kqb, n, kappa);
    const double Rp = Rb[0] * Sj.px + Rb[1] * Sj.py + Rb[2] * Sj.pz;
    const double vp = vb[0] * Sj.px + vb[1] * Sj.py + vb[2] * Sj.pz;
    const double ap = ab[0] * Sj.px + ab[1] * Sj.py + ab[2] * Sj.pz;
    const double np = n[0] * Sj.px + n[1] * Sj.py + n[2] * Sj.pz;
    // R = Delta - cf d(t - tau) p,  v = cf d_dot(t - tau) p,  a = cf d_ddot(t - tau) p
    const double stau = cf * (e.sd * Rp - e.sv * vp - e.sa * ap);      // d J / d tau at fixed samples
    const double gp = C_LIGHT - cf * e.sd * np;                          // d g / d tau
    const double q = stau / gp;
    for (int i = 0; i < 3; ++i) Db[i] = Rb[i] + q * n[i];
    hb.region = e.region;
    hb.k = e.k;
    if (e.region == 0) return;                                            // static pre-history: no samples
    const double db = -cf * Rp - q * cf * np;                             // cotangent of d(t') at fixed t'
    const double vbb = cf * vp, abb = cf * ap;
    if (e.region == 1) {
        const double w0 = 1.0 - e.u, w1 = e.u;
        hb.c0[0] = w0 * db;
        hb.c0[1] = w0 * vbb;
        hb.c0[2] = w0 * abb;
        hb.c1[0] = w1 * db;
        hb.c1[1] = w1 * vbb;
        hb.c1[2] = w1 * abb;
    } else {
        // Taylor step from sample k: d = d_k + v_k tt + a_k tt^2/2, v = v_k + a_k tt, a = a_k
        const double tt = e.u;
        hb.c0[0] = db;
        hb.c0[1] = tt * db + vbb;
        hb.c0[2] = 0.5 * tt * tt * db + tt * vbb + abb;
        hb.c1[0] = hb.c1[1] = hb.c1[2] = 0.0;
    }
}

// Adds a pair's sample cotangents into hbar ([ring][n][3]) with device atomics.
__device__ __forceinline__ void scatter_global(const Hist &H, int j, const HistBar &hb, double *hbar)
{
    if (hb.region == 0) return;
    double *h0 = hbar + ((int64_t)(hb.k & H.mask) * H.n + j) * 3;
    for (int c = 0; c < 3; ++c) atomicAdd(h0 + c, hb.c0[c]);
    if (hb.region == 1) {
        double *h1 = hbar + ((int64_t)((hb.k + 1) & H.mask) * H.n + j) * 3;
        for (int c = 0; c < 3; ++c) atomicAdd(h1 + c, hb.c1[c]);
    }
}

// History samples row0 .. row0 + nrows - 1 from a stride-1 run's outputs into
// a ring of `ring` steps ([ring][n_dip][3]).
__global__ void hist_rows_kernel(const DipDev *__restrict__ dev, const double *__restrict__ D,
                                 const double *__restrict__ V, const double *__restrict__ Ed, int n_dip, int64_t nrows,
                                 int64_t row0, int ring, double *__restrict__ hist)
{
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= nrows * n_dip) return;
    const int64_t row = idx / n_dip;
    const int i = (int)(idx - row * n_dip);
    const DipDev &P = dev[i];
    const double d = D[idx], v = V[idx];
    double *h = hist + (((row0 + row) & (int64_t)(ring - 1)) * n_dip + i) * 3;
    h[0] = d;
    h[1] = v;
    h[2] = P.f * Ed[idx] - P.gamma0 * v - P.omega0 * P.omega0 * d;
}

// History samples lo .. hi (at most the run state's depth) from a run state's
// per-instance rings into the adjoint's ring ([ring][n_dip][3]).
__global__ void hist_from_state_kernel(const double *__restrict__ state, const int32_t *__restrict__ off, int n_inst,
                                       int n_dip, int ring_state, int64_t lo, int64_t hi, int ring,
                                       double *__restrict__ hist)
{
    const int64_t nk = hi - lo + 1;
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (nk <= 0 || idx >= nk * n_dip) return;
    const int64_t k = lo + idx / n_dip;
    const int g = (int)(idx % n_dip);
    const int inst = instance_of(off, n_inst, g);
    const int a0 = off[inst], n = off[inst + 1] - a0;
    const double *src = state + state_ring_off(a0, ring_state) + ((k & (int64_t)(ring_state - 1)) * n + (g - a0)) * 3;
    double *dst = hist + ((k & (int64_t)(ring - 1)) * n_dip + g) * 3;
    dst[0] = src[0];
    dst[1] = src[1];
    dst[2] = src[2];
}

// Detector field, objective partials and the detector's cotangents: one lane
// per (snapshot, point); instances are laid out in the history by the global
// dipole index (one shared [ring][n_dip][3] array).  The lanes of a workgroup
// see a source at nearby retarded times, so their sample cotangents are first
// summed in LDS, then added to hbar with one device atomic per touched slot.
// Sources are taken DET_JG at a time, each with its own window of DET_SJ
// samples, whose start is the workgroup's earliest possible sample of that
// source from geometry (floor(t / dt - L / (c dt)) - 2, minimised over the
// lanes; the charges sit far less than 2 c dt from their origins).  So the
// sources' reverses need no barrier between them: three per group of sources
// (a lane whose sample falls outside its window adds it to hbar directly).
constexpr int DET_JG = 32, DET_SJ = 48;

__global__ __launch_bounds__(256) void detector_vjp_kernel(const DipDev *__restrict__ dev, int n_dip,
                                                           const double *__restrict__ hist, double *__restrict__ hbar,
                                                           int ring, int64_t nstep, double dt,
                                                           const double *__restrict__ pts, int64_t npts,
                                                           const double *__restrict__ times, int n_snap, int n_norm,
                                                           double *__restrict__ Rbar, double *__restrict__ Jpart,
                                                           int max_iter, uint32_t *__restrict__ d_err)
{
    __shared__ double red[4];
    __shared__ double slot[DET_JG * DET_SJ * 3];
    __shared__ int kb_s[2][DET_JG];                 // window starts, by group parity
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int64_t gid = (int64_t)blockIdx.x * 256 + tid;
    const bool live = gid < npts * n_snap;
    const int64_t p = live ? gid % npts : 0;
    const int ks = live ? (int)(gid / npts) : 0;
    const double x[3] = {pts[p], pts[npts + p], pts[2 * npts + p]};
    const double base = times[ks] / dt;
    Hist H{hist, n_dip, ring - 1, dt, 1.0 / dt};
    uint32_t err = 0u;
    for (int t = tid; t < DET_JG * DET_SJ * 3; t += 256) slot[t] = 0.0;
    for (int t = tid; t < 2 * DET_JG; t += 256) kb_s[t / DET_JG][t % DET_JG] = INT_MAX;
    double E[3] = {0.0, 0.0, 0.0};
    if (live) {
        for (int j = 0; j < n_dip; ++j) {
            const DipDev &Dj = dev[j];
            const DipLds Sj = dip_lds(Dj);
            for (int w = 0; w < 2; ++w) {
                const double cf = w ? Sj.cfm : Sj.cfp;
                const double kq = (w ? -Dj.q : Dj.q) * K_COUL;
                Kin k;
                HistEval e;
                pair_solve(H, x, Sj, j, cf, nstep, base, max_iter, k, e, err);
                double o[10];
                lw_terms<double>(k, kq, F_TOTAL, o);
                E[0] += o[4];
                E[1] += o[5];
                E[2] += o[6];
            }
        }
    }
    // objective partial per workgroup (fixed order)
    double jv = live ? (E[0] * E[0] + E[1] * E[1] + E[2] * E[2]) / n_norm : 0.0;
    for (int off = 32; off > 0; off >>= 1) jv += __shfl_xor(jv, off, 64);
    if (lane == 0) red[wave] = jv;
    __syncthreads();
    if (tid == 0) Jpart[blockIdx.x] = ((red[0] + red[1]) + red[2]) + red[3];
    // cotangent of E and its scatter, DET_JG sources at a time
    const double Eb[3] = {2.0 * E[0] / n_norm, 2.0 * E[1] / n_norm, 2.0 * E[2] / n_norm};
    for (int j0 = 0, par = 0; j0 < n_dip; j0 += DET_JG, par ^= 1) {
        const int jn = min(DET_JG, n_dip - j0);
        int *kb = kb_s[par];
        if (live)
            for (int jl = 0; jl < jn; ++jl) {
                const DipDev &Dj = dev[j0 + jl];
                const double dx = x[0] - Dj.origin[0], dy = x[1] - Dj.origin[1], dz = x[2] - Dj.origin[2];
                const double L = sqrt(dx * dx + dy * dy + dz * dz);
                atomicMin(&kb[jl], (int)floor(base - L * INV_C * H.inv_dt) - 2);
            }
        // the other parity's starts are free again: the previous group's flush is done
        for (int t = tid; t < DET_JG; t += 256) kb_s[par ^ 1][t] = INT_MAX;
        __syncthreads();
        for (int jl = 0; jl < jn; ++jl) {
            const int j = j0 + jl;
            const DipDev &Dj = dev[j];
            const DipLds Sj = dip_lds(Dj);
            const int64_t kbj = kb[jl];
            double Rj[3] = {0.0, 0.0, 0.0};
            if (live)
                for (int w = 0; w < 2; ++w) {
                    const double cf = w ? Sj.cfm : Sj.cfp;
                    const double kq = (w ? -Dj.q : Dj.q) * K_COUL;
                    Kin k;
                    HistEval e;
                    pair_solve(H, x, Sj, j, cf, nstep, base, max_iter, k, e, err);
                    double Db[3];
                    HistBar hb;
                    pair_vjp(k, e, Sj, cf, kq, Eb, Db, hb);
                    // Delta = x - R_j: the source position gets -Db
                    Rj[0] -= Db[0];
                    Rj[1] -= Db[1];
                    Rj[2] -= Db[2];
                    if (hb.region == 0) continue;
                    const int64_t sl = hb.k - kbj;
                    if (sl >= 0 && sl + 1 < DET_SJ) {
                        double *r = slot + ((int64_t)jl * DET_SJ + sl) * 3;
                        for (int c = 0; c < 3; ++c) atomicAdd(r + c, hb.c0[c]);
                        if (hb.region == 1)
                            for (int c = 0; c < 3; ++c) atomicAdd(r + 3 + c, hb.c1[c]);
                    } else {
                        scatter_global(H, j, hb, hbar);
                    }
                }
            for (int c = 0; c < 3; ++c) {
                double v = Rj[c];
                for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
                if (lane == 0 && v != 0.0) atomicAdd(&Rbar[j * 3 + c], v);
            }
        }
        __syncthreads();
        for (int t = tid; t < jn * DET_SJ * 3; t += 256) {
            const double v = slot[t];
            if (v != 0.0) {
                const int jl = t / (DET_SJ * 3), r = t - jl * DET_SJ * 3;
                atomicAdd(hbar + ((int64_t)(((int64_t)kb[jl] + r / 3) & H.mask) * H.n + j0 + jl) * 3 + r % 3, v);
                slot[t] = 0.0;
            }
        }
        __syncthreads();
    }
    if (err) atomicOr(d_err, err);
}

// Sum of the per-workgroup objective partials in a fixed order (one workgroup).
__global__ __launch_bounds__(256) void sum_partials_kernel(const double *__restrict__ part, int64_t n,
                                                           double *__restrict__ out)
{
    __shared__ double red[256];
    const int tid = threadIdx.x;
    double s = 0.0;
    for (int64_t i = tid; i < n; i += 256) s += part[i];
    red[tid] = s;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if (tid < off) red[tid] += red[tid + off];
        __syncthreads();
    }
    if (tid == 0) *out = red[0];
}

__device__ __forceinline__ double load_agent(const double *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Per-dipole cotangent state of the backward sweep once steps >= n are
// reversed.  yd, yv: cotangent of the state (d, d_dot) at t_n (partial until
// sample n's own cotangent is added); ec: cotangent of the drive at t_n from
// the first stage of step n; ext: after the sweep, the whole cotangent of the
// drive at t = 0 (sample 0's d_ddot and ec).
struct AdjState {
    double *yd, *yv, *ext, *ec;
};
constexpr int ADJ_FIELDS = 4;

// Transpose of one RK4 step of a dipole (linear in y and in the three stage
// drives): maps the cotangents (yd, yv, ext) of y[n+1] to those of y[n]
// (partial: sample n's own cotangent is added once complete), returned in
// yd, yv, and to the cotangents of the drives Ec, Em, Ee.
__device__ __forceinline__ void rk4_transpose(const DipDev &P, double h, double &yd, double &yv, double ext,
                                              double &Em, double &Ee, double &Ec)
{
    const double w2 = P.omega0 * P.omega0, gm = P.gamma0, f = P.f;
    double k1d = h / 6.0 * yd, k1v = h / 6.0 * yv;
    double k2d = h / 3.0 * yd, k2v = h / 3.0 * yv;
    double k3d = h / 3.0 * yd, k3v = h / 3.0 * yv;
    const double k4d = h / 6.0 * yd, k4v = h / 6.0 * yv;
    double ad = yd, av = yv;
    Ee = ext;
    Em = 0.0;
    Ec = 0.0;
    // k4 = A y4 + e Ee;  y4 = y + h k3
    double td = -w2 * k4v, tv = k4d - gm * k4v;
    Ee += f * k4v;
    ad += td; av += tv; k3d += h * td; k3v += h * tv;
    // k3 = A y3 + e Em;  y3 = y + h/2 k2
    td = -w2 * k3v; tv = k3d - gm * k3v;
    Em += f * k3v;
    ad += td; av += tv; k2d += 0.5 * h * td; k2v += 0.5 * h * tv;
    // k2 = A y2 + e Em;  y2 = y + h/2 k1
    td = -w2 * k2v; tv = k2d - gm * k2v;
    Em += f * k2v;
    ad += td; av += tv; k1d += 0.5 * h * td; k1v += 0.5 * h * tv;
    // k1 = A y + e Ec
    ad += -w2 * k1v; av += k1d - gm * k1v;
    Ec += f * k1v;
    yd = ad;
    yv = av;
}

// Adds the completed cotangent of sample n (d, d_dot, d_ddot = f Ec - gamma0
// d_dot - omega0^2 d) of dipole g: into y[n] unless n = 0 (y[0] is fixed), and
// into the drive at t_n (ext for the step before); clears the slot.
__device__ __forceinline__ void take_sample(const DipDev &P, double *hbar, int64_t n, int n_dip, int mask,
                                            AdjState &A, int g)
{
    double *hb = hbar + ((int64_t)(n & mask) * n_dip + g) * 3;
    const double bd = load_agent(hb), bv = load_agent(hb + 1), ba = load_agent(hb + 2);
    hb[0] = 0.0;
    hb[1] = 0.0;
    hb[2] = 0.0;
    if (n > 0) {
        A.yd[g] += bd - P.omega0 * P.omega0 * ba;
        A.yv[g] += bv - P.gamma0 * ba;
    }
    A.ext[g] = A.ec[g] + P.f * ba;
}

// Start of the sweep: zero cotangent state; the step base starts at the last step.
__global__ void adj_init_kernel(int n_dip, int64_t steps, AdjState A, int64_t *__restrict__ step_base)
{
    for (int g = blockIdx.x * blockDim.x + threadIdx.x; g < n_dip; g += gridDim.x * blockDim.x) {
        A.yd[g] = 0.0;
        A.yv[g] = 0.0;
        A.ext[g] = 0.0;
        A.ec[g] = 0.0;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) *step_base = steps - 1;
}

__global__ void adj_base_kernel(int64_t *__restrict__ step_base, int64_t delta)
{
    if (blockIdx.x == 0 && threadIdx.x == 0) *step_base += delta;
}


// Maps a pair index of the flattened list to (instance, stage, target, source,
// charge).  Per instance of n dipoles: stages x n targets x (n - 1) sources x
// 2 charges, stages first; `pair_off` holds the prefix sums over instances
// (instances without pairs repeat an offset and are never selected).
struct PairIx {
    int i0, n, th, i, j, w;
};
__device__ __forceinline__ PairIx pair_index(const int64_t *pair_off, const int32_t *off, int n_inst, int64_t idx)
{
    int lo = 0, hi = n_inst;                     // last instance with pair_off <= idx
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (pair_off[mid] <= idx) lo = mid; else hi = mid;
    }
    PairIx P;
    P.i0 = off[lo];
    P.n = off[lo + 1] - P.i0;
    const int M = 2 * (P.n - 1);
    const int64_t rem = idx - pair_off[lo];
    const int64_t per_stage = (int64_t)P.n * M;
    P.th = (int)(rem / per_stage);
    const int64_t r2 = rem - P.th * per_stage;
    P.i = (int)(r2 / M);
    const int mm = (int)(r2 - (int64_t)P.i * M);
    const int jj = mm >> 1;
    P.w = mm & 1;
    P.j = jj < P.i ? jj : jj + 1;
    return P;
}

// One step n = *step_base - k of the backward sweep, one workgroup per source
// dipole j.
//  1. Every workgroup of an instance finishes the step's drive cotangents of
//     all the instance's dipoles (read-only): the cotangent state S_{n+1}
//     (buffer (n+1) & 1) plus the completed sample n + 1 (every pair that
//     reads it belongs to a later step, already reversed), transposed through
//     RK4 step n.  Workgroup j alone writes dipole j's S_n (buffer n & 1) and
//     clears its sample n + 2, which the step before was the last to read.
//  2. Every drive pair with source j (targets i != j, charges w, stages
//     t_n + dt/2 and t_n + dt) reverses its field evaluation for a unit drive
//     cotangent; this does not depend on step 1 and runs beside it.  The
//     pair's retarded time is kept in taup as the next (earlier) step's start.
//  3. Each pair scales its products by its target's stage cotangent, adds the
//     (target - source) separation cotangent into its slot of rbp, and its
//     sample cotangents into LDS slots relative to the workgroup's earliest
//     sample.  The slots then go to source j's adjoint history with one
//     device atomic each: only this workgroup writes source j's samples in the
//     step, so the atomics are uncontended (a detector reverse running on
//     another stream may add to the same samples).
constexpr int ADJ_SLOTS = 128;

template <int BLOCK>
__global__ __launch_bounds__(BLOCK) void adj_step_kernel(const DipDev *__restrict__ dev,
                                                         const int32_t *__restrict__ off,
                                                         const int64_t *__restrict__ pair_off, int n_inst, int n_dip,
                                                         const double *__restrict__ hist, double *__restrict__ hbar,
                                                         int mask, double dt, AdjState A0, AdjState A1,
                                                         double *__restrict__ rbp, double *__restrict__ taup,
                                                         const int64_t *__restrict__ step_base, int k, int64_t last,
                                                         int max_iter, const double *__restrict__ soa,
                                                         uint32_t *__restrict__ d_err)
{
    __shared__ double s_es[2][1024];            // stage drive cotangents of the instance's dipoles
    __shared__ double slot[ADJ_SLOTS * 3];
    __shared__ int64_t kmin_w[BLOCK / 64];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int j = blockIdx.x;
    const int64_t nstep = *step_base - k;
    if (nstep < 0) return;
    const int inst = instance_of(off, n_inst, j);
    const int i0 = off[inst], n = off[inst + 1] - i0, jl = j - i0;
    const int M = 2 * (n - 1);
    const bool odd = (nstep & 1) != 0;
    const AdjState &Ain = odd ? A0 : A1;        // S_{n+1}
    const AdjState &Aout = odd ? A1 : A0;       // S_n
    uint32_t err = 0u;
    const Hist H{hist, n_dip, mask, dt, 1.0 / dt};
    const DipLds Sj = soa_lds(soa, n_dip, (uint32_t)j);
    const double qj = soa_get(soa, n_dip, SF_Q, (uint32_t)j);
    for (int t = tid; t < ADJ_SLOTS * 3; t += BLOCK) slot[t] = 0.0;
    // 2. the pair work (first pair of each lane)
    int m2 = tid;
    double Du[3] = {0.0, 0.0, 0.0};
    HistBar hu;
    hu.region = 0;
    hu.k = 0;
    int th = 0, il = 0;
    int64_t idx = 0;
    double rb[3] = {0.0, 0.0, 0.0};     // the pair's separation cotangent so far, read early
    auto solve_unit = [&](int mm2) {
        th = mm2 >= M ? 1 : 0;                      // (2 M units: two stages)
        const int m = mm2 - th * M;
        const int ii = m >> 1, w = m & 1;
        il = ii < jl ? ii : ii + 1;                   // target (local index)
        const uint32_t gi = (uint32_t)(i0 + il);
        const double x[3] = {soa_get(soa, n_dip, SF_OX, gi), soa_get(soa, n_dip, SF_OY, gi),
                             soa_get(soa, n_dip, SF_OZ, gi)};
        const double Eu[3] = {soa_get(soa, n_dip, SF_PX, gi), soa_get(soa, n_dip, SF_PY, gi),
                              soa_get(soa, n_dip, SF_PZ, gi)};       // unit drive cotangent
        const double cf = w ? Sj.cfm : Sj.cfp;
        const double kq = (w ? -qj : qj) * K_COUL;
        const int jj = jl < il ? jl : jl - 1;         // the source's place in the target's list
        idx = pair_off[inst] + ((int64_t)th * n + il) * M + 2 * jj + w;
        rb[0] = rbp[idx * 3];
        rb[1] = rbp[idx * 3 + 1];
        rb[2] = rbp[idx * 3 + 2];
        const double tw = taup[idx];
        Kin kn;
        HistEval e;
        double tau = tw;
        pair_solve(H, x, Sj, j, cf, nstep, (double)nstep + (th ? 1.0 : 0.5), max_iter, kn, e, err, tw, &tau);
        if (tau != tw) taup[idx] = tau;     // (only Newton reads it; the closed form leaves it)
        pair_vjp(kn, e, Sj, cf, kq, Eu, Du, hu);
    };
    // step 1's first dipole: its loads go out before the pair work, which does
    // not depend on them
    double pb[3] = {0.0, 0.0, 0.0}, py[3] = {0.0, 0.0, 0.0};
    if (tid < n) {
        const int gq = i0 + tid;
        const double *hb = hbar + ((int64_t)((nstep + 1) & mask) * n_dip + gq) * 3;
        pb[0] = load_agent(hb);
        pb[1] = load_agent(hb + 1);
        pb[2] = load_agent(hb + 2);
        py[0] = Ain.yd[gq];
        py[1] = Ain.yv[gq];
        py[2] = Ain.ec[gq];
    }
    if (m2 < 2 * M) solve_unit(m2);
    // 1. the instance's drive cotangents; dipole j's S_n
    for (int ql = tid; ql < n; ql += BLOCK) {
        const int gq = i0 + ql;
        const DipDev &P = dev[gq];
        if (ql != tid) {
            const double *hb = hbar + ((int64_t)((nstep + 1) & mask) * n_dip + gq) * 3;
            pb[0] = load_agent(hb);
            pb[1] = load_agent(hb + 1);
            pb[2] = load_agent(hb + 2);
            py[0] = Ain.yd[gq];
            py[1] = Ain.yv[gq];
            py[2] = Ain.ec[gq];
        }
        const double bd = pb[0], bv = pb[1], ba = pb[2];
        double yd = py[0] + (bd - P.omega0 * P.omega0 * ba);
        double yv = py[1] + (bv - P.gamma0 * ba);
        const double ext = py[2] + P.f * ba;
        double em, ee, ec;
        rk4_transpose(P, dt, yd, yv, ext, em, ee, ec);
        s_es[0][ql] = em;
        s_es[1][ql] = ee;
        if (gq == j) {
            Aout.yd[gq] = yd;
            Aout.yv[gq] = yv;
            Aout.ec[gq] = ec;
            if (nstep + 2 <= last) {
                double *hc = hbar + ((int64_t)((nstep + 2) & mask) * n_dip + gq) * 3;
                hc[0] = 0.0;
                hc[1] = 0.0;
                hc[2] = 0.0;
            }
        }
    }
    // earliest sample the workgroup's first pairs touch
    int64_t km = (m2 < 2 * M && hu.region) ? hu.k : INT64_MAX;
    for (int o = 32; o > 0; o >>= 1) km = min(km, (int64_t)__shfl_xor(km, o, 64));
    if (lane == 0) kmin_w[wave] = km;
    __syncthreads();
    int64_t kb = kmin_w[0];
    for (int v = 1; v < BLOCK / 64; ++v) kb = min(kb, kmin_w[v]);
    // 3. scale, separation cotangents, sample cotangents into the slots
    for (; m2 < 2 * M; m2 += BLOCK) {
        if (m2 != tid) solve_unit(m2);
        const double Es = s_es[th][il];
        double *r = rbp + idx * 3;
        r[0] = rb[0] + Es * Du[0];
        r[1] = rb[1] + Es * Du[1];
        r[2] = rb[2] + Es * Du[2];
        if (hu.region == 0) continue;
        HistBar hb = hu;
        for (int c = 0; c < 3; ++c) {
            hb.c0[c] = Es * hu.c0[c];
            hb.c1[c] = Es * hu.c1[c];
        }
        const int64_t sl = hb.k - kb;
        if (sl >= 0 && sl + 1 < ADJ_SLOTS) {
            for (int c = 0; c < 3; ++c) atomicAdd(&slot[sl * 3 + c], hb.c0[c]);
            if (hb.region == 1)
                for (int c = 0; c < 3; ++c) atomicAdd(&slot[(sl + 1) * 3 + c], hb.c1[c]);
        } else {
            scatter_global(H, j, hb, hbar);
        }
    }
    __syncthreads();
    if (kb != INT64_MAX)
        for (int t = tid; t < ADJ_SLOTS * 3; t += BLOCK) {
            const double v = slot[t];
            if (v != 0.0) atomicAdd(hbar + ((int64_t)((kb + t / 3) & mask) * n_dip + j) * 3 + t % 3, v);
        }
    if (err) atomicOr(d_err, err);
}

// After the sweep: sample 0 gives the cotangent of E_d(0) (y[0] is fixed).
__global__ void adj_finish_kernel(const DipDev *__restrict__ dev, int n_dip, double *__restrict__ hbar, int mask,
                                  AdjState A)
{
    for (int g = blockIdx.x * blockDim.x + threadIdx.x; g < n_dip; g += gridDim.x * blockDim.x)
        take_sample(dev[g], hbar, 0, n_dip, mask, A, g);
}

// E_d(0): the drive from the static pre-history depends on the positions only;
// its cotangent is ext after the sweep.  One stage per pair.
template <int BLOCK>
__global__ __launch_bounds__(BLOCK) void adj_drive0_kernel(const DipDev *__restrict__ dev,
                                                           const int32_t *__restrict__ off,
                                                           const int64_t *__restrict__ pair_off0, int n_inst,
                                                           int64_t n_pairs0, int n_dip, const double *__restrict__ hist,
                                                           int mask, double dt, AdjState A, double *__restrict__ rbp0,
                                                           int max_iter, uint32_t *__restrict__ d_err)
{
    const int64_t idx = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    if (idx >= n_pairs0) return;
    uint32_t err = 0u;
    const Hist H{hist, n_dip, mask, dt, 1.0 / dt};
    const PairIx P = pair_index(pair_off0, off, n_inst, idx);
    const int gi = P.i0 + P.i, gj = P.i0 + P.j;
    const double Es = A.ext[gi];
    double Db[3] = {0.0, 0.0, 0.0};
    if (Es != 0.0) {
        const DipDev &Di = dev[gi];
        const DipDev &Dj = dev[gj];
        const DipLds Sj = dip_lds(Dj);
        const double cf = P.w ? Sj.cfm : Sj.cfp;
        const double kq = (P.w ? -Dj.q : Dj.q) * K_COUL;
        const double x[3] = {Di.origin[0], Di.origin[1], Di.origin[2]};
        Kin k;
        HistEval e;
        pair_solve(H, x, Sj, gj, cf, 0, 0.0, max_iter, k, e, err);
        const double Eb[3] = {Es * Di.axis[0], Es * Di.axis[1], Es * Di.axis[2]};
        HistBar hb;
        pair_vjp(k, e, Sj, cf, kq, Eb, Db, hb);      // pre-history: no sample cotangents
    }
    rbp0[idx * 3 + 0] = Db[0];
    rbp0[idx * 3 + 1] = Db[1];
    rbp0[idx * 3 + 2] = Db[2];
    if (err) atomicOr(d_err, err);
}

// Position gradient of each dipole from the per-pair separation cotangents
// (fixed order): + for pairs it targets, - for pairs it sources.
__global__ void adj_positions_kernel(const int32_t *__restrict__ off, const int64_t *__restrict__ pair_off,
                                     const int64_t *__restrict__ pair_off0, int n_inst, const double *__restrict__ rbp,
                                     const double *__restrict__ rbp0, double *__restrict__ Rbar)
{
    const int inst = blockIdx.x;
    const int i0 = off[inst], n = off[inst + 1] - i0;
    const int M = 2 * (n - 1);
    for (int a = threadIdx.x; a < n; a += blockDim.x) {
        double s[3] = {0.0, 0.0, 0.0};
        for (int b = 0; b < n; ++b) {
            if (b == a) continue;
            for (int w = 0; w < 2; ++w) {
                // a as target of source b, and b as target of source a
                const int ja = (b < a ? b : b - 1) * 2 + w;     // slot of source b in a's list
                const int jb = (a < b ? a : a - 1) * 2 + w;     // slot of source a in b's list
                for (int th = 0; th < 2; ++th) {
                    const double *pa = rbp + (pair_off[inst] + ((int64_t)th * n + a) * M + ja) * 3;
                    const double *pb = rbp + (pair_off[inst] + ((int64_t)th * n + b) * M + jb) * 3;
                    for (int c = 0; c < 3; ++c) s[c] += pa[c] - pb[c];
                }
                const double *qa = rbp0 + (pair_off0[inst] + (int64_t)a * M + ja) * 3;
                const double *qb = rbp0 + (pair_off0[inst] + (int64_t)b * M + jb) * 3;
                for (int c = 0; c < 3; ++c) s[c] += qa[c] - qb[c];
            }
        }
        for (int c = 0; c < 3; ++c) Rbar[(int64_t)(i0 + a) * 3 + c] += s[c];
    }
}

__global__ void fill_zero_kernel(double *__restrict__ p, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0.0;
}

// --- pieces of the checkpointed sweep (segments recomputed from run states) ---

hipError_t launch_hist_rows(const DipDev *d_dev, const double *d_D, const double *d_V, const double *d_Ed, int n_dip,
                            int64_t nrows, int64_t row0, int ring, double *d_hist, hipStream_t s)
{
    const int64_t n = nrows * n_dip;
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(hist_rows_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, d_dev, d_D, d_V, d_Ed,
                       n_dip, nrows, row0, ring, d_hist);
    return hipGetLastError();
}

hipError_t launch_hist_from_state(const double *d_state, const int32_t *d_off, int n_inst, int n_dip, int ring_state,
                                  int64_t lo, int64_t hi, int ring, double *d_hist, hipStream_t s)
{
    const int64_t n = (hi - lo + 1) * n_dip;
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(hist_from_state_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, d_state, d_off,
                       n_inst, n_dip, ring_state, lo, hi, ring, d_hist);
    return hipGetLastError();
}

static AdjState adj_state(double *d_state, int n_dip)
{
    return AdjState{d_state, d_state + n_dip, d_state + 2 * (int64_t)n_dip, d_state + 3 * (int64_t)n_dip};
}

hipError_t launch_vjp_begin(int n_dip, int64_t n_pairs, int64_t steps, double *d_hbar, int64_t hbar_doubles,
                            double *d_grad, double *d_rbp, double *d_taup, double *d_state, int64_t *d_step,
                            hipStream_t s)
{
    hipLaunchKernelGGL(fill_zero_kernel, dim3(1024), dim3(256), 0, s, d_hbar, hbar_doubles);
    hipLaunchKernelGGL(fill_zero_kernel, dim3(1), dim3(256), 0, s, d_grad, (int64_t)n_dip * 3);
    hipLaunchKernelGGL(fill_zero_kernel, dim3(1024), dim3(256), 0, s, d_rbp, n_pairs * 3);
    hipLaunchKernelGGL(fill_zero_kernel, dim3(1024), dim3(256), 0, s, d_taup, n_pairs);
    hipLaunchKernelGGL(adj_init_kernel, dim3((unsigned)((n_dip + 255) / 256)), dim3(256), 0, s, n_dip, steps,
                       adj_state(d_state, n_dip), d_step);
    hipLaunchKernelGGL(adj_init_kernel, dim3((unsigned)((n_dip + 255) / 256)), dim3(256), 0, s, n_dip, steps,
                       adj_state(d_state + ADJ_FIELDS * (int64_t)n_dip, n_dip), d_step);
    return hipGetLastError();
}

hipError_t launch_vjp_detector(const DipDev *d_dev, int n_dip, const double *d_hist, double *d_hbar, int ring,
                               int64_t steps, double dt, const double *d_pts, int64_t npts, const double *d_times,
                               int n_snap, int n_norm, double *d_grad, double *d_Jpart, uint32_t *d_err,
                               hipStream_t s)
{
    const int64_t lanes = npts * n_snap;
    if (lanes <= 0) return hipSuccess;
    hipLaunchKernelGGL(detector_vjp_kernel, dim3((unsigned)((lanes + 255) / 256)), dim3(256), 0, s, d_dev, n_dip,
                       d_hist, d_hbar, ring, steps, dt, d_pts, npts, d_times, n_snap, n_norm, d_grad, d_Jpart, 60,
                       d_err);
    return hipGetLastError();
}

hipError_t launch_vjp_steps(const DipDev *d_dev, const int32_t *d_off, const int64_t *d_pair_off, int n_inst,
                            int n_dip, const double *d_hist, double *d_hbar, int ring, double dt, double *d_state,
                            double *d_rbp, double *d_taup, int64_t *d_step, int64_t count, int64_t steps,
                            uint32_t *d_err, hipStream_t s)
{
    constexpr int B = 256;
    if (count <= 0) return hipSuccess;
    const AdjState A0 = adj_state(d_state, n_dip), A1 = adj_state(d_state + ADJ_FIELDS * (int64_t)n_dip, n_dip);
    const double *soa = dip_soa(const_cast<DipDev *>(d_dev), n_dip);
    for (int64_t k = 0; k < count; ++k)
        hipLaunchKernelGGL(adj_step_kernel<B>, dim3((unsigned)n_dip), dim3(B), 0, s, d_dev, d_off, d_pair_off, n_inst,
                           n_dip, d_hist, d_hbar, ring - 1, dt, A0, A1, d_rbp, d_taup, d_step, (int)k, steps, 60,
                           soa, d_err);
    hipLaunchKernelGGL(adj_base_kernel, dim3(1), dim3(1), 0, s, d_step, -count);
    return hipGetLastError();
}

hipError_t launch_vjp_end(const DipDev *d_dev, const int32_t *d_off, const int64_t *d_pair_off,
                          const int64_t *d_pair_off0, int n_inst, int64_t n_pairs0, int n_dip, const double *d_hist,
                          double *d_hbar, int ring, double dt, double *d_state, double *d_rbp, double *d_rbp0,
                          double *d_grad, const double *d_Jpart, int64_t n_jpart, double *d_J, uint32_t *d_err,
                          hipStream_t s)
{
    constexpr int B = 256;
    const AdjState A = adj_state(d_state, n_dip);
    hipLaunchKernelGGL(adj_finish_kernel, dim3((unsigned)((n_dip + 255) / 256)), dim3(256), 0, s, d_dev, n_dip, d_hbar,
                       ring - 1, A);
    if (n_pairs0 > 0)
        hipLaunchKernelGGL(adj_drive0_kernel<B>, dim3((unsigned)((n_pairs0 + B - 1) / B)), dim3(B), 0, s, d_dev, d_off,
                           d_pair_off0, n_inst, n_pairs0, n_dip, d_hist, ring - 1, dt, A, d_rbp0, 60, d_err);
    hipLaunchKernelGGL(adj_positions_kernel, dim3((unsigned)n_inst), dim3(256), 0, s, d_off, d_pair_off, d_pair_off0,
                       n_inst, d_rbp, d_rbp0, d_grad);
    hipLaunchKernelGGL(sum_partials_kernel, dim3(1), dim3(256), 0, s, d_Jpart, n_jpart, d_J);
    return hipGetLastError();
}

}  // namespace lw
