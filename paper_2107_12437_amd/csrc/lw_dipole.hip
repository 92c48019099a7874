// lw_dipole.hip -- self-consistent Lorentz-oscillator runs on gfx950.
//
// Algorithm 1 of the paper.  Small instances run persistently over all time
// steps in one workgroup each (lo_instances_kernel); large ones take one
// launch per step with one workgroup per target dipole (lo_step_kernel).
// Each step:
//   1. every (target i, stage time, source dipole j != i, charge +/-) pair
//      solves its retarded time against j's stored history (in closed form on
//      the linear interpolation segment, Newton past the newest stored step or
//      for a moving source) and evaluates the Lienard-Wiechert field of Eq. (E)
//      at R_i projected on p_i: per charge in FP64, or in the mixed form per
//      source dipole (FP64 static monopole difference, FP32 remainder);
//   2. the pairs of one (target, stage) are summed in a fixed order by a lane
//      group and a shuffle tree (bitwise reproducible);
//   3. one lane per dipole takes the RK4 step of Eq. (LO_equation), writes
//      (d, d_dot, d_ddot) at t_{n+1} into the history ring and the outputs.
// The history ring holds the last `ring` steps of every dipole of the
// instance (in LDS when it fits); its depth covers the longest light travel
// time inside the instance, so step n+1 overwrites a slot no retarded time can
// reach any more.
#include <math.h>

#include "lw_device.hpp"
#include "lw_dipole.hpp"
#include "lw_internal.hpp"

#include <type_traits>

namespace lw {

size_t dip_dev_bytes(int n) { return dip_dev_array_bytes(n) + sizeof(double) * SF_COUNT * (size_t)n; }

__global__ void dipole_prep_kernel(const lw_dipole *__restrict__ in, int n, DipDev *__restrict__ dev,
                                   double *__restrict__ soa)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const lw_dipole &D = in[i];
    DipDev o;
    for (int k = 0; k < 3; ++k) {
        o.origin[k] = D.origin[k];
        o.axis[k] = D.axis[k];
    }
    const double M = D.m1 + D.m2;
    const double m = D.m1 * D.m2 / M;
    o.omega0 = D.omega0;
    o.q = D.q;
    o.f = D.q * D.q / m;
    o.gamma0 = D.q * D.q * D.omega0 * D.omega0 / (6.0 * PI * EPS0 * C_LIGHT * C_LIGHT * C_LIGHT * m);
    o.cfp = D.m2 / M / D.q;
    o.cfm = -D.m1 / M / D.q;
    o.vfac = fmax(D.m1, D.m2) / M / D.q;
    o.d0 = D.d0;
    const double am = sqrt(D.motion_amp[0] * D.motion_amp[0] + D.motion_amp[1] * D.motion_amp[1] +
                           D.motion_amp[2] * D.motion_amp[2]);
    const bool moves = am > 0.0;                  // the host requires motion_omega != 0 then
    for (int k = 0; k < 3; ++k) o.mamp[k] = moves ? D.motion_amp[k] : 0.0;
    o.mw = moves ? D.motion_omega : 0.0;
    o.mph = moves ? D.motion_phase : 0.0;
    o.mspeed = moves ? fabs(D.motion_omega) * am : 0.0;
    o.ehalf = 0.5 / o.f;
    dev[i] = o;
    const double f[SF_COUNT] = {o.origin[0], o.origin[1], o.origin[2], o.axis[0], o.axis[1], o.axis[2], o.cfp,
                                o.cfm,       o.d0,        o.q,         o.mamp[0], o.mamp[1], o.mamp[2], o.mw, o.mph};
    for (int k = 0; k < SF_COUNT; ++k) soa[(int64_t)k * n + i] = f[k];
}

hipError_t launch_dipole_prep(const lw_dipole *d_in, int n, DipDev *d_dev, hipStream_t s)
{
    hipLaunchKernelGGL(dipole_prep_kernel, dim3((n + 255) / 256), dim3(256), 0, s, d_in, n, d_dev,
                       dip_soa(d_dev, n));
    return hipGetLastError();
}

// region: 0 before t = 0, 1 between stored samples, 2 past the newest sample.
template <typename I>
__device__ __forceinline__ void hist_at(const Hist &H, int j, double d0, I nstep, double s, double out[3],
                                        double &slope, int &region, uint32_t &err)
{
    if (s < 0.0) {
        out[0] = d0;
        out[1] = 0.0;
        out[2] = 0.0;
        slope = 0.0;
        region = 0;
        return;
    }
    const double fk = floor(s);
    const I k = (I)fk;
    if (k >= nstep) {
        const double *h = H.ring + ((I)(nstep & H.mask) * H.n + j) * 3;
        const double tt = (s - (double)nstep) * H.dt;
        out[0] = h[0] + h[1] * tt + 0.5 * h[2] * tt * tt;
        out[1] = h[1] + h[2] * tt;
        out[2] = h[2];
        slope = out[1];
        region = 2;
        return;
    }
    if (k + H.mask < nstep) err |= 1u;          // the slot was overwritten: history too short
    const double u = s - fk;
    const double *h0 = H.ring + ((I)(k & H.mask) * H.n + j) * 3;
    const double *h1 = H.ring + ((I)((k + 1) & H.mask) * H.n + j) * 3;
    out[0] = (1.0 - u) * h0[0] + u * h1[0];
    out[1] = (1.0 - u) * h0[1] + u * h1[1];
    out[2] = (1.0 - u) * h0[2] + u * h1[2];
    slope = (h1[0] - h0[0]) * H.inv_dt;           // d/dt' of the interpolated moment
    region = 1;
}

// Retarded time of the charge at offset cf d(t') p_j of source j, seen from a
// point at separation Delta (|Delta|^2 = L2, Delta . p_j = sD) from the
// source's origin at time base * dt, by Newton (where the closed form of
// retarded_seg does not apply: past the newest stored step): the root of
// c tau = |Delta - cf d(t - tau) p_j| in [0, tau_hi], from tau.  Newton uses the exact slope of the
// interpolated moment.  Within one interpolation segment (or one side of the
// history's ends) g is smooth with |g''| <= rho'^2 / D + |rho''| (rho = cf d),
// so once Newton's error bound from the current iterate is below tol/4 the new
// iterate is accepted and the history evaluated there once more.  h holds the
// stored (d, d_dot, d_ddot) at the returned root.
template <typename I>
__device__ __forceinline__ double retarded_hist(const Hist &H, int j, double d0, I nstep, double base, double L2,
                                                double sD, double cf, double tau, double tau_hi, int max_iter,
                                                double h[3], uint32_t &err)
{
    const double tol = 4.0 * 2.220446049250313e-16;
    Bracket b(0.0, tau_hi);
    bool ok = false;
    for (int it = 0; it < max_iter; ++it) {
        const double s = base - tau * H.inv_dt;
        double slope;
        int region;
        hist_at(H, j, d0, nstep, s, h, slope, region, err);
        const double rho = cf * h[0];                            // charge offset along p_j
        double D, iD;
        root_rsqrt<true>(fmax(L2 - 2.0 * rho * sD + rho * rho, 1e-300), D, iD);
        const double r1 = cf * slope;
        const double dD = r1 * (sD - rho) * iD;
        bool free_step;
        const double tn = halley_step(tau, D, dD, 0.0, b, free_step);
        ok = converged(tn, tau, tol, b);
        if (ok) break;                                           // keep h at the last evaluated tau
        const double st = tn - tau;
        const double r2 = (region == 2) ? cf * h[2] : 0.0;
        const double sn = base - tn * H.inv_dt;
        const bool same_seg = (region == 1) ? (floor(sn) == floor(s) && sn < (double)nstep)
                                            : (region == 2 ? sn >= (double)nstep : sn < 0.0);
        tau = tn;
        if (free_step && same_seg && (r1 * r1 + fabs(r2) * D) * (st * st) <= 0.5 * tol * tn * D * (C_LIGHT - fabs(r1))) {
            double sl;
            int rg;
            hist_at(H, j, d0, nstep, sn, h, sl, rg, err);
            ok = true;
            break;
        }
    }
    if (!ok) err |= 2u;
    return tau;
}

// Retarded time past the newest stored step (the Taylor extrapolation of the
// history from sample nstep, Sec. 2.3 with the dt reading of the extrapolating
// policy): there the charge's offset is quadratic in tau,
//   rho(tau) = cf (d + v u + a u^2 / 2),  u = (base - nstep) dt - tau,
// and c tau = |Delta - rho p_j| is solved by the closed form of retarded_seg
// on the tangent line of rho, taken twice (at tau = L/c, then at the first
// root).  The linearisation error is rho'' (tau1 - tau0)^2 / 2, with
// |tau1 - tau0| ~ |rho| / c.  The result is accepted under retarded_hist's
// a-posteriori bound on the last step; returns false (the caller then uses
// Newton) when the root lies inside the stored history or the bound fails.
template <typename I>
__device__ __forceinline__ bool retarded_ext(const Hist &H, int j, I nstep, double base, double L2, double L,
                                             double sD, double cf, double h[3], double &tau_out)
{
    constexpr double C2 = C_LIGHT * C_LIGHT;
    const double *hn = H.ring + ((I)(nstep & H.mask) * H.n + j) * 3;
    const double U = (base - (double)nstep) * H.dt;
    const double al = cf * hn[0], be = cf * hn[1], ga = 0.5 * cf * hn[2];
    double tau = L * INV_C, step = 0.0, r1 = 0.0;
    for (int pass = 0; pass < 2; ++pass) {
        const double u = U - tau;
        const double rho = al + u * (be + u * ga);
        r1 = -(be + 2.0 * ga * u);                      // d rho / d tau
        const double a = rho - r1 * tau;                // tangent line a + r1 tau
        const double P = sD - a;
        const double Q = fma(a, a - 2.0 * sD, L2);
        const double bP = r1 * P;
        double S, iS;
        root_rsqrt<true>(fma(bP, bP, (C2 - r1 * r1) * Q), S, iS);
        const double tn = Q * recip<double>(bP + S);
        step = tn - tau;
        tau = tn;
    }
    const double u = U - tau;
    if (!(u >= 0.0)) return false;                      // inside the stored history
    const double D = C_LIGHT * tau, r2 = 2.0 * ga;
    const double tol = 4.0 * 2.220446049250313e-16;
    if (!((r1 * r1 + fabs(r2) * D) * (step * step) <= 0.5 * tol * tau * D * (C_LIGHT - fabs(r1)))) return false;
    h[0] = hn[0] + hn[1] * u + 0.5 * hn[2] * u * u;
    h[1] = hn[1] + hn[2] * u;
    h[2] = hn[2];
    tau_out = tau;
    return true;
}

// Retarded time of the charge at offset cf d(t') p_j of a moving source j seen
// from X at time base * dt: the root of c tau = |X - R_j(t') - cf d(t') p_j|,
// t' = t - tau, with R_j(t') = O_j + m_j cos(w t' + phi).  The same iteration
// and stopping rule as retarded_hist, with the origin's velocity and
// acceleration in the slope and the bound on g''.  Returns tau; h holds the
// stored state at the root and Ro, Vo, Ao the origin's position, velocity and
// acceleration there.
__device__ double retarded_hist_moving(const Hist &H, int j, const DipLds &Sj, const double X[3], double cf,
                                       int64_t nstep, double base, double tau, double tau_hi, int max_iter,
                                       double h[3], double Ro[3], double Vo[3], double Ao[3], uint32_t &err)
{
    const double tol = 4.0 * 2.220446049250313e-16;
    const double O[3] = {Sj.ox, Sj.oy, Sj.oz};
    const double m[3] = {Sj.mx, Sj.my, Sj.mz};
    const double p[3] = {Sj.px, Sj.py, Sj.pz};
    const double am = sqrt(m[0] * m[0] + m[1] * m[1] + m[2] * m[2]);
    Bracket b(0.0, tau_hi);
    bool ok = false;
    auto origin = [&](double s) {
        double sn, c;
        sincos_reduced(Sj.mw * (s * H.dt) + Sj.mph, sn, c);
        for (int k = 0; k < 3; ++k) {
            Ro[k] = O[k] + m[k] * c;
            Vo[k] = -Sj.mw * m[k] * sn;
            Ao[k] = -Sj.mw * Sj.mw * m[k] * c;
        }
    };
    for (int it = 0; it < max_iter; ++it) {
        const double s = base - tau * H.inv_dt;
        double slope;
        int region;
        hist_at(H, j, Sj.d0, nstep, s, h, slope, region, err);
        origin(s);
        const double rho = cf * h[0];
        double Rv[3], vel[3];
        for (int k = 0; k < 3; ++k) {
            Rv[k] = X[k] - Ro[k] - rho * p[k];
            vel[k] = Vo[k] + cf * slope * p[k];                 // d/dt' of the charge position
        }
        double D, iD;
        root_rsqrt<true>(fmax(Rv[0] * Rv[0] + Rv[1] * Rv[1] + Rv[2] * Rv[2], 1e-300), D, iD);
        const double dD = (Rv[0] * vel[0] + Rv[1] * vel[1] + Rv[2] * vel[2]) * iD;
        bool free_step;
        const double tn = halley_step(tau, D, dD, 0.0, b, free_step);
        ok = converged(tn, tau, tol, b);
        if (ok) break;
        const double st = tn - tau;
        const double sn = base - tn * H.inv_dt;
        const bool same_seg = (region == 1) ? (floor(sn) == floor(s) && sn < (double)nstep)
                                            : (region == 2 ? sn >= (double)nstep : sn < 0.0);
        const double v2 = vel[0] * vel[0] + vel[1] * vel[1] + vel[2] * vel[2];
        const double acc = Sj.mw * Sj.mw * am + ((region == 2) ? fabs(cf * h[2]) : 0.0);
        tau = tn;
        if (free_step && same_seg && (v2 + acc * D) * (st * st) <= 0.5 * tol * tn * D * (C_LIGHT - sqrt(v2))) {
            double sl;
            int rg;
            hist_at(H, j, Sj.d0, nstep, sn, h, sl, rg, err);
            origin(sn);
            ok = true;
            break;
        }
    }
    if (!ok) err |= 2u;
    return tau;
}

// Interpolated state h at the retarded time of the charge (cf) of fixed source
// j seen at separation Delta (|Delta|^2 = L2, |Delta| = L, Delta . p_j = sD):
// the closed form on the segment cached in g; past the newest stored step the
// closed form on the extrapolation; else Newton.  g.k = seg_none<I>() marks an
// empty cache.
template <typename I>
__device__ __forceinline__ void charge_fixed(const Hist &H, int j, double d0, I nstep, double base, double L2,
                                             double L, double sD, double cf, int max_iter, SegT<I> &g, double h[3],
                                             uint32_t &err)
{
    if (g.k == seg_none<I>()) {
        const double s0 = base - L * INV_C * H.inv_dt;
        const I k0 = s0 < 0.0 ? -1 : (I)floor(s0);
        if (k0 < nstep) seg_load(H, j, d0, nstep, k0, g, err);
    }
    double tau;
    if (g.k != seg_none<I>() && retarded_seg(H, j, d0, nstep, base, L2, sD, cf, g, h, tau, err)) return;
    if (retarded_ext(H, j, nstep, base, L2, L, sD, cf, h, tau)) return;
    retarded_hist(H, j, d0, nstep, base, L2, sD, cf, L * INV_C, 2.0 * L * INV_C, max_iter, h, err);
}

// Retarded separation R = X - r(t'), velocity and acceleration of the charge
// (cf) of a moving source j seen from X at time base * dt (Sec. 4.3: the
// charges ride on the source's origin at the retarded time).
__device__ __forceinline__ void charge_moving(const Hist &H, const DipLds &Sj, int j, double cf, int64_t nstep,
                                              double base, const double X[3], int max_iter, double R[3],
                                              double v[3], double a[3], uint32_t &err)
{
    // start from the present separation of the origins; the bracket's upper
    // end covers the origin's whole swing
    const double dx = X[0] - Sj.ox, dy = X[1] - Sj.oy, dz = X[2] - Sj.oz;
    const double reach = sqrt(dx * dx + dy * dy + dz * dz) + sqrt(Sj.mx * Sj.mx + Sj.my * Sj.my + Sj.mz * Sj.mz);
    double h[3], Ro[3], Vo[3], Ao[3];
    retarded_hist_moving(H, j, Sj, X, cf, nstep, base, reach * INV_C, 2.0 * reach * INV_C, max_iter, h, Ro, Vo, Ao,
                         err);
    const double rho = cf * h[0];
    const double p[3] = {Sj.px, Sj.py, Sj.pz};
    for (int c = 0; c < 3; ++c) {
        R[c] = X[c] - Ro[c] - rho * p[c];
        v[c] = Vo[c] + cf * h[1] * p[c];
        a[c] = Ao[c] + cf * h[2] * p[c];
    }
}

// p_i . E of one charge from its retarded separation, velocity and
// acceleration (FP64 field, Eq. (E)).
__device__ __forceinline__ double charge_field(const DipLds &Si, const double R[3], const double v[3],
                                               const double a[3], double kq)
{
    Kin k;
    for (int c = 0; c < 3; ++c) {
        k.R[c] = R[c];
        k.v[c] = v[c];
        k.a[c] = a[c];
    }
    k.tp = 0.0;
    k.cph = 1.0;
    k.sph = 0.0;
    k.flags = 0u;
    double o[10];
    lw_terms<double>(k, kq, F_TOTAL, o);
    return o[4] * Si.px + o[5] * Si.py + o[6] * Si.pz;
}

// p_i . E at the origin of target i of the charge (cf, kq) of source j, at
// time (nstep + theta) dt, all in FP64.  Moving origins (Sec. 4.3): the field is
// taken at the target's origin at that time.  MOVING: origins may move; without
// it every origin is taken as fixed (the kernels for fixed origins carry none
// of the moving-origin code).
// p_i . E (Eq. (E), total field, FP64) at the origin of target i of the charge
// (cf, kq) of a fixed source j, from its stored state h at the retarded time.
// The charge moves along p_j, so beta and beta_dot are multiples of p_j and
// every vector product of Eq. (E) reduces to the scalars
//   w = R . p_j = sD - rho,  p_i . R = sI - rho pij,  pij = p_i . p_j,
// with R = Delta - rho p_j, rho = cf d:
//   p_i . E = f [(p_i . n - b pij) (1 - b^2) / |R| - e q / c],  n = R / |R|,
//   b = cf d_dot / c, e = cf d_ddot / c, kappa = 1 - b (n . p_j),
//   f = kq / (kappa^3 |R|), q = pij - (p_i . n)(n . p_j),
// where the radiation term's beta parts cancel exactly (q is p_i . the part
// of p_j across n).
__device__ __forceinline__ double drive_scalar(double L2, double sD, double sI, double pij, double cf, double kq,
                                               const double h[3])
{
    const double rho = cf * h[0];
    double D, iD;
    root_rsqrt<true>(fma(rho, rho - 2.0 * sD, L2), D, iD);
    iD = fma(iD, fma(-D, iD, 1.0), iD);
    const double b = cf * h[1] * INV_C, e = cf * h[2] * INV_C;
    const double wn = (sD - rho) * iD;                  // n . p_j
    const double pin = (sI - rho * pij) * iD;           // p_i . n
    const double kappa = 1.0 - b * wn;
    const double ik = recip<double>(kappa);
    const double f = kq * iD * ik * ik * ik;
    const double q = pij - pin * wn;
    return f * ((pin - b * pij) * (1.0 - b * b) * iD - e * q * INV_C);
}

// Separation of a target at X from a fixed source j: |Delta|^2, |Delta|, and
// the projections Delta . p_j, Delta . p_i and p_i . p_j that the scalar drive
// needs (constant over a run when both origins are fixed).
struct PairGeo {
    double L2, L, sD, sI, pij;
};

__device__ __forceinline__ PairGeo pair_geo(const double X[3], const DipLds &Si, const DipLds &Sj)
{
    PairGeo P;
    const double dx = X[0] - Sj.ox, dy = X[1] - Sj.oy, dz = X[2] - Sj.oz;
    P.L2 = dx * dx + dy * dy + dz * dz;
    P.sD = dx * Sj.px + dy * Sj.py + dz * Sj.pz;     // Delta . p_j
    P.L = sqrt(P.L2);
    P.sI = dx * Si.px + dy * Si.py + dz * Si.pz;     // Delta . p_i
    P.pij = Si.px * Sj.px + Si.py * Sj.py + Si.pz * Sj.pz;
    return P;
}

// p_i . E of the charge (cf, kq) of the fixed source j at separation P, at
// time base * dt, from the stored history.
template <typename I>
__device__ __forceinline__ double fixed_drive(const Hist &H, const PairGeo &P, int j, double d0, double cf,
                                              double kq, I nstep, double base, int max_iter, uint32_t &err)
{
    SegT<I> g;
    g.k = seg_none<I>();
    double h[3];
    charge_fixed(H, j, d0, nstep, base, P.L2, P.L, P.sD, cf, max_iter, g, h, err);
    return drive_scalar(P.L2, P.sD, P.sI, P.pij, cf, kq, h);
}

template <bool MOVING>
__device__ double pair_drive(const Hist &H, const DipLds &Si, const DipLds &Sj, int j, double cf, double kq,
                             int64_t nstep, double theta, int max_iter, uint32_t &err)
{
    const double base = (double)nstep + theta;
    double X[3] = {Si.ox, Si.oy, Si.oz};
    if (MOVING) origin_at(Si, base * H.dt, X);
    if (!MOVING || Sj.mw == 0.0)
        return fixed_drive(H, pair_geo(X, Si, Sj), j, Sj.d0, cf, kq, nstep, base, max_iter, err);
    if constexpr (MOVING) {
        double R[3], v[3], a[3];
        charge_moving(H, Sj, j, cf, nstep, base, X, max_iter, R, v, a, err);
        return charge_field(Si, R, v, a, kq);
    }
    return 0.0;
}

// Velocity and radiation part of one charge's field in the mixed form: with
// n = R/|R|, beta = v/c and kappa = 1 - n.beta, the field of Eq. (E) less its
// static monopole term kq R / |R|^3, projected on p_i, per unit kq, in lengths
// scaled by 1/Ls (ix = Ls / |R|, ga = acceleration Ls / c^2).  The charge
// moves along p_j (beta = be p_j, acceleration ga p_j), so with P = p_i . n,
// X = n . p_j, pij = p_i . p_j and q = pij - P X (p_i . the part of p_j across
// n) it is
//   ix^2 be kappa^-3 [P (X (1 + kappa + kappa^2) - be) - pij (1 - be^2)]
//     - ga q ix kappa^-3,
// where the radiation term's beta parts have cancelled exactly.  Its first
// order in beta, lead = ix^2 be (3 P X - pij) - ga q ix, carries the
// near-field coupling in the phase of the velocity: for close pairs the
// reactive coupling is 1e4 times the dissipative one, so FP32 rounding there
// moves the collective rates by 1e-3 gamma_0.  lead is FP64 (dynamic_lead);
// the rest, which is smaller by a factor of order beta (dynamic_corr_f32:
// (kappa^-3 - 1) = be X (1 + kappa + kappa^2) kappa^-3 taken out exactly), is
// FP32.
__device__ __forceinline__ double dynamic_lead(double P, double X, double ix, double be, double ga, double pij,
                                               double q)
{
    return be * ix * ix * (3.0 * P * X - pij) - ga * q * ix;
}
__device__ __forceinline__ float dynamic_corr_f32(float P, float X, float ix, float be, float ga, float pij, float q)
{
    const float kap = 1.0f - be * X;
    const float s3 = 1.0f + kap + kap * kap;
    const float ik = __builtin_amdgcn_rcpf(kap);
    const float ik3 = ik * ik * ik;
    const float A = P * X * s3 - P * be - pij + pij * be * be;
    return be * be * ix * ix * (X * s3 * ik3 * A - P * X * X * (kap + 2.0f) - P + pij * be) -
           ga * q * ix * be * X * s3 * ik3;
}

// Mixed form of the drive of one source dipole at a target (both charges: +q
// at cfp d p_j, -q at cfm d p_j), at time (nstep + theta) dt.  The retarded
// times are FP64 (the closed form, the two charges sharing one history
// segment).  The field is the sum of
//  - the static monopole difference kq [f(R+) - f(R-)], f(R) = R / |R|^3, the
//    dominant term in the near field, in FP64.  R+ and R- differ by
//    D = (rho- - rho+) p_j, taken exactly from the charges' offsets although
//    far below |R| (1e-4 |R| at 10 nm for a 1e-12 m displacement, down to
//    1e-13 |R| for the small induced moments of distant dipoles), by the
//    identities
//      f(a) - f(b) = D / |a|^3 + b (|b|^3 - |a|^3) / (|a|^3 |b|^3),
//      |b|^3 - |a|^3 = (|b| - |a|) (|a|^2 + |a| |b| + |b|^2),
//      |b| - |a| = -D . (a + b) / (|a| + |b|),
//    in which nothing cancels;
//  - each charge's velocity and radiation terms, first order in beta in FP64
//    (dynamic_lead) and the remainder in FP32 (dynamic_corr_f32).  Against
//    the static term they are of relative size omega |R| / c and its square
//    in the near field, and they have the same sign for both charges (their
//    q beta and q beta_dot agree), so the FP32 remainder's rounding stays at
//    its own size times 2^-24.
// Lengths are scaled by 1/|Delta| so that FP32 stays in range at nanometre
// separations.  A moving source's origin velocity is common to both charges,
// so its velocity terms would cancel: moving sources take the FP64 field of
// each charge.  kq is that of the +q charge.
// Separation of a target at X from a fixed source j for the mixed drive: |Delta|^2,
// |Delta| and its reciprocal, Delta . p_j, and the scaled projections u . p_j,
// p_i . u (u = Delta / |Delta|), p_i . p_j and the acceleration scale L / c^2.
struct MixedGeo {
    double L2, L, iL, sD, cup, ciu, pij, gsc;
};

__device__ __forceinline__ MixedGeo mixed_geo(const double X[3], const DipLds &Si, const DipLds &Sj)
{
    MixedGeo G;
    const double p[3] = {Sj.px, Sj.py, Sj.pz};
    const double dl[3] = {X[0] - Sj.ox, X[1] - Sj.oy, X[2] - Sj.oz};
    G.L2 = dl[0] * dl[0] + dl[1] * dl[1] + dl[2] * dl[2];
    G.sD = dl[0] * p[0] + dl[1] * p[1] + dl[2] * p[2];
    root_rsqrt<true>(G.L2, G.L, G.iL);
    G.cup = G.sD * G.iL;
    G.ciu = (dl[0] * Si.px + dl[1] * Si.py + dl[2] * Si.pz) * G.iL;
    G.pij = Si.px * p[0] + Si.py * p[1] + Si.pz * p[2];
    G.gsc = INV_C * INV_C * G.L;                    // acceleration -> beta_dot L / c
    return G;
}

// The mixed drive of a fixed source from its two charges' stored states hp (+q,
// offset cfp) and hm (-q, offset cfm) at their retarded times.
__device__ __forceinline__ double mixed_field(const MixedGeo &G, double cfp, double cfm, const double hp[3],
                                              const double hm[3], double kq)
{
    const double rp = cfp * hp[0] * G.iL, rm = cfm * hm[0] * G.iL;   // scaled offsets
    // a = u - rp p_j and b = u - rm p_j enter only through u . p_j, p_i . u,
    // p_i . p_j and their own lengths
    const double cup = G.cup, ciu = G.ciu, pij = G.pij;
    // static monopole difference (FP64)
    const double dsc = rm - rp;                     // D = dsc p_j (scaled)
    double ra, ia, rb, ib;
    root_rsqrt<true>(fma(rp, rp - 2.0 * cup, 1.0), ra, ia);
    root_rsqrt<true>(fma(rm, rm - 2.0 * cup, 1.0), rb, ib);
    const double ia3 = ia * ia * ia, ib3 = ib * ib * ib;
    const double dab = -dsc * (2.0 * cup - (rp + rm)) * recip<double>(ra + rb);   // |b| - |a|
    const double c3 = dab * (ra * ra + ra * rb + rb * rb) * ia3 * ib3;
    const double st = dsc * ia3 * pij + c3 * (ciu - rm * pij);
    // velocity and radiation terms of both charges: first order in beta in
    // FP64, the rest in FP32
    const double Pa = (ciu - rp * pij) * ia, Xa = (cup - rp) * ia, Pb = (ciu - rm * pij) * ib, Xb = (cup - rm) * ib;
    const double qa = pij - Pa * Xa, qb = pij - Pb * Xb;
    const double bea = cfp * hp[1] * INV_C, gaa = cfp * hp[2] * G.gsc;
    const double beb = cfm * hm[1] * INV_C, gab = cfm * hm[2] * G.gsc;
    const float fpij = (float)pij;
    const float corr = dynamic_corr_f32((float)Pa, (float)Xa, (float)ia, (float)bea, (float)gaa, fpij, (float)qa) -
                       dynamic_corr_f32((float)Pb, (float)Xb, (float)ib, (float)beb, (float)gab, fpij, (float)qb);
    const double rest = dynamic_lead(Pa, Xa, ia, bea, gaa, pij, qa) - dynamic_lead(Pb, Xb, ib, beb, gab, pij, qb) +
                        (double)corr;
    return kq * G.iL * G.iL * (st + rest);
}

template <bool MOVING>
__device__ double dipole_drive_mixed(const Hist &H, const DipLds &Si, const DipLds &Sj, int j, double kq,
                                     int64_t nstep, double theta, int max_iter, uint32_t &err)
{
    const double base = (double)nstep + theta;
    double X[3] = {Si.ox, Si.oy, Si.oz};
    if (MOVING) origin_at(Si, base * H.dt, X);
    if constexpr (MOVING) {
        if (Sj.mw != 0.0) {
            double R[3], v[3], a[3];
            charge_moving(H, Sj, j, Sj.cfp, nstep, base, X, max_iter, R, v, a, err);
            double e = charge_field(Si, R, v, a, kq);
            charge_moving(H, Sj, j, Sj.cfm, nstep, base, X, max_iter, R, v, a, err);
            return e + charge_field(Si, R, v, a, -kq);
        }
    }
    const MixedGeo G = mixed_geo(X, Si, Sj);
    Seg g;
    g.k = seg_none<int64_t>();
    double hp[3], hm[3];
    charge_fixed(H, j, Sj.d0, nstep, base, G.L2, G.L, G.sD, Sj.cfp, max_iter, g, hp, err);
    charge_fixed(H, j, Sj.d0, nstep, base, G.L2, G.L, G.sD, Sj.cfm, max_iter, g, hm, err);
    return mixed_field(G, Sj.cfp, Sj.cfm, hp, hm, kq);
}

// p_i . E of both charges of source j in FP64 (Eq. (E), total field), one after
// the other in one lane: they share the separation of the origins, its
// projections and the cached history segment (the two charges' retarded times
// lie about 1e-4 of a step apart), so the lane loads the segment once.  The
// per-charge terms are those of pair_drive.
template <bool MOVING>
__device__ double dipole_drive_fp64(const Hist &H, const DipLds &Si, const DipLds &Sj, int j, double kq,
                                    int64_t nstep, double theta, int max_iter, uint32_t &err)
{
    const double base = (double)nstep + theta;
    double X[3] = {Si.ox, Si.oy, Si.oz};
    if (MOVING) origin_at(Si, base * H.dt, X);
    if constexpr (MOVING) {
        if (Sj.mw != 0.0) {
            double R[3], v[3], a[3];
            charge_moving(H, Sj, j, Sj.cfp, nstep, base, X, max_iter, R, v, a, err);
            const double e = charge_field(Si, R, v, a, kq);
            charge_moving(H, Sj, j, Sj.cfm, nstep, base, X, max_iter, R, v, a, err);
            return e + charge_field(Si, R, v, a, -kq);
        }
    }
    const double dx = X[0] - Sj.ox, dy = X[1] - Sj.oy, dz = X[2] - Sj.oz;
    const double L2 = dx * dx + dy * dy + dz * dz;
    const double sD = dx * Sj.px + dy * Sj.py + dz * Sj.pz;     // Delta . p_j
    const double sI = dx * Si.px + dy * Si.py + dz * Si.pz;     // Delta . p_i
    const double pij = Si.px * Sj.px + Si.py * Sj.py + Si.pz * Sj.pz;
    const double L = sqrt(L2);
    Seg g;
    g.k = seg_none<int64_t>();
    double hp[3], hm[3];
    charge_fixed(H, j, Sj.d0, nstep, base, L2, L, sD, Sj.cfp, max_iter, g, hp, err);
    charge_fixed(H, j, Sj.d0, nstep, base, L2, L, sD, Sj.cfm, max_iter, g, hm, err);
    return drive_scalar(L2, sD, sI, pij, Sj.cfp, kq, hp) + drive_scalar(L2, sD, sI, pij, Sj.cfm, -kq, hm);
}

// The segments charge_fixed starts from at both stage times of a step (those
// of tau = L/c at base_h = n + 1/2 and base_f = n + 1), with the values
// seg_load gives each, loaded without a branch.  The two start points differ
// by half a step (rounding is monotonic, so by less than one), so the second
// segment is the first or the next one, and three ring rows hold both.  Rows
// are taken modulo the ring, so every load stays in bounds, also where a
// segment lies past the newest stored step (a row this launch may be writing):
// that segment is marked empty and its values are not used (charge_fixed goes
// on to the extrapolation, as it would have).
template <typename I>
__device__ __forceinline__ void seg_stages(const Hist &H, int j, double d0, I nstep, double base_h, double base_f,
                                           double L, SegT<I> &gh, SegT<I> &gf, uint32_t &err)
{
    const double sh = base_h - L * INV_C * H.inv_dt, sf = base_f - L * INV_C * H.inv_dt;
    const I kh = sh < 0.0 ? -1 : (I)floor(sh);
    const I kf = sf < 0.0 ? -1 : (I)floor(sf);
    const I k = kh < 0 ? -1 : kh;
    const double *p0 = H.ring + ((I)(k & H.mask) * H.n + j) * 3;
    const double *p1 = H.ring + ((I)((k + 1) & H.mask) * H.n + j) * 3;
    const double *p2 = H.ring + ((I)((k + 2) & H.mask) * H.n + j) * 3;
    const double r0[3] = {p0[0], p0[1], p0[2]}, r1[3] = {p1[0], p1[1], p1[2]}, r2[3] = {p2[0], p2[1], p2[2]};
    const bool preh = kh < 0, pref = kf < 0, next = kf != kh;
    gh.k = preh ? -1 : kh;
    gh.d0 = preh ? d0 : r0[0];
    gh.v0 = preh ? 0.0 : r0[1];
    gh.a0 = preh ? 0.0 : r0[2];
    gh.d1 = preh ? d0 : r1[0];
    gh.v1 = preh ? 0.0 : r1[1];
    gh.a1 = preh ? 0.0 : r1[2];
    gf.k = pref ? -1 : kf;
    gf.d0 = pref ? d0 : (next ? r1[0] : r0[0]);
    gf.v0 = pref ? 0.0 : (next ? r1[1] : r0[1]);
    gf.a0 = pref ? 0.0 : (next ? r1[2] : r0[2]);
    gf.d1 = pref ? d0 : (next ? r2[0] : r1[0]);
    gf.v1 = pref ? 0.0 : (next ? r2[1] : r1[1]);
    gf.a1 = pref ? 0.0 : (next ? r2[2] : r1[2]);
    if ((!preh && kh + H.mask < nstep) || (!pref && kf + H.mask < nstep)) err |= ERR_HISTORY;
    if (kh >= nstep) gh.k = seg_none<I>();
    if (kf >= nstep) gf.k = seg_none<I>();
}

// Both stage times of a step (t_n + dt/2 and t_n + dt) for both charges of a
// fixed source, with the operations of two dipole_drive_fp64 calls (so the
// same results).  The history rows of both stages' first segments are loaded
// together at the start, so the second stage does not wait on memory after the
// first stage's solves: 176 against 184 us per step on 64 clusters of 12,530
// dipoles, although the lane then holds 147 VGPRs (3 waves per SIMD, against 4
// at 115).  Loading each stage's two rows separately (144 VGPRs) was slower,
// 196 us, and so was solving all four charges before their fields, 179 us.
__device__ __forceinline__ void dipole_drive_fp64_stages(const Hist &H, const DipLds &Si, const DipLds &Sj, int j,
                                                         double kq, int64_t nstep, int max_iter, uint32_t &err,
                                                         double &e_half, double &e_full)
{
    const double dx = Si.ox - Sj.ox, dy = Si.oy - Sj.oy, dz = Si.oz - Sj.oz;
    const double L2 = dx * dx + dy * dy + dz * dz;
    const double sD = dx * Sj.px + dy * Sj.py + dz * Sj.pz;     // Delta . p_j
    const double sI = dx * Si.px + dy * Si.py + dz * Si.pz;     // Delta . p_i
    const double pij = Si.px * Sj.px + Si.py * Sj.py + Si.pz * Sj.pz;
    const double L = sqrt(L2);
    const double base_h = (double)nstep + 0.5, base_f = (double)nstep + 1.0;
    Seg gh, gf;
    seg_stages(H, j, Sj.d0, nstep, base_h, base_f, L, gh, gf, err);
    double hp[3], hm[3];
    charge_fixed(H, j, Sj.d0, nstep, base_h, L2, L, sD, Sj.cfp, max_iter, gh, hp, err);
    charge_fixed(H, j, Sj.d0, nstep, base_h, L2, L, sD, Sj.cfm, max_iter, gh, hm, err);
    e_half = drive_scalar(L2, sD, sI, pij, Sj.cfp, kq, hp) + drive_scalar(L2, sD, sI, pij, Sj.cfm, -kq, hm);
    charge_fixed(H, j, Sj.d0, nstep, base_f, L2, L, sD, Sj.cfp, max_iter, gf, hp, err);
    charge_fixed(H, j, Sj.d0, nstep, base_f, L2, L, sD, Sj.cfm, max_iter, gf, hm, err);
    e_full = drive_scalar(L2, sD, sI, pij, Sj.cfp, kq, hp) + drive_scalar(L2, sD, sI, pij, Sj.cfm, -kq, hm);
}

// The mixed drive of a fixed source at both stage times of a step, with the
// operations of two dipole_drive_mixed calls and the segment loads of
// dipole_drive_fp64_stages: 189 against 207 us per step on 64 clusters of
// 12,530 dipoles, against a lane per (stage, source).
__device__ __forceinline__ void dipole_drive_mixed_stages(const Hist &H, const DipLds &Si, const DipLds &Sj, int j,
                                                          double kq, int64_t nstep, int max_iter, uint32_t &err,
                                                          double &e_half, double &e_full)
{
    const double X[3] = {Si.ox, Si.oy, Si.oz};
    const MixedGeo G = mixed_geo(X, Si, Sj);
    const double base_h = (double)nstep + 0.5, base_f = (double)nstep + 1.0;
    Seg gh, gf;
    seg_stages(H, j, Sj.d0, nstep, base_h, base_f, G.L, gh, gf, err);
    double hp[3], hm[3];
    charge_fixed(H, j, Sj.d0, nstep, base_h, G.L2, G.L, G.sD, Sj.cfp, max_iter, gh, hp, err);
    charge_fixed(H, j, Sj.d0, nstep, base_h, G.L2, G.L, G.sD, Sj.cfm, max_iter, gh, hm, err);
    e_half = mixed_field(G, Sj.cfp, Sj.cfm, hp, hm, kq);
    charge_fixed(H, j, Sj.d0, nstep, base_f, G.L2, G.L, G.sD, Sj.cfp, max_iter, gf, hp, err);
    charge_fixed(H, j, Sj.d0, nstep, base_f, G.L2, G.L, G.sD, Sj.cfm, max_iter, gf, hm, err);
    e_full = mixed_field(G, Sj.cfp, Sj.cfm, hp, hm, kq);
}

// Drive contribution of work unit w of source j: in FP64 one unit per charge
// (w = 0: +q, 1: -q), in the mixed form one unit per source dipole.
template <bool MOVING, bool MIXED>
__device__ __forceinline__ double unit_drive(const Hist &H, const DipLds &Si, const DipLds &Sj, int j, double qj,
                                             int w, int64_t nstep, double theta, int max_iter, uint32_t &err)
{
    if constexpr (MIXED) {
        return dipole_drive_mixed<MOVING>(H, Si, Sj, j, qj * K_COUL, nstep, theta, max_iter, err);
    } else {
        const double cf = w ? Sj.cfm : Sj.cfp;
        const double kq = (w ? -qj : qj) * K_COUL;
        return pair_drive<MOVING>(H, Si, Sj, j, cf, kq, nstep, theta, max_iter, err);
    }
}

template <bool MIXED> constexpr int units_per_source() { return MIXED ? 1 : 2; }

// The stepped kernel's work unit: one source dipole per lane in both forms (its
// targets have many sources, so fewer, fuller units pay; the persistent kernel
// keeps a lane per charge, which shortens the serial chain of small instances).
template <bool MOVING, bool MIXED>
__device__ __forceinline__ double source_drive(const Hist &H, const DipLds &Si, const DipLds &Sj, int j, double qj,
                                               int64_t nstep, double theta, int max_iter, uint32_t &err)
{
    if constexpr (MIXED) return dipole_drive_mixed<MOVING>(H, Si, Sj, j, qj * K_COUL, nstep, theta, max_iter, err);
    else return dipole_drive_fp64<MOVING>(H, Si, Sj, j, qj * K_COUL, nstep, theta, max_iter, err);
}

// Drive fields of all targets of the instance at stage times theta in
// `thetas[0..nth)` (in steps after nstep), written to Eout[th * n + i].
template <int BLOCK, bool MOVING, bool MIXED>
__device__ void drive_all(const Hist &H, const DipLds *S, const double *qv, int n, int64_t nstep,
                          const double *thetas, int nth, double *Eout, int max_iter, uint32_t &err)
{
    constexpr int U = units_per_source<MIXED>();
    const int M = U * (n - 1);                    // work units per (target, stage)
    const int G = nth * n;                        // (target, stage) groups
    // lanes per group Lg = 2^lg; the index arithmetic uses shifts (integer
    // division has no hardware instruction), and a group's stage is 0 or 1
    int lg = 0;
    while ((1 << lg) < M && lg < 6) ++lg;
    while (lg > 0 && (G << lg) > BLOCK) --lg;
    const int Lg = 1 << lg;
    const int per_pass = BLOCK >> lg;
    const int tid = threadIdx.x;
    const int sub = tid & (Lg - 1);
    for (int g0 = 0; g0 < G; g0 += per_pass) {
        const int g = g0 + (tid >> lg);
        double acc = 0.0;
        if (g < G && M > 0) {
            const int th = g >= n ? 1 : 0, i = g - th * n;
            for (int m = sub; m < M; m += Lg) {
                const int jj = m / U, w = m % U;
                const int j = jj < i ? jj : jj + 1;
                acc += unit_drive<MOVING, MIXED>(H, S[i], S[j], j, qv[j], w, nstep, thetas[th], max_iter, err);
            }
        }
        for (int off = 1; off < Lg; off <<= 1) acc += __shfl_xor(acc, off, 64);
        if (g < G && sub == 0) Eout[g] = acc;
    }
}

template <int BLOCK, bool RING_LDS, bool MOVING, bool MIXED>
__global__ __launch_bounds__(BLOCK) void lo_instances_kernel(const DipDev *__restrict__ dev,
                                                             const int32_t *__restrict__ off,
                                                             const int32_t *__restrict__ inst_list, int ring,
                                                             int64_t steps, double dt,
                                                             double max_vel, int max_iter,
                                                             double *__restrict__ ring_global,
                                                             const int64_t *__restrict__ ring_off, RunOut out,
                                                             double *__restrict__ state, int resume,
                                                             uint32_t *__restrict__ d_err)
{
    extern __shared__ double lds[];
    const int inst = inst_list[blockIdx.x];
    const int i0 = off[inst];
    const int n = off[inst + 1] - i0;
    const int tid = threadIdx.x;
    if (n <= 0) return;

    // LDS layout: constants, q, Ecur, Emid/Eend, absorbed and radiated energy,
    // oscillator constants (w0^2, gamma0, f, vfac, origin speed, 0.5 / f), (ring)
    DipLds *S = (DipLds *)lds;
    double *qv = (double *)(S + n);
    double *Ecur = qv + n;
    double *Enew = Ecur + n;                    // [2][n]: mid, end
    double *Wab = Enew + 2 * n;
    double *Wra = Wab + n;
    double *Kc = Wra + n;                       // [6][n]
    double *ring_lds = Kc + 6 * n;
    double *ringp = RING_LDS ? ring_lds : ring_global + ring_off[blockIdx.x];
    __shared__ uint32_t s_err;

    for (int j = tid; j < n; j += BLOCK) {
        const DipDev &D = dev[i0 + j];
        S[j] = dip_lds(D);
        qv[j] = D.q;
        Kc[j] = D.omega0 * D.omega0;
        Kc[n + j] = D.gamma0;
        Kc[2 * n + j] = D.f;
        Kc[3 * n + j] = D.vfac;
        Kc[4 * n + j] = D.mspeed;
        Kc[5 * n + j] = D.ehalf;
    }
    if (tid == 0) s_err = 0u;
    __syncthreads();

    Hist H{ringp, n, ring - 1, dt, 1.0 / dt};
    uint32_t err = 0u;
    const int64_t ring3 = (int64_t)ring * n * 3;
    int64_t n0 = 0;                             // the run's first step

    if (resume) {
        // continue from the run state: history, E_d(t_n0) and the energy sums
        // (output row 0 is written from the state before this kernel runs)
        n0 = (int64_t)state[0];
        const double *sr = state + state_ring_off(i0, ring);
        for (int64_t k = tid; k < ring3; k += BLOCK) ringp[k] = sr[k];
        const int64_t oe = state_ecur_off(out.n_dip, ring), ow = state_w_off(out.n_dip, ring);
        for (int i = tid; i < n; i += BLOCK) {
            Ecur[i] = state[oe + i0 + i];
            Wab[i] = state[ow + 2 * (i0 + i)];
            Wra[i] = state[ow + 2 * (i0 + i) + 1];
        }
    } else {
        // t = 0: drive from the static pre-history, then sample 0 = (d0, 0, d_ddot(0))
        {
            const double th0[1] = {0.0};
            drive_all<BLOCK, MOVING, MIXED>(H, S, qv, n, 0, th0, 1, Ecur, max_iter, err);
        }
        __syncthreads();
        for (int i = tid; i < n; i += BLOCK) {
            const DipDev &D = dev[i0 + i];
            double *h = ringp + (int64_t)i * 3;
            h[0] = D.d0;
            h[1] = 0.0;
            h[2] = D.f * Ecur[i] - D.omega0 * D.omega0 * D.d0;
            const int gi = i0 + i;
            Wab[i] = 0.0;
            Wra[i] = 0.0;
            put_row(out, 0, gi, D.d0, 0.0, run_energy(D.omega0 * D.omega0, D.ehalf, D.d0, 0.0), Ecur[i], 0.0, 0.0);
        }
    }
    __syncthreads();

    const double thetas[2] = {0.5, 1.0};
    for (int64_t nstep = n0; nstep < n0 + steps; ++nstep) {
        drive_all<BLOCK, MOVING, MIXED>(H, S, qv, n, nstep, thetas, 2, Enew, max_iter, err);
        __syncthreads();
        for (int i = tid; i < n; i += BLOCK) {
            const double w2 = Kc[i], g = Kc[n + i], f = Kc[2 * n + i], vfac = Kc[3 * n + i], ms = Kc[4 * n + i];
            const double *h = ringp + ((int64_t)(nstep & (ring - 1)) * n + i) * 3;
            const double Em = Enew[i], Ee = Enew[n + i], Ec = Ecur[i];
            const double y0 = h[0], y1 = h[1];
            // classic RK4 on y = (d, d_dot), y' = (d_dot, f E_d(t) - gamma0 d_dot - w0^2 d)
            const double k1d = y1, k1v = f * Ec - g * y1 - w2 * y0;
            const double y0b = y0 + 0.5 * dt * k1d, y1b = y1 + 0.5 * dt * k1v;
            const double k2d = y1b, k2v = f * Em - g * y1b - w2 * y0b;
            const double y0c = y0 + 0.5 * dt * k2d, y1c = y1 + 0.5 * dt * k2v;
            const double k3d = y1c, k3v = f * Em - g * y1c - w2 * y0c;
            const double y0d = y0 + dt * k3d, y1d = y1 + dt * k3v;
            const double k4d = y1d, k4v = f * Ee - g * y1d - w2 * y0d;
            const double dn = y0 + dt / 6.0 * (k1d + 2.0 * k2d + 2.0 * k3d + k4d);
            const double vn = y1 + dt / 6.0 * (k1v + 2.0 * k2v + 2.0 * k3v + k4v);
            const double an = f * Ee - g * vn - w2 * dn;
            double *hn = ringp + ((int64_t)((nstep + 1) & (ring - 1)) * n + i) * 3;
            hn[0] = dn;
            hn[1] = vn;
            hn[2] = an;
            Ecur[i] = Ee;
            if (!(isfinite(dn) && isfinite(vn) && isfinite(an))) err |= ERR_NONFINITE;
            if (max_vel > 0.0 && ms + vfac * fabs(vn) > max_vel) err |= ERR_VELOCITY;
            // energy bookkeeping (Sec. 2.5), trapezoid rule over the step
            const double wa = Wab[i] + 0.5 * dt * (y1 * Ec + vn * Ee);
            const double wr = Wra[i] + 0.5 * dt * K_LARMOR * (h[2] * h[2] + an * an);
            Wab[i] = wa;
            Wra[i] = wr;
            const int64_t rel = nstep + 1 - n0;
            const int64_t row = out_row(rel, out.stride);
            if (row >= 0) put_row(out, row, i0 + i, dn, vn, run_energy(w2, Kc[5 * n + i], dn, vn), Ee, wa, wr);
        }
        if (err) atomicOr(&s_err, err);
        __syncthreads();
        if (s_err & (ERR_NONFINITE | ERR_VELOCITY | ERR_HISTORY)) break;
    }
    __syncthreads();
    if (state) {
        // save the run state: history, E_d and the energy sums
        double *sr = state + state_ring_off(i0, ring);
        for (int64_t k = tid; k < ring3; k += BLOCK) sr[k] = ringp[k];
        const int64_t oe = state_ecur_off(out.n_dip, ring), ow = state_w_off(out.n_dip, ring);
        for (int i = tid; i < n; i += BLOCK) {
            state[oe + i0 + i] = Ecur[i];
            state[ow + 2 * (i0 + i)] = Wab[i];
            state[ow + 2 * (i0 + i) + 1] = Wra[i];
        }
    }
    if (tid == 0 && s_err) atomicOr(d_err, s_err);
}

// ---------------------------------------------------------------------------
// Instances of at most SMALL_MAX_N fixed dipoles, one wave each.  A step of such
// an instance is a serial chain (drive, then RK4, then the next drive reads the
// new sample), so its time is the instructions its one wave issues.  Here
// every lane holds one work unit for the whole run (target i, stage theta,
// source j, charge w: 2 n (n - 1) units in groups of Lg lanes, drive_all's FP64
// layout), with the unit's separation and projections computed once, and lanes
// 0..n-1 keep their dipole's state, constants and energy sums in registers.
// The stage sums reach the RK4 lanes by cross-lane reads.
//   FP64: the arithmetic of every drive, sum and RK4 step is that of
//         lo_instances_kernel, in the same order, so both give the same bits.
//   MIXED: the two lanes of a source's charges each solve their charge's
//         retarded time, swap the stored states (d, d_dot, d_ddot) there, and
//         the +q lane evaluates the source's mixed drive (mixed_field).  The
//         general kernel solves both charges in one lane on one cached history
//         segment; here each lane loads its own, which finds the same root (to
//         its last bit but for roots within rounding of a segment end).
// ---------------------------------------------------------------------------
constexpr int SMALL_MAX_N = 4;     // 2 n * Lg <= 64 lanes for n <= 4

template <bool MIXED>
__global__ __launch_bounds__(64) void lo_small_kernel(const DipDev *__restrict__ dev, const int32_t *__restrict__ off,
                                                      const int32_t *__restrict__ inst_list, int ring, int64_t steps,
                                                      double dt, double max_vel, int max_iter, RunOut out,
                                                      double *__restrict__ state, int resume,
                                                      uint32_t *__restrict__ d_err)
{
    constexpr int BLOCK = 64;
    extern __shared__ double lds[];
    const int inst = inst_list[blockIdx.x];
    const int i0 = off[inst];
    const int n = off[inst + 1] - i0;
    const int tid = threadIdx.x;
    if (n <= 0) return;
    if (n > SMALL_MAX_N) {                      // the host launches none; never silently skip one
        if (tid == 0) atomicOr(d_err, (uint32_t)ERR_STATE);
        return;
    }

    // LDS layout as lo_instances_kernel's (the t = 0 drive and the run state
    // use it); the step loop reads only the ring
    DipLds *S = (DipLds *)lds;
    double *qv = (double *)(S + n);
    double *Ecur = qv + n;
    double *Wab = Ecur + 3 * n;
    double *Wra = Wab + n;
    double *ringp = Wra + 7 * n;
    __shared__ uint32_t s_err;

    for (int j = tid; j < n; j += BLOCK) {
        const DipDev &D = dev[i0 + j];
        S[j] = dip_lds(D);
        qv[j] = D.q;
    }
    if (tid == 0) s_err = 0u;
    __syncthreads();

    Hist H{ringp, n, ring - 1, dt, 1.0 / dt};
    uint32_t err = 0u;
    int64_t n0 = 0;
    if (resume) {
        n0 = (int64_t)state[0];
        const double *sr = state + state_ring_off(i0, ring);
        const int64_t ring3 = (int64_t)ring * n * 3;
        for (int64_t k = tid; k < ring3; k += BLOCK) ringp[k] = sr[k];
        const int64_t oe = state_ecur_off(out.n_dip, ring), ow = state_w_off(out.n_dip, ring);
        for (int i = tid; i < n; i += BLOCK) {
            Ecur[i] = state[oe + i0 + i];
            Wab[i] = state[ow + 2 * (i0 + i)];
            Wra[i] = state[ow + 2 * (i0 + i) + 1];
        }
    } else {
        {
            const double th0[1] = {0.0};
            drive_all<BLOCK, false, MIXED>(H, S, qv, n, 0, th0, 1, Ecur, max_iter, err);
        }
        __syncthreads();
        for (int i = tid; i < n; i += BLOCK) {
            const DipDev &D = dev[i0 + i];
            double *h = ringp + (int64_t)i * 3;
            h[0] = D.d0;
            h[1] = 0.0;
            h[2] = D.f * Ecur[i] - D.omega0 * D.omega0 * D.d0;
            Wab[i] = 0.0;
            Wra[i] = 0.0;
            put_row(out, 0, i0 + i, D.d0, 0.0, run_energy(D.omega0 * D.omega0, D.ehalf, D.d0, 0.0), Ecur[i], 0.0,
                    0.0);
        }
    }
    __syncthreads();

    // this lane's work unit, as drive_all lays them out for two stage times
    const int M = 2 * (n - 1), G = 2 * n;
    int lg = 0;
    while ((1 << lg) < M) ++lg;
    const int Lg = 1 << lg;
    const int grp = tid >> lg, sub = tid & (Lg - 1);
    const bool active = grp < G && sub < M;
    int uj = 0;
    double ucf = 0.0, ukq = 0.0, ud0 = 0.0, utheta = 0.0, ucfp = 0.0, ucfm = 0.0;
    PairGeo P{0.0, 0.0, 0.0, 0.0, 0.0};
    MixedGeo MG{0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    const bool plus = (sub & 1) == 0;           // the +q lane of its source's pair
    if (active) {
        const int th = grp >= n ? 1 : 0, i = grp - th * n;
        const int jj = sub >> 1, w = sub & 1;
        uj = jj < i ? jj : jj + 1;
        const DipLds Si = S[i], Sj = S[uj];
        ucf = w ? Sj.cfm : Sj.cfp;
        ud0 = Sj.d0;
        utheta = th ? 1.0 : 0.5;
        const double X[3] = {Si.ox, Si.oy, Si.oz};
        if constexpr (MIXED) {
            ukq = qv[uj] * K_COUL;                  // the +q charge's (mixed_field)
            ucfp = Sj.cfp;
            ucfm = Sj.cfm;
            MG = mixed_geo(X, Si, Sj);
            P.L2 = MG.L2;
            P.L = MG.L;
            P.sD = MG.sD;
        } else {
            ukq = (w ? -qv[uj] : qv[uj]) * K_COUL;
            P = pair_geo(X, Si, Sj);
        }
    }
    // lanes 0..n-1: dipole tid's state at the run's first step, constants and sums
    const bool owner = tid < n;
    const int me = owner ? tid : 0;
    double y0 = 0.0, y1 = 0.0, y2 = 0.0, Ec = 0.0, wab = 0.0, wra = 0.0;
    double w2 = 0.0, gm = 0.0, fq = 0.0, vfac = 0.0, ms = 0.0, eh = 0.0;
    if (owner) {
        const DipDev &D = dev[i0 + me];
        w2 = D.omega0 * D.omega0;
        gm = D.gamma0;
        fq = D.f;
        vfac = D.vfac;
        ms = D.mspeed;
        eh = D.ehalf;
        const double *h = ringp + ((int64_t)(n0 & (ring - 1)) * n + me) * 3;
        y0 = h[0];
        y1 = h[1];
        y2 = h[2];
        Ec = Ecur[me];
        wab = Wab[me];
        wra = Wra[me];
    }
    const int src_mid = me << lg, src_end = (n + me) << lg;
    const double hdt = 0.5 * dt, dt6 = dt / 6.0, hdtl = 0.5 * dt * K_LARMOR;
    const uint32_t stop_bits = ERR_NONFINITE | ERR_VELOCITY | ERR_HISTORY;

    // the steps, with 32-bit step indices when the run's last step fits
    auto run_steps = [&](auto index_type) {
      using I = decltype(index_type);
      for (I nstep = (I)n0; nstep < (I)(n0 + steps); ++nstep) {
        double acc = 0.0;
        if constexpr (MIXED) {
            double h[3] = {0.0, 0.0, 0.0};
            if (active) {
                SegT<I> g;
                g.k = seg_none<I>();
                charge_fixed(H, uj, ud0, nstep, (double)nstep + utheta, P.L2, P.L, P.sD, ucf, max_iter, g, h, err);
            }
            double ho[3];
            for (int q = 0; q < 3; ++q) ho[q] = __shfl_xor(h[q], 1, 64);
            if (active && plus) acc += mixed_field(MG, ucfp, ucfm, h, ho, ukq);
        } else {
            if (active) acc += fixed_drive(H, P, uj, ud0, ucf, ukq, nstep, (double)nstep + utheta, max_iter, err);
        }
        for (int o = 1; o < Lg; o <<= 1) acc += __shfl_xor(acc, o, 64);
        const double Em = __shfl(acc, src_mid, 64), Ee = __shfl(acc, src_end, 64);
        if (owner) {
            // classic RK4 on y = (d, d_dot), as lo_instances_kernel
            const double k1d = y1, k1v = fq * Ec - gm * y1 - w2 * y0;
            const double y0b = y0 + hdt * k1d, y1b = y1 + hdt * k1v;
            const double k2d = y1b, k2v = fq * Em - gm * y1b - w2 * y0b;
            const double y0c = y0 + hdt * k2d, y1c = y1 + hdt * k2v;
            const double k3d = y1c, k3v = fq * Em - gm * y1c - w2 * y0c;
            const double y0d = y0 + dt * k3d, y1d = y1 + dt * k3v;
            const double k4d = y1d, k4v = fq * Ee - gm * y1d - w2 * y0d;
            const double dn = y0 + dt6 * (k1d + 2.0 * k2d + 2.0 * k3d + k4d);
            const double vn = y1 + dt6 * (k1v + 2.0 * k2v + 2.0 * k3v + k4v);
            const double an = fq * Ee - gm * vn - w2 * dn;
            double *hn = ringp + ((I)((nstep + 1) & (ring - 1)) * n + me) * 3;
            hn[0] = dn;
            hn[1] = vn;
            hn[2] = an;
            if (!(isfinite(dn) && isfinite(vn) && isfinite(an))) err |= ERR_NONFINITE;
            if (max_vel > 0.0 && ms + vfac * fabs(vn) > max_vel) err |= ERR_VELOCITY;
            wab = wab + hdt * (y1 * Ec + vn * Ee);
            wra = wra + hdtl * (y2 * y2 + an * an);
            const int64_t row = out_row((int64_t)nstep + 1 - n0, out.stride);
            if (row >= 0) put_row(out, row, i0 + me, dn, vn, run_energy(w2, eh, dn, vn), Ee, wab, wra);
            y0 = dn;
            y1 = vn;
            y2 = an;
            Ec = Ee;
        }
        // the new samples are read by other lanes of this wave in the next step
        __syncthreads();
        if (__any((err & stop_bits) != 0u)) break;
      }
    };
    if (n0 + steps < (int64_t)INT32_MAX) run_steps(int{});
    else run_steps(int64_t{});
    if (owner) {
        Ecur[me] = Ec;
        Wab[me] = wab;
        Wra[me] = wra;
    }
    if (err) atomicOr(&s_err, err);
    __syncthreads();
    if (state) {
        double *sr = state + state_ring_off(i0, ring);
        const int64_t ring3 = (int64_t)ring * n * 3;
        for (int64_t k = tid; k < ring3; k += BLOCK) sr[k] = ringp[k];
        const int64_t oe = state_ecur_off(out.n_dip, ring), ow = state_w_off(out.n_dip, ring);
        for (int i = tid; i < n; i += BLOCK) {
            state[oe + i0 + i] = Ecur[i];
            state[ow + 2 * (i0 + i)] = Wab[i];
            state[ow + 2 * (i0 + i) + 1] = Wra[i];
        }
    }
    if (tid == 0 && s_err) atomicOr(d_err, s_err);
}

// ---------------------------------------------------------------------------
// Large instances: one workgroup per target dipole, one launch per step.
// The step index comes from a device counter (advanced by step_advance_kernel)
// so that a captured sequence of steps can be replayed.  Block b advances dipole
// tgt[b]; its sources are the other dipoles of the same instance, whose history
// ring sits at ring + ring_base[b] ([ring][n][3]).  Writing step n+1 of dipole
// i touches the slot of step n+1-ring, which no retarded time of this step can
// reach, so all blocks of a launch may run in any order.
// ---------------------------------------------------------------------------


template <int BLOCK, bool MOVING, bool MIXED>
__global__ __launch_bounds__(BLOCK) void lo_step_kernel(const DipDev *__restrict__ dev, const int32_t *__restrict__ tgt,
                                                        const int32_t *__restrict__ tgt_lo,
                                                        const int32_t *__restrict__ tgt_n,
                                                        const int64_t *__restrict__ ring_base, double *__restrict__ ring,
                                                        double *__restrict__ Ecur, double *__restrict__ W,
                                                        const int64_t *__restrict__ step_ctr, int kstep,
                                                        int ring_depth, double dt, double max_vel, int max_iter,
                                                        int init, int wide, RunOut out,
                                                        const double *__restrict__ soa, uint32_t *__restrict__ d_err)
{
    __shared__ double red[2][BLOCK / 64];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int gi = tgt[blockIdx.x];
    const int i0 = tgt_lo[blockIdx.x];
    const int n = tgt_n[blockIdx.x];
    const int i = gi - i0;
    const int64_t nstep = init ? 0 : *step_ctr + kstep;
    double *rp = ring + ring_base[blockIdx.x];
    Hist H{rp, n, ring_depth - 1, dt, 1.0 / dt};
    uint32_t err = 0u;
    const DipLds Si = dip_lds(dev[gi]);
    const int M = n - 1;                             // source dipoles per stage
    const int nth = init ? 1 : 2;
    // Lane layout.  A launch with many targets is throughput-bound: a lane
    // takes one source for both stage times (the fewest instructions per drive).
    // A launch with few targets (`wide`: at most one workgroup per SIMD) is a
    // latency chain, and the shortest chain that fits the block wins: in FP64
    // one charge per lane (4 drives' worth of lanes per source), else one source
    // per (stage, lane); the mixed form always takes one source per (stage, lane)
    // there.
    const int layout = MIXED ? (wide ? 1 : 0)
                             : (wide && 2 * nth * M <= BLOCK ? 2 : (wide && nth * M <= BLOCK ? 1 : 0));
    const int units = layout == 2 ? 2 * nth * M : (layout == 1 ? nth * M : M);
    // the target's own state (only this workgroup writes it, and only at its
    // end): when the last lane has no pair work it reads the state into LDS
    // while the others solve, so the tail does not wait on those loads; held
    // in LDS, the values add no register pressure to the pair loop
    __shared__ double own[6];
    const bool early = !init && units < BLOCK;
    if (early && tid == BLOCK - 1) {
        const double *h = rp + ((int64_t)(nstep & (ring_depth - 1)) * n + i) * 3;
        own[0] = h[0];
        own[1] = h[1];
        own[2] = h[2];
        own[3] = Ecur[gi];
        own[4] = W[2 * gi];
        own[5] = W[2 * gi + 1];
    }
    double acc0 = 0.0, acc1 = 0.0;                   // stage t_n + dt/2 (or t = 0), stage t_n + dt
    if (layout == 0) {
        // a lane takes one source for both stage times, which share its
        // constants and separation (and often the history segment)
        for (int jj = tid; jj < M; jj += BLOCK) {
            const int j = jj < i ? jj : jj + 1;
            const DipLds Sj = soa_lds(soa, out.n_dip, (uint32_t)(i0 + j));
            const double qj = soa_get(soa, out.n_dip, SF_Q, (uint32_t)(i0 + j));
            if constexpr (!MOVING) {
                if (!init) {
                    double eh, ef;
                    if constexpr (MIXED)
                        dipole_drive_mixed_stages(H, Si, Sj, j, qj * K_COUL, nstep, max_iter, err, eh, ef);
                    else
                        dipole_drive_fp64_stages(H, Si, Sj, j, qj * K_COUL, nstep, max_iter, err, eh, ef);
                    acc0 += eh;
                    acc1 += ef;
                    continue;
                }
            }
            acc0 += source_drive<MOVING, MIXED>(H, Si, Sj, j, qj, nstep, init ? 0.0 : 0.5, max_iter, err);
            if (!init) acc1 += source_drive<MOVING, MIXED>(H, Si, Sj, j, qj, nstep, 1.0, max_iter, err);
        }
    } else if (layout == 2) {
        // FP64, few targets: a lane per (stage, source, charge)
        for (int m = tid; m < 2 * nth * M; m += BLOCK) {
            const int th = m >= 2 * M ? 1 : 0, r = m - th * 2 * M;
            const int jj = r >> 1, w = r & 1;
            const int j = jj < i ? jj : jj + 1;
            const DipLds Sj = soa_lds(soa, out.n_dip, (uint32_t)(i0 + j));
            const double qj = soa_get(soa, out.n_dip, SF_Q, (uint32_t)(i0 + j));
            const double cf = w ? Sj.cfm : Sj.cfp, kq = (w ? -qj : qj) * K_COUL;
            const double theta = init ? 0.0 : (th ? 1.0 : 0.5);
            const double e = pair_drive<MOVING>(H, Si, Sj, j, cf, kq, nstep, theta, max_iter, err);
            if (th) acc1 += e; else acc0 += e;
        }
    } else {
        // a lane per (stage, source), for few targets
        for (int m = tid; m < nth * M; m += BLOCK) {
            const int th = m >= M ? 1 : 0, jj = m - th * M;    // (nth <= 2 stages)
            const int j = jj < i ? jj : jj + 1;
            const DipLds Sj = soa_lds(soa, out.n_dip, (uint32_t)(i0 + j));
            const double qj = soa_get(soa, out.n_dip, SF_Q, (uint32_t)(i0 + j));
            const double theta = init ? 0.0 : (th ? 1.0 : 0.5);
            const double e = source_drive<MOVING, MIXED>(H, Si, Sj, j, qj, nstep, theta, max_iter, err);
            if (th) acc1 += e; else acc0 += e;
        }
    }
    // lane 0 reads the target's constants here, and its state too without the
    // early read, so that the loads are in flight during the block sums (read
    // after the barrier they added one memory round trip to every workgroup)
    double st[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    double om = 0.0, gm = 0.0, fq = 0.0, dd0 = 0.0, eh = 0.0, ms = 0.0, vf = 0.0;
    if (tid == 0) {
        const DipDev &D = dev[gi];
        om = D.omega0;
        gm = D.gamma0;
        fq = D.f;
        dd0 = D.d0;
        eh = D.ehalf;
        ms = D.mspeed;
        vf = D.vfac;
        if (!init && !early) {
            const double *h = rp + ((int64_t)(nstep & (ring_depth - 1)) * n + i) * 3;
            st[0] = h[0];
            st[1] = h[1];
            st[2] = h[2];
            st[3] = Ecur[gi];
            st[4] = W[2 * gi];
            st[5] = W[2 * gi + 1];
        }
    }
    // block sums in a fixed order: within each wave, then over the waves
    for (int o = 32; o > 0; o >>= 1) {
        acc0 += __shfl_xor(acc0, o, 64);
        acc1 += __shfl_xor(acc1, o, 64);
    }
    if (lane == 0) {
        red[0][wave] = acc0;
        red[1][wave] = acc1;
    }
    __syncthreads();
    if (tid == 0) {
        double s0 = red[0][0], s1 = red[1][0];
        for (int v = 1; v < BLOCK / 64; ++v) {
            s0 += red[0][v];
            s1 += red[1][v];
        }
        const double w2 = om * om, g = gm, f = fq;
        if (init) {
            // t = 0: drive from the static pre-history, sample 0 = (d0, 0, d_ddot(0))
            const double E0 = s0;
            double *h = rp + (int64_t)i * 3;
            h[0] = dd0;
            h[1] = 0.0;
            h[2] = f * E0 - w2 * dd0;
            Ecur[gi] = E0;
            W[2 * gi] = 0.0;
            W[2 * gi + 1] = 0.0;
            put_row(out, 0, gi, dd0, 0.0, run_energy(w2, eh, dd0, 0.0), E0, 0.0, 0.0);
        } else {
            const double Em = s0, Ee = s1;
            double y0, y1, a0, Ec, W0, W1;
            if (early) {
                y0 = own[0];
                y1 = own[1];
                a0 = own[2];
                Ec = own[3];
                W0 = own[4];
                W1 = own[5];
            } else {
                y0 = st[0];
                y1 = st[1];
                a0 = st[2];
                Ec = st[3];
                W0 = st[4];
                W1 = st[5];
            }
            const double k1d = y1, k1v = f * Ec - g * y1 - w2 * y0;
            const double y0b = y0 + 0.5 * dt * k1d, y1b = y1 + 0.5 * dt * k1v;
            const double k2d = y1b, k2v = f * Em - g * y1b - w2 * y0b;
            const double y0c = y0 + 0.5 * dt * k2d, y1c = y1 + 0.5 * dt * k2v;
            const double k3d = y1c, k3v = f * Em - g * y1c - w2 * y0c;
            const double y0d = y0 + dt * k3d, y1d = y1 + dt * k3v;
            const double k4d = y1d, k4v = f * Ee - g * y1d - w2 * y0d;
            const double dn = y0 + dt / 6.0 * (k1d + 2.0 * k2d + 2.0 * k3d + k4d);
            const double vn = y1 + dt / 6.0 * (k1v + 2.0 * k2v + 2.0 * k3v + k4v);
            const double an = f * Ee - g * vn - w2 * dn;
            double *hn = rp + ((int64_t)((nstep + 1) & (ring_depth - 1)) * n + i) * 3;
            hn[0] = dn;
            hn[1] = vn;
            hn[2] = an;
            Ecur[gi] = Ee;
            if (!(isfinite(dn) && isfinite(vn) && isfinite(an))) err |= ERR_NONFINITE;
            if (max_vel > 0.0 && ms + vf * fabs(vn) > max_vel) err |= ERR_VELOCITY;
            // energy bookkeeping (Sec. 2.5), trapezoid rule over the step
            const double wa = W0 + 0.5 * dt * (y1 * Ec + vn * Ee);
            const double wr = W1 + 0.5 * dt * K_LARMOR * (a0 * a0 + an * an);
            W[2 * gi] = wa;
            W[2 * gi + 1] = wr;
            const int64_t rel = nstep + 1 - step_ctr[1];       // steps since the run's first
            const int64_t row = out_row(rel, out.stride);
            if (row >= 0) put_row(out, row, gi, dn, vn, run_energy(w2, eh, dn, vn), Ee, wa, wr);
        }
    }
    if (err) atomicOr(d_err, err);
}

__global__ void step_advance_kernel(int64_t *step_ctr, int64_t delta)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) *step_ctr += delta;
}

// The run's first step: 0, or the step count of the run state it resumes.
__global__ void step_start_kernel(int64_t *step_ctr, const double *resume)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        const int64_t n0 = resume ? (int64_t)resume[0] : 0;
        step_ctr[0] = n0;
        step_ctr[1] = n0;
    }
}

// A resumed run: the header check and output row 0 of every dipole from the
// state (d, d_dot at the state's step, E_d and the energy sums).
__global__ void state_rows_kernel(const DipDev *__restrict__ dev, const int32_t *__restrict__ off, int n_inst,
                                  const double *__restrict__ state, int ring, RunOut out,
                                  uint32_t *__restrict__ d_err)
{
    const int gi = blockIdx.x * blockDim.x + threadIdx.x;
    if (gi == 0 && !(state[1] == (double)ring && state[2] == (double)out.n_dip)) atomicOr(d_err, ERR_STATE);
    if (gi >= out.n_dip) return;
    const int inst = instance_of(off, n_inst, gi);
    const int a0 = off[inst], n = off[inst + 1] - a0;
    const int64_t n0 = (int64_t)state[0];
    const double *h = state + state_ring_off(a0, ring) + ((int64_t)(n0 & (ring - 1)) * n + (gi - a0)) * 3;
    const DipDev &D = dev[gi];
    const int64_t ow = state_w_off(out.n_dip, ring);
    put_row(out, 0, gi, h[0], h[1], run_energy(D.omega0 * D.omega0, D.ehalf, h[0], h[1]),
            state[state_ecur_off(out.n_dip, ring) + gi], state[ow + 2 * gi], state[ow + 2 * gi + 1]);
}

__global__ void state_header_kernel(double *state, int ring, int n_dip, int64_t steps, int resume)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        const int64_t n0 = resume ? (int64_t)state[0] : 0;
        state[0] = (double)(n0 + steps);
        state[1] = (double)ring;
        state[2] = (double)n_dip;
        state[3] = 0.0;
    }
}

hipError_t launch_state_rows(const DipDev *d_dev, const int32_t *d_off, int n_inst, const double *d_state, int ring,
                             const RunOut &out, uint32_t *d_err, hipStream_t s)
{
    hipLaunchKernelGGL(state_rows_kernel, dim3((out.n_dip + 255) / 256), dim3(256), 0, s, d_dev, d_off, n_inst,
                       d_state, ring, out, d_err);
    return hipGetLastError();
}

hipError_t launch_state_header(double *d_state, int ring, int n_dip, int64_t steps, bool resume, hipStream_t s)
{
    hipLaunchKernelGGL(state_header_kernel, dim3(1), dim3(1), 0, s, d_state, ring, n_dip, steps, resume ? 1 : 0);
    return hipGetLastError();
}

// Calls fn(std::integral_constant<bool, a>, std::integral_constant<bool, b>).
template <typename Fn> static void with_flags(bool a, bool b, Fn &&fn)
{
    if (a) {
        if (b) fn(std::true_type{}, std::true_type{});
        else fn(std::true_type{}, std::false_type{});
    } else {
        if (b) fn(std::false_type{}, std::true_type{});
        else fn(std::false_type{}, std::false_type{});
    }
}

hipError_t launch_dipole_steps(const DipDev *d_dev, const int32_t *d_tgt, const int32_t *d_tgt_lo, const int32_t *d_tgt_n,
                               const int64_t *d_ring_base, int n_tgt, double *d_ring, double *d_Ecur, double *d_W,
                               int64_t *d_step, int ring, int64_t steps, double dt, double max_vel, int max_iter,
                               const RunOut &out, bool moving, bool mixed, const double *d_resume, uint32_t *d_err,
                               int graph_chunk, hipStream_t s, hipStream_t cap, hipGraph_t *graph_out,
                               hipGraphExec_t *exec_out)
{
    constexpr int B = 256;
    if (n_tgt <= 0) return hipSuccess;
    const dim3 grid((unsigned)n_tgt), block(B);
    // at most one workgroup per SIMD (256 CUs x 4): a latency-bound launch
    const int wide = n_tgt <= 1024 ? 1 : 0;
    const double *soa = dip_soa(const_cast<DipDev *>(d_dev), out.n_dip);
    auto step = [&](hipStream_t q, int k, int init) {
        with_flags(moving, mixed, [&](auto mv, auto mx) {
            hipLaunchKernelGGL((lo_step_kernel<B, decltype(mv)::value, decltype(mx)::value>), grid, block, 0, q,
                               d_dev, d_tgt, d_tgt_lo, d_tgt_n, d_ring_base, d_ring, d_Ecur, d_W, d_step, k, ring, dt,
                               max_vel, max_iter, init, wide, out, soa, d_err);
        });
    };
    hipLaunchKernelGGL(step_start_kernel, dim3(1), dim3(1), 0, s, d_step, d_resume);
    if (!d_resume) step(s, 0, 1);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || steps == 0) return e;
    // a chunk of steps is captured once into a graph and replayed: launch k of
    // a chunk advances step base + k, and the base (on the device) moves by the
    // chunk at its end, so every replay continues where the last ended
    auto enqueue = [&](hipStream_t q, int64_t count) {
        for (int64_t k = 0; k < count; ++k) step(q, (int)k, 0);
        hipLaunchKernelGGL(step_advance_kernel, dim3(1), dim3(1), 0, q, d_step, count);
    };
    const int64_t chunk = graph_chunk > 0 ? graph_chunk : 0;
    if (chunk == 0 || steps < chunk || !cap) {
        enqueue(s, steps);
        return hipGetLastError();
    }
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
        enqueue(cap, chunk);
        e = hipStreamEndCapture(cap, &graph);
    }
    if (e == hipSuccess) e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    const int64_t reps = steps / chunk;
    for (int64_t r = 0; r < reps && e == hipSuccess; ++r) e = hipGraphLaunch(exec, s);
    if (e == hipSuccess && steps > reps * chunk) {
        enqueue(s, steps - reps * chunk);
        e = hipGetLastError();
    }
    // handed to the caller, which releases them once the stream has passed them
    *graph_out = graph;
    *exec_out = exec;
    return e;
}

int ring_lds_bytes(int n, int ring)
{
    return (int)(sizeof(DipLds) * n + sizeof(double) * 12 * n + sizeof(double) * 3 * (size_t)ring * n);
}

template <int BLOCK>
static hipError_t launch_lo(bool ring_lds, bool moving, bool mixed, dim3 grid, size_t shmem, hipStream_t s,
                            const DipDev *d_dev, const int32_t *d_off, const int32_t *d_list, int ring, int64_t steps,
                            double dt, double max_vel, int max_iter, double *d_ring_global,
                            const int64_t *d_ring_off, const RunOut &out, double *d_state, bool resume,
                            uint32_t *d_err)
{
    const int rs = resume ? 1 : 0;
    with_flags(moving, mixed, [&](auto mv, auto mx) {
        constexpr bool MV = decltype(mv)::value, MX = decltype(mx)::value;
        if (ring_lds)
            hipLaunchKernelGGL((lo_instances_kernel<BLOCK, true, MV, MX>), grid, dim3(BLOCK), shmem, s, d_dev, d_off,
                               d_list, ring, steps, dt, max_vel, max_iter, d_ring_global, d_ring_off, out, d_state,
                               rs, d_err);
        else
            hipLaunchKernelGGL((lo_instances_kernel<BLOCK, false, MV, MX>), grid, dim3(BLOCK), shmem, s, d_dev,
                               d_off, d_list, ring, steps, dt, max_vel, max_iter, d_ring_global, d_ring_off, out,
                               d_state, rs, d_err);
    });
    return hipGetLastError();
}

hipError_t launch_dipole_instances(const DipDev *d_dev, const int32_t *d_off, const int32_t *d_list, int n_list,
                                   int max_n, bool ring_lds, const int64_t *d_ring_off, double *d_ring_global,
                                   int ring, int64_t steps, double dt, double max_vel, int max_iter,
                                   const RunOut &out, bool moving, bool mixed, double *d_state, bool resume,
                                   uint32_t *d_err, hipStream_t s)
{
    if (n_list <= 0) return hipSuccess;
    const size_t shmem = (size_t)ring_lds_bytes(max_n, ring_lds ? ring : 0);
    const dim3 grid((unsigned)n_list);
    if (ring_lds && !moving && max_n <= SMALL_MAX_N) {
        if (mixed)
            hipLaunchKernelGGL(lo_small_kernel<true>, grid, dim3(64), shmem, s, d_dev, d_off, d_list, ring, steps, dt,
                               max_vel, max_iter, out, d_state, resume ? 1 : 0, d_err);
        else
            hipLaunchKernelGGL(lo_small_kernel<false>, grid, dim3(64), shmem, s, d_dev, d_off, d_list, ring, steps, dt,
                               max_vel, max_iter, out, d_state, resume ? 1 : 0, d_err);
        return hipGetLastError();
    }
    if (max_n <= 8)
        return launch_lo<64>(ring_lds, moving, mixed, grid, shmem, s, d_dev, d_off, d_list, ring, steps, dt, max_vel,
                             max_iter, d_ring_global, d_ring_off, out, d_state, resume, d_err);
    return launch_lo<256>(ring_lds, moving, mixed, grid, shmem, s, d_dev, d_off, d_list, ring, steps, dt, max_vel,
                          max_iter, d_ring_global, d_ring_off, out, d_state, resume, d_err);
}

}  // namespace lw
