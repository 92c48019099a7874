// lw_dipole.hpp -- oscillator records and history access shared by the
// forward run (lw_dipole.hip) and its adjoint (lw_dipole_adjoint.hip).
#pragma once

#include <limits>

#include "lw_device.hpp"
#include "lw_internal.hpp"

namespace lw {

struct DipDev {
    double origin[3];
    double axis[3];
    double omega0;
    double q;
    double f;        // q^2 / m  (m = m1 m2 / (m1 + m2), Eq. (eff_mass))
    double gamma0;   // q^2 omega0^2 / (6 pi eps0 c^3 m)  (Sec. 2.3)
    double cfp;      // offset of the +q charge per unit moment: m2 / (m1 + m2) / q   (Eq. (r_1))
    double cfm;      // offset of the -q charge per unit moment: -m1 / (m1 + m2) / q  (Eq. (r_2))
    double vfac;     // charge speed per unit d_dot: max(m1, m2) / (m1 + m2) / q
    double d0;
    double mamp[3];  // origin motion: origin + mamp cos(mw t + mph) (Sec. 4.3); mw = 0 when fixed
    double mw, mph;
    double mspeed;   // largest origin speed, mw |mamp|
    double ehalf;    // 0.5 / f, the factor of the energy (run_energy)
};

// Per-dipole constants of the instance, staged in LDS.
struct DipLds {
    double ox, oy, oz;
    double px, py, pz;
    double cfp, cfm;
    double d0;
    double mx, my, mz, mw, mph;   // origin motion (mw = 0: fixed origin)
};

// Structure-of-arrays copy of the source fields the pair loops read: field f of
// dipole j at soa[f * n + j] (n dipoles in the run), so that a wave's load of
// one field over consecutive sources is coalesced.  It follows the DipDev
// array in the same block (dip_soa).
enum { SF_OX, SF_OY, SF_OZ, SF_PX, SF_PY, SF_PZ, SF_CFP, SF_CFM, SF_D0, SF_Q, SF_MX, SF_MY, SF_MZ, SF_MW, SF_MPH,
       SF_COUNT };

__host__ __device__ inline size_t dip_dev_array_bytes(int n) { return (sizeof(DipDev) * (size_t)n + 255) & ~(size_t)255; }
__host__ __device__ inline double *dip_soa(DipDev *dev, int n) { return (double *)((char *)dev + dip_dev_array_bytes(n)); }

// Field f of dipole j (the 32-bit byte offset of j lets each load take the
// field's base as a scalar operand).
__device__ __forceinline__ double soa_get(const double *__restrict__ s, int64_t n, int f, uint32_t j)
{
    return *(const double *)((const char *)(s + f * n) + j * 8u);
}

__device__ __forceinline__ DipLds soa_lds(const double *__restrict__ s, int64_t n, uint32_t j)
{
    return DipLds{soa_get(s, n, SF_OX, j),  soa_get(s, n, SF_OY, j),  soa_get(s, n, SF_OZ, j),
                  soa_get(s, n, SF_PX, j),  soa_get(s, n, SF_PY, j),  soa_get(s, n, SF_PZ, j),
                  soa_get(s, n, SF_CFP, j), soa_get(s, n, SF_CFM, j), soa_get(s, n, SF_D0, j),
                  soa_get(s, n, SF_MX, j),  soa_get(s, n, SF_MY, j),  soa_get(s, n, SF_MZ, j),
                  soa_get(s, n, SF_MW, j),  soa_get(s, n, SF_MPH, j)};
}

// Origin of a dipole at time t (fixed, or moving as O + m cos(w t + phi); the
// phase stays far below the 2^30 limit of sincos_reduced over any run).
__device__ __forceinline__ void origin_at(const DipLds &S, double t, double R[3])
{
    R[0] = S.ox;
    R[1] = S.oy;
    R[2] = S.oz;
    if (S.mw != 0.0) {
        double sn, c;
        sincos_reduced(S.mw * t + S.mph, sn, c);
        R[0] += S.mx * c;
        R[1] += S.my * c;
        R[2] += S.mz * c;
    }
}

// Stored kinematics (d, d_dot, d_ddot) of source j at s steps after t = 0 (s
// real).  Static at d0 before t = 0 (Sec. 3.2); linear interpolation between
// stored steps (Sec. 3.1); beyond the newest step `nstep` a second-order
// Taylor step from it (reached only when c dt exceeds a separation).
struct Hist {
    const double *ring;   // [ring][n][3]
    int n;
    int mask;             // ring - 1
    double dt;
    double inv_dt;
};

__device__ __forceinline__ DipLds dip_lds(const DipDev &D)
{
    return DipLds{D.origin[0], D.origin[1], D.origin[2], D.axis[0], D.axis[1], D.axis[2], D.cfp, D.cfm, D.d0,
                  D.mamp[0], D.mamp[1], D.mamp[2], D.mw, D.mph};
}

enum { ERR_HISTORY = 1u, ERR_NOCONV = 2u, ERR_VELOCITY = 4u, ERR_NONFINITE = 8u, ERR_STATE = 16u };

// Instance of global dipole g (last instance whose first dipole is <= g).
__device__ __forceinline__ int instance_of(const int32_t *off, int n_inst, int g)
{
    int lo = 0, hi = n_inst;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (off[mid] <= g) lo = mid; else hi = mid;
    }
    return lo;
}


// Stored samples k and k + 1 of one source; k = -1 stands for the static
// pre-history (t' < 0), where the state is (d0, 0, 0).  Step indices are of
// type I: int64_t, or int in a kernel that has checked its run fits (32-bit
// integer arithmetic is single instructions; 64-bit is not).  Every floating
// value is the same for both.
template <typename I>
struct SegT {
    I k;
    double d0, v0, a0;    // sample k: d, d_dot, d_ddot
    double d1, v1, a1;    // sample k + 1
};
using Seg = SegT<int64_t>;

// Segment index meaning "none loaded".
template <typename I> __host__ __device__ constexpr I seg_none() { return std::numeric_limits<I>::min(); }

template <typename I>
__device__ __forceinline__ void seg_load(const Hist &H, int j, double d0, I nstep, I k, SegT<I> &g, uint32_t &err)
{
    // k = -1 reads ring slot `mask` (in bounds) and discards it
    const bool pre = k < 0;
    g.k = pre ? -1 : k;
    if (!pre && k + H.mask < nstep) err |= ERR_HISTORY;   // the slot was overwritten: history too short
    const double *p0 = H.ring + ((I)(g.k & H.mask) * H.n + j) * 3;
    const double *p1 = H.ring + ((I)((g.k + 1) & H.mask) * H.n + j) * 3;
    g.d0 = pre ? d0 : p0[0];
    g.v0 = pre ? 0.0 : p0[1];
    g.a0 = pre ? 0.0 : p0[2];
    g.d1 = pre ? d0 : p1[0];
    g.v1 = pre ? 0.0 : p1[1];
    g.a1 = pre ? 0.0 : p1[2];
}

// Retarded time of the charge at offset cf d(t') p_j of a fixed source j, in
// closed form on the interpolated history.  Within the segment [k, k + 1] of
// stored steps the moment is linear in tau (t' = t - tau), so the charge's
// offset is rho = a + b tau and c tau = |Delta - rho p_j| becomes
//   (c^2 - b^2) tau^2 + 2 b P tau - Q = 0,
// P = sD - a, Q = |Delta - a p_j|^2 = L2 - 2 a sD + a^2, whose positive root
// tau = Q / (b P + sqrt(b^2 P^2 + (c^2 - b^2) Q)) has no cancellation
// (|b| << c).  The root is unique (the charge is slower than light), so if it
// falls outside the loaded segment it lies in the segment its own s points to,
// which is loaded next.  Returns false when the root lies past the newest
// stored step (the caller then uses the Newton solve with the extrapolation)
// or the hops do not settle.  On success tau_out is the root, h the
// interpolated state there and g the segment it lies in.
template <typename I>
__device__ __forceinline__ bool retarded_seg(const Hist &H, int j, double d0, I nstep, double base, double L2,
                                             double sD, double cf, SegT<I> &g, double h[3], double &tau_out,
                                             uint32_t &err)
{
    constexpr double C2 = C_LIGHT * C_LIGHT;
    for (int hop = 0; hop < 4; ++hop) {
        double a = cf * d0, b = 0.0;
        if (g.k >= 0) {
            const double dd = g.d1 - g.d0;
            a = cf * fma(base - (double)g.k, dd, g.d0);
            b = -cf * dd * H.inv_dt;
        }
        const double P = sD - a;
        const double Q = fma(a, a - 2.0 * sD, L2);
        const double bP = b * P;
        double S, iS;
        root_rsqrt<true>(fma(bP, bP, (C2 - b * b) * Q), S, iS);
        const double tau = Q * recip<double>(bP + S);
        const double s = base - tau * H.inv_dt;
        // a root within rounding of a segment end belongs to either side
        const double eps = 1e-9;
        if (g.k < 0 ? s <= eps : (s >= (double)g.k - eps && s <= (double)g.k + 1.0 + eps)) {
            const double u = g.k < 0 ? 0.0 : s - (double)g.k;
            h[0] = fma(u, g.d1 - g.d0, g.d0);
            h[1] = fma(u, g.v1 - g.v0, g.v0);
            h[2] = fma(u, g.a1 - g.a0, g.a0);
            tau_out = tau;
            return true;
        }
        const I kn = s < 0.0 ? -1 : (I)floor(s);
        if (kn >= nstep) return false;
        seg_load(H, j, d0, nstep, kn, g, err);
    }
    return false;
}

// Larmor power per |d_ddot|^2 (Sec. 2.5): 1 / (6 pi eps0 c^3).
constexpr double K_LARMOR = 1.0 / (6.0 * PI * EPS0 * C_LIGHT * C_LIGHT * C_LIGHT);

// Energy of Eq. (dipoleE) from (d, d_dot): (omega0^2 d^2 + d_dot^2) / (2 f),
// f = q^2 / m, in one fixed order of operations wherever it is evaluated.
// ehalf = 0.5 / f is the dipole's constant (DipDev::ehalf), so that no
// division sits on a step's critical path.
__device__ __forceinline__ double run_energy(double w2, double ehalf, double d, double v)
{
    return fma(w2 * d, d, v * v) * ehalf;
}

// Output row of the state after `rel` steps of the call, or -1 when the
// stride skips it (stride 1, the usual case, needs no 64-bit division, which
// has no hardware instruction and would sit on each step's critical path).
__device__ __forceinline__ int64_t out_row(int64_t rel, int64_t stride)
{
    if (stride == 1) return rel;
    return rel % stride == 0 ? rel / stride : -1;
}

// Writes row `row` of the outputs for dipole gi.
__device__ __forceinline__ void put_row(const RunOut &o, int64_t row, int gi, double d, double v, double E, double Ed,
                                        double wa, double wr)
{
    const int64_t k = row * o.n_dip + gi;
    o.d[k] = d;
    if (o.v) o.v[k] = v;
    if (o.E) o.E[k] = E;
    if (o.Ed) o.Ed[k] = Ed;
    if (o.wabs) o.wabs[k] = wa;
    if (o.wrad) o.wrad[k] = wr;
}

}  // namespace lw
