// lw_fields.hip -- grid-field kernels for gfx950.
//
// One lane per observation point.  A workgroup covers `block` consecutive
// points and a chunk of observation times; for each time it loops over all
// charges, whose per-(time, charge) records are wave-uniform and come in
// through scalar loads.  Per pair: FP64 retarded-time solve (Eq. (ret_t)),
// Lienard-Wiechert terms in the working precision, running sum over charges in
// FP64 (exact enough that the FP32 path needs no compensation term).
// The ten outputs of a (point, time) are written as ten coalesced SoA rows
// with non-temporal stores (written once, never re-read by the kernel).
#include <math.h>

#include "lw_device.hpp"
#include "lw_internal.hpp"

namespace lw {

size_t src_rec_bytes() { return sizeof(SrcRec); }

int output_mask(int outputs) { return outputs == 0 ? (OUT_PHI | OUT_A | OUT_E | OUT_B) : outputs; }

int output_rows(int outputs)
{
    const int m = output_mask(outputs);
    return ((m & OUT_PHI) ? 1 : 0) + 3 * (((m & OUT_A) ? 1 : 0) + ((m & OUT_E) ? 1 : 0) + ((m & OUT_B) ? 1 : 0) +
                                          ((m & OUT_S) ? 1 : 0));
}

__global__ void fill_zero_f64_kernel(double *__restrict__ p, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0.0;
}

hipError_t launch_fill_zero(double *d, int64_t n, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    const int64_t blocks = (n + 255) / 256;
    hipLaunchKernelGGL(fill_zero_f64_kernel, dim3((unsigned)(blocks < 1024 ? blocks : 1024)), dim3(256), 0, s, d, n);
    return hipGetLastError();
}

__global__ void prep_kernel(const lw_traj *__restrict__ ch, int nch, const double *__restrict__ times, int nt,
                            SrcRec *__restrict__ recs, uint32_t *__restrict__ flags, int64_t npts)
{
    const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t gsz = (int64_t)gridDim.x * blockDim.x;
    for (int64_t r = gid; r < (int64_t)nt * nch; r += gsz) {
        const int ti = (int)(r / nch), c = (int)(r % nch);
        const lw_traj &T = ch[c];
        SrcRec R;
        const double t = times[ti];
        R.kind = T.kind;
        R.kq = T.q * K_COUL;
        R.kqf = (float)R.kq;
        R.t = t;
        for (int i = 0; i < 3; ++i) {
            R.c0[i] = T.c0[i];
            R.e1[i] = T.e1[i];
            R.e2[i] = T.e2[i];
            R.v[i] = T.v[i];
            R.rt[i] = T.c0[i] + T.v[i] * t;
        }
        R.e3[0] = T.e1[1] * T.e2[2] - T.e1[2] * T.e2[1];
        R.e3[1] = T.e1[2] * T.e2[0] - T.e1[0] * T.e2[2];
        R.e3[2] = T.e1[0] * T.e2[1] - T.e1[1] * T.e2[0];
        R.amp = T.amp;
        R.omega = T.omega;
        double s, c_;
        sincos(fma(T.omega, t, T.phase), &s, &c_);
        R.cT = c_;
        R.sT = s;
        R.accel = T.accel;
        R.Lmax = (t > 0.0) ? 0.5 * T.accel * t * t : 0.0;
        const double bw = T.amp * T.omega * INV_C, aw = bw * T.omega;
        for (int i = 0; i < 3; ++i) {
            R.bw1[i] = (float)(bw * T.e1[i]);
            R.bw2[i] = (float)(bw * T.e2[i]);
            R.aw1[i] = (float)(aw * T.e1[i]);
            R.aw2[i] = (float)(aw * T.e2[i]);
        }
        if (T.kind == K_UNIFORM_VELOCITY) {
            // the closed form's constants (solve_uniform) and beta in FP32, once
            // per record instead of once per point
            const double vv = T.v[0] * T.v[0] + T.v[1] * T.v[1] + T.v[2] * T.v[2];
            R.amp = C_LIGHT * C_LIGHT - vv;
            R.omega = rcp_steer(R.amp);
            for (int i = 0; i < 3; ++i) R.bw1[i] = (float)(T.v[i] * INV_C);
        }
        recs[r] = R;
    }
    if (flags)
        for (int64_t p = gid; p < npts; p += gsz) flags[p] = 0u;
}

template <typename F> __device__ __forceinline__ F qnan();
template <> __device__ __forceinline__ float qnan<float>() { return __builtin_nanf(""); }
template <> __device__ __forceinline__ double qnan<double>() { return __builtin_nan(""); }

// F: working precision of the field terms and of the outputs.  The sums over
// charges are FP64 in both (an FP32 term converts exactly, and an FP64 add needs
// no compensation term).  Each lane owns one point and TCH consecutive times: the
// charge loop is outermost, so the part of each retarded-time problem that does
// not depend on time (frame coordinates, starting value and its sincos) is built
// once per (point, charge) and serves all TCH times.  The register cap: 4 waves
// per SIMD (128 VGPRs) at one time, 3 (168) at two and 2 (256) at four, whose
// sums stay in registers.  With their sums in LDS the one- and two-time forms
// compile to 61-83 VGPRs; LDS then holds the two-time form at 4 waves per SIMD.
// The launch tuner picks among them.
constexpr int waves_for(bool fp64, int tch) { return tch == 1 ? 4 : (tch == 2 ? 3 : 2); }

// Where the sums over charges live: in LDS for one and two times per lane (80 and
// 160 bytes per lane, so a CU's 160 KB hold 32 and 16 waves), in registers for
// four (320 bytes per lane would leave 8 waves per CU) and in the histogram
// instance.
constexpr bool lds_sums(bool hist, int tch) { return !hist && tch <= 2; }

// One charge of family KIND at the lane's point and its nti (>= 1) times: the
// geometry once, then per time the retarded kinematics, the terms in precision
// F, the flags and the FP64 sums of the requested rows (in LDS at lsum[(j * 10 +
// q) * 64] with LSUM, else in sum[j][q]).
template <typename F, int TCH, bool HIST, int KIND, bool LSUM>
__device__ __forceinline__ void charge_times(double *lsum, const SrcRec *__restrict__ R0, int nch, int c, const double x[3],
                                             int nti, int field_kind, int outputs, int max_iter, double tol_rel,
                                             double mask_r, bool live, double (&sum)[TCH][10],
                                             uint32_t (&fl)[TCH], unsigned int *s_hist)
{
    Geo g;
    // no bracket (the correction solves' fallback builds its own); the mixed path
    // also takes its start phase to about 1e-11
    geo_prepare_k<KIND, false, sizeof(F) == 8>(R0[c], x, g);
#pragma unroll
    for (int j = 0; j < TCH; ++j) {
        if (j == 0 || j < nti) {
            const SrcRec &S = R0[(int64_t)j * nch + c];
            Kin k;
            retarded_kind<sizeof(F) == 8, true, KIND>(S, g, x, max_iter, tol_rel, k);
            F o[10];
            // A and B without their factor 1/c: the sums are scaled once at the end
            const F D = lw_terms<F, false>(k, sizeof(F) == 4 ? (F)S.kqf : (F)S.kq, field_kind, o);
            fl[j] |= k.flags | ((D >= (F)mask_r) ? 0u : FLAG_MASKED);
            if constexpr (HIST) {
                if (live) {
                    const int bin = (k.iters & ITER_FALLBACK) ? ITER_BIN_FALLBACK : min(k.iters, ITER_BIN_FALLBACK - 1);
                    atomicAdd(&s_hist[bin], 1u);
                    if (k.flags & FLAG_NOCONV) atomicAdd(&s_hist[ITER_BIN_NOCONV], 1u);
                }
            }
            // the sums the requested rows need (the mask is uniform)
            auto add = [&](int q) {
                if constexpr (LSUM)
                    __hip_atomic_fetch_add(lsum + (j * 10 + q) * 64, (double)o[q], __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_WORKGROUP);
                else
                    sum[j][q] += (double)o[q];
            };
            if (outputs & OUT_PHI) add(0);
            if (outputs & OUT_A)
#pragma unroll
                for (int q = 1; q < 4; ++q) add(q);
            if (outputs & (OUT_E | OUT_S))
#pragma unroll
                for (int q = 4; q < 7; ++q) add(q);
            if (outputs & (OUT_B | OUT_S))
#pragma unroll
                for (int q = 7; q < 10; ++q) add(q);
        }
    }
}

// HIST (a debugging instance, launched with TCH = 1): each workgroup also counts
// its pairs by the iterations their retarded-time solve took, in LDS, and adds
// the counts to hist[ITER_BINS] (bins 0..30: that many iterations, 31: more;
// ITER_BIN_FALLBACK: mixed-path solves that fell back to the safeguarded
// solver; ITER_BIN_NOCONV: solves flagged as not converged).  Lanes past the
// last point stay alive to the final barrier.
template <typename F, int TCH, bool HIST = false>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(waves_for(sizeof(F) == 8, TCH)))) void fields_kernel(const SrcRec *__restrict__ recs, int nch,
                                                     const double *__restrict__ pts, int64_t npts, int nt,
                                                     int t_base, int field_kind, int outputs, int nrows,
                                                     int max_iter, double tol_rel, double mask_r,
                                                     F *__restrict__ out, uint32_t *__restrict__ flags,
                                                     unsigned long long *__restrict__ hist)
{
    const int64_t p0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    __shared__ unsigned int s_hist[HIST ? ITER_BINS : 1];
    if constexpr (HIST) {
        for (int i = threadIdx.x; i < ITER_BINS; i += blockDim.x) s_hist[i] = 0u;
        __syncthreads();
    } else {
        if (p0 >= npts) return;
    }
    const bool live = p0 < npts;
    const int64_t p = live ? p0 : 0;
    const double x[3] = {pts[p], pts[npts + p], pts[2 * npts + p]};
    const int t0 = t_base + blockIdx.y * TCH;
    const int nti = min(TCH, nt - t0);
    // The running sums: in LDS for one or two times per lane (each lane owns a
    // column of its wave's block of 10 TCH doubles x 64 lanes; ds_add_f64 adds
    // there without a VALU slot, in program order), else in registers.
    constexpr bool LSUM = lds_sums(HIST, TCH);
    extern __shared__ double s_sums[];
    double *lsum = s_sums + (threadIdx.x >> 6) * (TCH * 10 * 64) + (threadIdx.x & 63);
    double sum[TCH][10];
    uint32_t fl[TCH];
#pragma unroll
    for (int j = 0; j < TCH; ++j) {
        fl[j] = 0u;
#pragma unroll
        for (int q = 0; q < 10; ++q) {
            if constexpr (LSUM) lsum[(j * 10 + q) * 64] = 0.0;
            else sum[j][q] = 0.0;
        }
    }
    const SrcRec *R0 = recs + (int64_t)t0 * nch;
    for (int c = 0; c < nch; ++c) {
        // every time's record of a charge carries the charge's family, so the
        // solver is chosen once per charge and each family's times run as
        // straight-line code that shares the per-charge constants
        switch (R0[c].kind) {
        case K_CIRCULAR:
            charge_times<F, TCH, HIST, K_CIRCULAR, LSUM>(lsum, R0, nch, c, x, nti, field_kind, outputs, max_iter, tol_rel,
                                                   mask_r, live, sum, fl, s_hist);
            break;
        case K_LINEAR_OSC:
            charge_times<F, TCH, HIST, K_LINEAR_OSC, LSUM>(lsum, R0, nch, c, x, nti, field_kind, outputs, max_iter, tol_rel,
                                                     mask_r, live, sum, fl, s_hist);
            break;
        case K_ACCEL:
            charge_times<F, TCH, HIST, K_ACCEL, LSUM>(lsum, R0, nch, c, x, nti, field_kind, outputs, max_iter, tol_rel,
                                                mask_r, live, sum, fl, s_hist);
            break;
        case K_UNIFORM_VELOCITY:
            charge_times<F, TCH, HIST, K_UNIFORM_VELOCITY, LSUM>(lsum, R0, nch, c, x, nti, field_kind, outputs, max_iter,
                                                           tol_rel, mask_r, live, sum, fl, s_hist);
            break;
        default:
            charge_times<F, TCH, HIST, K_STATIONARY, LSUM>(lsum, R0, nch, c, x, nti, field_kind, outputs, max_iter, tol_rel,
                                                     mask_r, live, sum, fl, s_hist);
            break;
        }
    }
    if constexpr (HIST) {
        __syncthreads();
        for (int i = threadIdx.x; i < ITER_BINS; i += blockDim.x)
            if (s_hist[i]) atomicAdd(hist + i, (unsigned long long)s_hist[i]);
        if (!live) return;
    }
    uint32_t fl_all = 0u;
#pragma unroll
    for (int j = 0; j < TCH; ++j) {
        if (j < nti) {
            F *dst = out + (int64_t)(t0 + j) * nrows * npts + p;
            const bool masked = (fl[j] & FLAG_MASKED) != 0u;
            int r = 0;
            auto put = [&](double v) {
                __builtin_nontemporal_store(masked ? qnan<F>() : (F)v, dst + (int64_t)r * npts);
                ++r;
            };
            double S[10];
#pragma unroll
            for (int q = 0; q < 10; ++q) {
                const double v = LSUM ? lsum[(j * 10 + q) * 64] : sum[j][q];
                S[q] = (q >= 1 && q <= 3) || q >= 7 ? v * INV_C : v;
            }
            if (outputs & OUT_PHI) put(S[0]);
            if (outputs & OUT_A) { put(S[1]); put(S[2]); put(S[3]); }
            if (outputs & OUT_E) { put(S[4]); put(S[5]); put(S[6]); }
            if (outputs & OUT_B) { put(S[7]); put(S[8]); put(S[9]); }
            if (outputs & OUT_S) {
                // Poynting vector E x B / mu0 of the summed fields, 1/mu0 = eps0 c^2
                constexpr double IMU0 = EPS0 * C_LIGHT * C_LIGHT;
                put((S[5] * S[9] - S[6] * S[8]) * IMU0);
                put((S[6] * S[7] - S[4] * S[9]) * IMU0);
                put((S[4] * S[8] - S[5] * S[7]) * IMU0);
            }
            fl_all |= fl[j];
        }
    }
    if (flags && fl_all) atomicOr(flags + p, fl_all);
}

hipError_t launch_prep(const lw_traj *d_ch, int nch, const double *d_times, int nt, SrcRec *d_recs,
                       uint32_t *d_flags, int64_t npts, hipStream_t s)
{
    const int64_t work = (int64_t)nt * nch;
    const int64_t fill = d_flags ? npts : 0;
    int64_t n = work > fill ? work : fill;
    int blocks = (int)((n + 255) / 256);
    if (blocks < 1) blocks = 1;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(prep_kernel, dim3(blocks), dim3(256), 0, s, d_ch, nch, d_times, nt, d_recs, d_flags,
                       npts);
    return hipGetLastError();
}

template <typename F, int TCH, bool HIST = false>
static hipError_t launch_fields_t(const SrcRec *d_recs, int nch, const double *d_pts, int64_t npts, int nt,
                                  const lw_opts &o, double tol_rel, double mask_r, F *d_out, uint32_t *d_flags,
                                  int block, hipStream_t s, unsigned long long *d_hist = nullptr)
{
    // whole waves only: the LDS sums are laid out per wave of 64 lanes
    if (block < 64 || block > 256 || block % 64 != 0) return hipErrorInvalidValue;
    const int max_iter = o.max_iter > 0 ? o.max_iter : 100;
    const unsigned gx = (unsigned)((npts + block - 1) / block);
    // grid.y holds at most 65535 time tiles: longer time lists go in slices
    const int per_launch = 65535 * TCH;
    for (int tb = 0; tb < nt; tb += per_launch) {
        const int n_here = min(per_launch, nt - tb);
        const dim3 grid(gx, (unsigned)((n_here + TCH - 1) / TCH));
        const size_t lds = lds_sums(HIST, TCH) ? (size_t)TCH * 10 * block * sizeof(double) : 0;
        hipLaunchKernelGGL((fields_kernel<F, TCH, HIST>), grid, dim3(block), lds, s, d_recs, nch, d_pts, npts, nt, tb,
                           o.field_kind, output_mask(o.outputs), output_rows(o.outputs), max_iter, tol_rel, mask_r,
                           d_out, d_flags, d_hist);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

template <typename F>
static hipError_t launch_fields_f(const SrcRec *d_recs, int nch, const double *d_pts, int64_t npts, int nt,
                                  const lw_opts &o, double tol_rel, double mask_r, F *d_out, uint32_t *d_flags,
                                  const FieldLaunch &L, hipStream_t s, unsigned long long *d_hist)
{
    if (d_hist)
        return launch_fields_t<F, 1, true>(d_recs, nch, d_pts, npts, nt, o, tol_rel, mask_r, d_out, d_flags, 256, s,
                                           d_hist);
    if (L.tchunk >= 4)
        return launch_fields_t<F, 4>(d_recs, nch, d_pts, npts, nt, o, tol_rel, mask_r, d_out, d_flags, L.block, s);
    if (L.tchunk >= 2)
        return launch_fields_t<F, 2>(d_recs, nch, d_pts, npts, nt, o, tol_rel, mask_r, d_out, d_flags, L.block, s);
    return launch_fields_t<F, 1>(d_recs, nch, d_pts, npts, nt, o, tol_rel, mask_r, d_out, d_flags, L.block, s);
}

hipError_t launch_fields(const SrcRec *d_recs, int nch, const double *d_pts, int64_t npts, int nt,
                         const lw_opts &o, double tol_rel, double mask_r, void *d_out, uint32_t *d_flags,
                         const FieldLaunch &L, hipStream_t s, unsigned long long *d_hist)
{
    if (o.precision == LW_MIXED)
        return launch_fields_f<float>(d_recs, nch, d_pts, npts, nt, o, tol_rel, mask_r, (float *)d_out, d_flags, L, s,
                                      d_hist);
    return launch_fields_f<double>(d_recs, nch, d_pts, npts, nt, o, tol_rel, mask_r, (double *)d_out, d_flags, L, s,
                                   d_hist);
}

}  // namespace lw
