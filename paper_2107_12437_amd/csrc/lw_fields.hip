// lw_fields.hip -- grid-field kernels for gfx950.
//
// One lane per observation point.  A workgroup covers `block` consecutive
// points and a chunk of observation times; for each time it loops over all
// charges, whose per-(time, charge) records are wave-uniform and come in
// through scalar loads.  Per pair: FP64 retarded-time solve (Eq. (ret_t)),
// Lienard-Wiechert terms in the working precision, compensated running sum.
// The ten outputs of a (point, time) are written as ten coalesced SoA rows
// with non-temporal stores (written once, never re-read by the kernel).
#include <math.h>

#include "lw_device.hpp"
#include "lw_internal.hpp"

namespace lw {

size_t src_rec_bytes() { return sizeof(SrcRec); }

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
        R.pad_ = 0;
        R.kq = T.q * K_COUL;
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
        recs[r] = R;
    }
    if (flags)
        for (int64_t p = gid; p < npts; p += gsz) flags[p] = 0u;
}

template <typename F> __device__ __forceinline__ F qnan();
template <> __device__ __forceinline__ float qnan<float>() { return __builtin_nanf(""); }
template <> __device__ __forceinline__ double qnan<double>() { return __builtin_nan(""); }

// F: working precision of the field terms and of the outputs.  In FP32 the
// running sums over charges carry a Kahan compensation term.
template <typename F>
__global__ __launch_bounds__(256) void fields_kernel(const SrcRec *__restrict__ recs, int nch,
                                                     const double *__restrict__ pts, int64_t npts, int nt,
                                                     int tchunk, int field_kind, int max_iter, double tol_rel,
                                                     double mask_r, F *__restrict__ out,
                                                     uint32_t *__restrict__ flags)
{
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= npts) return;
    const double x[3] = {pts[p], pts[npts + p], pts[2 * npts + p]};
    const int t0 = blockIdx.y * tchunk;
    const int t1 = min(t0 + tchunk, nt);
    uint32_t fl_all = 0u;
    for (int ti = t0; ti < t1; ++ti) {
        F sum[10], cmp[10];
#pragma unroll
        for (int j = 0; j < 10; ++j) { sum[j] = (F)0; cmp[j] = (F)0; }
        uint32_t fl = 0u;
        const SrcRec *R = recs + (int64_t)ti * nch;
        for (int c = 0; c < nch; ++c) {
            Kin k;
            retarded(R[c], x, max_iter, tol_rel, k);
            fl |= k.flags;
            F o[10];
            const F D = lw_terms<F>(k, R[c].kq, field_kind, o);
            if (!(D >= (F)mask_r)) fl |= FLAG_MASKED;
#pragma unroll
            for (int j = 0; j < 10; ++j) {
                if constexpr (sizeof(F) == 4) {
                    const F y = o[j] - cmp[j];
                    const F t = sum[j] + y;
                    cmp[j] = (t - sum[j]) - y;
                    sum[j] = t;
                } else {
                    sum[j] += o[j];
                }
            }
        }
        F *dst = out + (int64_t)ti * 10 * npts + p;
        if (fl & FLAG_MASKED) {
#pragma unroll
            for (int j = 0; j < 10; ++j) __builtin_nontemporal_store(qnan<F>(), dst + (int64_t)j * npts);
        } else {
#pragma unroll
            for (int j = 0; j < 10; ++j) __builtin_nontemporal_store(sum[j] - cmp[j], dst + (int64_t)j * npts);
        }
        fl_all |= fl;
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

hipError_t launch_fields(const SrcRec *d_recs, int nch, const double *d_pts, int64_t npts, int nt,
                         const lw_opts &o, double tol_rel, double mask_r, void *d_out, uint32_t *d_flags,
                         const FieldLaunch &L, hipStream_t s)
{
    const int block = L.block;
    int tchunk = L.tchunk < 1 ? 1 : L.tchunk;
    if ((nt + tchunk - 1) / tchunk > 65535) tchunk = (nt + 65534) / 65535;   // grid.y limit
    const dim3 grid((unsigned)((npts + block - 1) / block), (unsigned)((nt + tchunk - 1) / tchunk));
    const int max_iter = o.max_iter > 0 ? o.max_iter : 100;
    if (o.precision == LW_MIXED)
        hipLaunchKernelGGL(fields_kernel<float>, grid, dim3(block), 0, s, d_recs, nch, d_pts, npts, nt, tchunk,
                           o.field_kind, max_iter, tol_rel, mask_r, (float *)d_out, d_flags);
    else
        hipLaunchKernelGGL(fields_kernel<double>, grid, dim3(block), 0, s, d_recs, nch, d_pts, npts, nt, tchunk,
                           o.field_kind, max_iter, tol_rel, mask_r, (double *)d_out, d_flags);
    return hipGetLastError();
}

}  // namespace lw
