// lw_api.cpp -- host runtime and C ABI of liblw.so (see include/lw.h).
//
// The context owns a growable device workspace, a pinned staging buffer for
// the small host-side inputs (trajectories, times, oscillator records) and a
// device error word that oscillator kernels latch errors into.  Every call
// validates its arguments on the host, stages its inputs, and enqueues the
// preparation and compute kernels on the caller's stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <complex>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "lw_device.hpp"
#include "lw_internal.hpp"

namespace {

thread_local std::string g_last_error;

lw_status fail(lw_status st, const std::string &msg)
{
    g_last_error = msg;
    return st;
}

#define LW_HIP(call)                                                                                   \
    do {                                                                                               \
        hipError_t e_ = (call);                                                                        \
        if (e_ != hipSuccess) return fail(LW_E_HIP, std::string(#call ": ") + hipGetErrorString(e_)); \
    } while (0)

constexpr double C_LIGHT = 299792458.0;
constexpr double EPS0 = 8.8541878128e-12;
constexpr double PI = 3.14159265358979323846;

bool finite3(const double *v) { return std::isfinite(v[0]) && std::isfinite(v[1]) && std::isfinite(v[2]); }
double norm3(const double *v) { return std::sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]); }
bool unit3(const double *v) { return std::fabs(norm3(v) - 1.0) <= 1e-9; }

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// Scratch of lw_fields_noalloc: the charges, the times and the (time, charge)
// records of one call.  It is static device memory, one copy per GPU, held until
// the process ends.  In host code the array's name is not a device address:
// scratch_setup takes each device's address with hipGetSymbolAddress (with that
// device current) and every host use goes through g_scratch[device].
static __device__ __align__(256) unsigned char scratch[LW_NOALLOC_SCRATCH_BYTES];

constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void *g_scratch[MAX_DEVICES] = {};

// Once per device, with `device` current: the device address of its scratch.
lw_status scratch_setup(int device)
{
    if (device < 0 || device >= MAX_DEVICES) return fail(LW_E_INVALID, "device index beyond the scratch table");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch[device]) return LW_OK;
    void *ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
        return fail(LW_E_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_scratch[device] = ptr;
    return LW_OK;
}

}  // namespace

struct lw_ctx {
    int device = 0;
    void *d_work = nullptr;
    size_t work_cap = 0;
    void *h_stage = nullptr;
    size_t stage_cap = 0;
    hipEvent_t stage_evt = nullptr;
    bool stage_pending = false;
    uint32_t *d_err = nullptr;
    lw::FieldLaunch field_launch{256, 2};  // untuned shape: the fastest on the grid benchmark in both precisions
    hipStream_t side = nullptr;        // small instances run here, joined back into the caller's stream
    hipStream_t capture = nullptr;     // graph capture of stepped runs
    hipEvent_t join_a = nullptr, join_b = nullptr;
    hipGraph_t graph = nullptr;        // last stepped run's graph, released once the stream passed it
    hipGraphExec_t graph_exec = nullptr;
    hipEvent_t graph_done = nullptr;
    // launch-shape tuner for the grid kernel: shape class -> best (block, tchunk)
    void *d_work2 = nullptr;           // adjoint runs: full history and its cotangents
    size_t work2_cap = 0;
    bool autotune = true;
    std::map<std::string, lw::FieldLaunch> tuned;
    std::map<std::string, int> tuned_dip;   // oscillator runs: shape class -> stepped-path threshold
    std::string tune_file;
    double *d_trial = nullptr;         // tuner trial outputs
    size_t trial_cap = 0;
    hipStream_t adj_side = nullptr;    // checkpointed adjoint: window builder
    hipEvent_t adj_built = nullptr, adj_swept = nullptr;
    unsigned long long *d_hist = nullptr;   // retarded-time iteration histogram (debugging)
    bool iter_hist = false;
};

namespace {

// Device workspace of at least `bytes`; reallocation waits for the stream so
// no enqueued kernel still reads the old buffer.
lw_status ensure_work(lw_ctx *ctx, size_t bytes, hipStream_t s)
{
    if (bytes <= ctx->work_cap) return LW_OK;
    LW_HIP(hipStreamSynchronize(s));
    if (ctx->d_work) LW_HIP(hipFree(ctx->d_work));
    ctx->d_work = nullptr;
    ctx->work_cap = 0;
    size_t cap = align_up(std::max(bytes, (size_t)1 << 20), (size_t)1 << 20);
    if (hipMalloc(&ctx->d_work, cap) != hipSuccess) {
        (void)hipGetLastError();
        return fail(LW_E_NOMEM, "device workspace allocation of " + std::to_string(cap) + " bytes failed");
    }
    ctx->work_cap = cap;
    return LW_OK;
}

// How far a dipole's origin strays from its mean position (0 when fixed; a
// nonzero amplitude needs a nonzero frequency).
double motion_reach(const lw_dipole &D) { return norm3(D.motion_amp); }

lw_status ensure_work2(lw_ctx *ctx, size_t bytes, hipStream_t s)
{
    if (bytes <= ctx->work2_cap) return LW_OK;
    LW_HIP(hipStreamSynchronize(s));
    if (ctx->d_work2) LW_HIP(hipFree(ctx->d_work2));
    ctx->d_work2 = nullptr;
    ctx->work2_cap = 0;
    size_t cap = align_up(std::max(bytes, (size_t)1 << 20), (size_t)1 << 20);
    if (hipMalloc(&ctx->d_work2, cap) != hipSuccess) {
        (void)hipGetLastError();
        return fail(LW_E_NOMEM, "adjoint workspace allocation of " + std::to_string(cap) + " bytes failed");
    }
    ctx->work2_cap = cap;
    return LW_OK;
}

// Pinned staging of at least `bytes`, free for writing (the previous upload
// from it has completed).
lw_status acquire_stage(lw_ctx *ctx, size_t bytes)
{
    if (ctx->stage_pending) {
        LW_HIP(hipEventSynchronize(ctx->stage_evt));
        ctx->stage_pending = false;
    }
    if (bytes <= ctx->stage_cap) return LW_OK;
    if (ctx->h_stage) LW_HIP(hipHostFree(ctx->h_stage));
    ctx->h_stage = nullptr;
    ctx->stage_cap = 0;
    size_t cap = align_up(std::max(bytes, (size_t)1 << 16), (size_t)1 << 16);
    if (hipHostMalloc(&ctx->h_stage, cap, hipHostMallocDefault) != hipSuccess) {
        (void)hipGetLastError();
        return fail(LW_E_NOMEM, "pinned staging allocation failed");
    }
    ctx->stage_cap = cap;
    return LW_OK;
}

lw_status upload(lw_ctx *ctx, void *d_dst, size_t bytes, hipStream_t s)
{
    LW_HIP(hipMemcpyAsync(d_dst, ctx->h_stage, bytes, hipMemcpyHostToDevice, s));
    LW_HIP(hipEventRecord(ctx->stage_evt, s));
    ctx->stage_pending = true;
    return LW_OK;
}

lw_status check_traj(const lw_traj &T, int idx, double t_max)
{
    const std::string who = "charge " + std::to_string(idx) + ": ";
    if (T.kind < LW_STATIONARY || T.kind > LW_ACCEL) return fail(LW_E_INVALID, who + "unknown trajectory kind");
    if (!std::isfinite(T.q) || !finite3(T.c0)) return fail(LW_E_INVALID, who + "non-finite q or c0");
    switch (T.kind) {
    case LW_UNIFORM_VELOCITY:
        if (!finite3(T.v)) return fail(LW_E_INVALID, who + "non-finite velocity");
        if (!(norm3(T.v) < C_LIGHT)) return fail(LW_E_SUPERLUMINAL, who + "|v| >= c");
        break;
    case LW_LINEAR_OSC:
    case LW_CIRCULAR:
        if (!std::isfinite(T.amp) || !std::isfinite(T.omega) || !std::isfinite(T.phase) || T.amp < 0.0)
            return fail(LW_E_INVALID, who + "bad amplitude, frequency or phase");
        if (!unit3(T.e1)) return fail(LW_E_INVALID, who + "e1 is not a unit vector");
        if (T.kind == LW_CIRCULAR) {
            if (!unit3(T.e2)) return fail(LW_E_INVALID, who + "e2 is not a unit vector");
            const double d = T.e1[0] * T.e2[0] + T.e1[1] * T.e2[1] + T.e1[2] * T.e2[2];
            if (std::fabs(d) > 1e-9) return fail(LW_E_INVALID, who + "e1 and e2 are not orthogonal");
        }
        if (!(std::fabs(T.amp * T.omega) < C_LIGHT)) return fail(LW_E_SUPERLUMINAL, who + "amp*omega >= c");
        break;
    case LW_ACCEL:
        if (!std::isfinite(T.accel) || T.accel < 0.0) return fail(LW_E_INVALID, who + "bad acceleration");
        if (!unit3(T.e1)) return fail(LW_E_INVALID, who + "e1 is not a unit vector");
        if (!(T.accel * std::max(t_max, 0.0) < C_LIGHT))
            return fail(LW_E_SUPERLUMINAL, who + "speed reaches c before the last time");
        break;
    default:
        break;
    }
    return LW_OK;
}

// Shape class of a grid-field call: precision, field kind, charges, times and
// the point count rounded up to a power of two.
// Shape class of a grid call: precision, field kind, charge and time counts, the
// point count rounded up to a power of two, the set of trajectory families present
// (bit k for kind k: each family's solver has its own cost and register needs) and
// the output rows when not all four groups.
std::string field_key(const lw_opts &o, const lw_traj *ch, int nch, int nt, int64_t npts)
{
    int64_t p2 = 1;
    while (p2 < npts) p2 <<= 1;
    unsigned fam = 0u;
    for (int c = 0; c < nch; ++c)
        if (ch[c].kind >= 0 && ch[c].kind < 32) fam |= 1u << ch[c].kind;
    const int om = lw::output_mask(o.outputs);
    return "fields p" + std::to_string(o.precision) + " k" + std::to_string(o.field_kind) + " c" + std::to_string(nch) +
           " t" + std::to_string(nt) + " n" + std::to_string(p2) + " f" + std::to_string(fam) +
           (om == 15 ? "" : " o" + std::to_string(om));
}

void load_tune_file(lw_ctx *ctx)
{
    const char *f = std::getenv("LW_TUNE_CACHE");
    if (!f || !*f) return;
    ctx->tune_file = f;
    FILE *fp = std::fopen(f, "r");
    if (!fp) return;
    char line[512];
    while (std::fgets(line, sizeof line, fp)) {
        // "<key words...> | <block> <tchunk>"
        char *bar = std::strchr(line, '|');
        if (!bar) continue;
        std::string key(line, bar - line);
        while (!key.empty() && key.back() == ' ') key.pop_back();
        int b = 0, t = 0;
        if (key.rfind("dipoles", 0) == 0) {
            if (std::sscanf(bar + 1, "%d", &b) == 1 && b >= 2) ctx->tuned_dip[key] = b;
        } else if (std::sscanf(bar + 1, "%d %d", &b, &t) == 2 && b >= 64 && b <= 256 && b % 64 == 0 && t >= 1) {
            ctx->tuned[key] = lw::FieldLaunch{b, t};
        }
    }
    std::fclose(fp);
}

void save_tune_entry(lw_ctx *ctx, const std::string &key, const lw::FieldLaunch &L)
{
    if (ctx->tune_file.empty()) return;
    FILE *fp = std::fopen(ctx->tune_file.c_str(), "a");
    if (!fp) return;
    std::fprintf(fp, "%s | %d %d\n", key.c_str(), L.block, L.tchunk);
    std::fclose(fp);
}

void save_tune_dip(lw_ctx *ctx, const std::string &key, int threshold)
{
    if (ctx->tune_file.empty()) return;
    FILE *fp = std::fopen(ctx->tune_file.c_str(), "a");
    if (!fp) return;
    std::fprintf(fp, "%s | %d\n", key.c_str(), threshold);
    std::fclose(fp);
}

}  // namespace

extern "C" {

const char *lw_last_error(void) { return g_last_error.c_str(); }

double lw_gamma0(double q, double m, double omega0)
{
    return q * q * omega0 * omega0 / (6.0 * PI * EPS0 * C_LIGHT * C_LIGHT * C_LIGHT * m);
}

namespace {

using cplx = std::complex<double>;

// p1 . G(R, omega) . p2 for the free-space dyadic Green's function of App. A in
// the form k^2 e^{ikR} / (4 pi R) [(1 + (ikR - 1)/(kR)^2) I + (3 - 3ikR - (kR)^2)/(kR)^2 R^R^]
// (the field of a dipole d is G d / eps0), and its derivative in k.
void green_pp(const double R[3], const double p1[3], const double p2[3], cplx k, cplx &G, cplx &dG)
{
    const double r = norm3(R);
    const double c1 = (p1[0] * R[0] + p1[1] * R[1] + p1[2] * R[2]) / r;
    const double c2 = (p2[0] * R[0] + p2[1] * R[1] + p2[2] * R[2]) / r;
    const double pp = p1[0] * p2[0] + p1[1] * p2[1] + p1[2] * p2[2];
    const cplx I(0.0, 1.0);
    // G = e^{ikr} / (4 pi r^3) [pp (k^2 r^2 + ikr - 1) + c1 c2 (3 - 3ikr - k^2 r^2)]
    const cplx e = std::exp(I * k * r) / (4.0 * PI * r * r * r);
    const cplx a = pp * (k * k * r * r + I * k * r - 1.0) + c1 * c2 * (3.0 - 3.0 * I * k * r - k * k * r * r);
    const cplx da = pp * (2.0 * k * r * r + I * r) + c1 * c2 * (-3.0 * I * r - 2.0 * k * r * r);
    G = e * a;
    dG = e * (I * r * a + da);
}

}  // namespace

lw_status lw_gf_pair(const double *R, const double *p1, const double *p2, double omega0, double *out)
{
    if (!R || !p1 || !p2 || !out) return fail(LW_E_INVALID, "lw_gf_pair: null argument");
    if (!finite3(R) || !(norm3(R) > 0.0) || !unit3(p1) || !unit3(p2) || !(omega0 > 0.0) || !std::isfinite(omega0))
        return fail(LW_E_INVALID, "lw_gf_pair: bad separation, axes or frequency");
    const double k = omega0 / C_LIGHT;
    cplx G, dG;
    green_pp(R, p1, p2, cplx(k, 0.0), G, dG);
    const double im_self = k * k * k / (6.0 * PI);      // Im G(r, r) for a unit axis
    out[0] = -G.real() / (2.0 * im_self);               // delta_12 / gamma_0   (Eq. (qed_delta))
    out[1] = G.imag() / im_self;                        // gamma_12 / gamma_0   (Eq. (qed_gamma_ab))
    return LW_OK;
}

lw_status lw_exact_modes(const double *R, const double *p, double q, double m, double omega0, double *out)
{
    if (!R || !p || !out) return fail(LW_E_INVALID, "lw_exact_modes: null argument");
    if (!finite3(R) || !(norm3(R) > 0.0) || !unit3(p) || !(q > 0.0) || !(m > 0.0) || !(omega0 > 0.0) ||
        !std::isfinite(q) || !std::isfinite(m) || !std::isfinite(omega0))
        return fail(LW_E_INVALID, "lw_exact_modes: bad arguments");
    // d1, d2 ~ e^{-i omega t}: the oscillator equation with the drive of the other
    // dipole's field at its origin, p . E = (1/eps0) p . G . p d (G as above at
    // k = omega / c), gives for d2 = +-d1
    //   F(omega) = omega0^2 - omega^2 - i gamma0 omega -+ (q^2 / (m eps0)) p.G(omega).p = 0
    const double g0 = lw_gamma0(q, m, omega0);
    const double f = q * q / (m * EPS0);
    const cplx I(0.0, 1.0);
    cplx roots[2];
    for (int s = 0; s < 2; ++s) {
        const double sign = s == 0 ? 1.0 : -1.0;
        cplx w(omega0, -0.5 * g0);
        bool ok = false;
        for (int it = 0; it < 100; ++it) {
            cplx G, dG;
            green_pp(R, p, p, w / C_LIGHT, G, dG);
            const cplx F = omega0 * omega0 - w * w - I * g0 * w - sign * f * G;
            const cplx dF = -2.0 * w - I * g0 - sign * f * dG / C_LIGHT;
            const cplx dw = F / dF;
            w -= dw;
            if (std::abs(dw) <= 1e-15 * std::abs(w)) {
                ok = true;
                break;
            }
        }
        if (!ok || !std::isfinite(w.real()) || !std::isfinite(w.imag()))
            return fail(LW_E_NOCONV, "lw_exact_modes: the mode root did not converge");
        roots[s] = w;
    }
    out[0] = -2.0 * roots[0].imag();                    // gamma_+ (in-phase mode)
    out[1] = -2.0 * roots[1].imag();                    // gamma_- (antiphase mode)
    out[2] = roots[0].real();
    out[3] = roots[1].real();
    out[4] = 0.5 * (roots[0].real() - roots[1].real());
    return LW_OK;
}

lw_status lw_create(lw_ctx **out, int32_t device)
{
    if (!out) return fail(LW_E_INVALID, "lw_create: null output pointer");
    *out = nullptr;
    int n = 0;
    LW_HIP(hipGetDeviceCount(&n));
    if (device < 0 || device >= n) return fail(LW_E_INVALID, "lw_create: no such device");
    LW_HIP(hipSetDevice(device));
    lw_ctx *c = new (std::nothrow) lw_ctx;
    if (!c) return fail(LW_E_NOMEM, "lw_create: out of host memory");
    c->device = device;
    if (hipMalloc(&c->d_err, 256) != hipSuccess) {
        delete c;
        return fail(LW_E_NOMEM, "lw_create: error word allocation failed");
    }
    if (hipMemset(c->d_err, 0, 256) != hipSuccess || hipEventCreateWithFlags(&c->stage_evt, hipEventDisableTiming) != hipSuccess) {
        (void)hipFree(c->d_err);
        delete c;
        return fail(LW_E_HIP, "lw_create: HIP initialisation failed");
    }
    const char *at = std::getenv("LW_AUTOTUNE");
    if (at && at[0] == '0') c->autotune = false;
    load_tune_file(c);
    const lw_status sst = scratch_setup(device);
    if (sst != LW_OK) {
        const std::string msg = g_last_error;
        lw_destroy(c);
        return fail(sst, "lw_create: " + msg);
    }
    *out = c;
    return LW_OK;
}

lw_status lw_set_autotune(lw_ctx *ctx, int32_t enable)
{
    if (!ctx) return fail(LW_E_INVALID, "lw_set_autotune: null context");
    ctx->autotune = enable != 0;
    return LW_OK;
}

lw_status lw_destroy(lw_ctx *ctx)
{
    if (!ctx) return LW_OK;
    (void)hipSetDevice(ctx->device);
    (void)hipDeviceSynchronize();
    if (ctx->graph_exec) (void)hipGraphExecDestroy(ctx->graph_exec);
    if (ctx->graph) (void)hipGraphDestroy(ctx->graph);
    if (ctx->graph_done) (void)hipEventDestroy(ctx->graph_done);
    if (ctx->join_a) (void)hipEventDestroy(ctx->join_a);
    if (ctx->join_b) (void)hipEventDestroy(ctx->join_b);
    if (ctx->side) (void)hipStreamDestroy(ctx->side);
    if (ctx->adj_side) (void)hipStreamDestroy(ctx->adj_side);
    if (ctx->adj_built) (void)hipEventDestroy(ctx->adj_built);
    if (ctx->adj_swept) (void)hipEventDestroy(ctx->adj_swept);
    if (ctx->capture) (void)hipStreamDestroy(ctx->capture);
    if (ctx->stage_evt) (void)hipEventDestroy(ctx->stage_evt);
    if (ctx->h_stage) (void)hipHostFree(ctx->h_stage);
    if (ctx->d_work) (void)hipFree(ctx->d_work);
    if (ctx->d_work2) (void)hipFree(ctx->d_work2);
    if (ctx->d_trial) (void)hipFree(ctx->d_trial);
    if (ctx->d_err) (void)hipFree(ctx->d_err);
    if (ctx->d_hist) (void)hipFree(ctx->d_hist);
    delete ctx;
    return LW_OK;
}

lw_status lw_set_iteration_histogram(lw_ctx *ctx, int32_t enable)
{
    if (!ctx) return fail(LW_E_INVALID, "lw_set_iteration_histogram: null context");
    LW_HIP(hipSetDevice(ctx->device));
    if (enable && !ctx->d_hist) {
        if (hipMalloc(&ctx->d_hist, sizeof(unsigned long long) * LW_ITER_BINS) != hipSuccess) {
            ctx->d_hist = nullptr;
            return fail(LW_E_NOMEM, "lw_set_iteration_histogram: allocation failed");
        }
        LW_HIP(lw::launch_fill_zero((double *)ctx->d_hist, LW_ITER_BINS, nullptr));
        LW_HIP(hipDeviceSynchronize());
    }
    ctx->iter_hist = enable != 0;
    return LW_OK;
}

lw_status lw_iteration_histogram(lw_ctx *ctx, uint64_t *h_bins, int32_t n_bins, int32_t reset, void *stream)
{
    if (!ctx) return fail(LW_E_INVALID, "lw_iteration_histogram: null context");
    if (!ctx->d_hist) return fail(LW_E_INVALID, "lw_iteration_histogram: counting was never turned on");
    if (n_bins < 0 || n_bins > LW_ITER_BINS || (n_bins > 0 && !h_bins))
        return fail(LW_E_INVALID, "lw_iteration_histogram: bad output");
    LW_HIP(hipSetDevice(ctx->device));
    hipStream_t s = (hipStream_t)stream;
    LW_HIP(hipStreamSynchronize(s));
    if (n_bins > 0) LW_HIP(hipMemcpy(h_bins, ctx->d_hist, sizeof(uint64_t) * (size_t)n_bins, hipMemcpyDeviceToHost));
    if (reset) {
        LW_HIP(lw::launch_fill_zero((double *)ctx->d_hist, LW_ITER_BINS, s));
        LW_HIP(hipStreamSynchronize(s));
    }
    return LW_OK;
}

lw_status lw_sync_status(lw_ctx *ctx, void *stream)
{
    if (!ctx) return fail(LW_E_INVALID, "lw_sync_status: null context");
    LW_HIP(hipSetDevice(ctx->device));
    hipStream_t s = (hipStream_t)stream;
    LW_HIP(hipStreamSynchronize(s));
    uint32_t e = 0;
    LW_HIP(hipMemcpy(&e, ctx->d_err, sizeof(e), hipMemcpyDeviceToHost));
    if (e) LW_HIP(hipMemset(ctx->d_err, 0, sizeof(uint32_t)));
    if (e & 8u) return fail(LW_E_NONFINITE, "an oscillator state became non-finite");
    if (e & 4u) return fail(LW_E_VELOCITY, "a dipole charge exceeded the speed limit");
    if (e & 1u) return fail(LW_E_HISTORY, "a retarded time fell outside the stored history");
    if (e & 2u) return fail(LW_E_NOCONV, "a retarded-time solve did not converge");
    if (e & 16u) return fail(LW_E_STATE, "a resumed run's state does not match its dipoles or history depth");
    return LW_OK;
}

}  // extern "C"

namespace {

// Argument checks shared by lw_fields and lw_fields_vjp.  Sets *noop when there
// is nothing to compute.
lw_status check_fields_args(const char *who, lw_ctx *ctx, const lw_traj *h_charges, int32_t n_charges,
                            const double *d_pts, int64_t n_pts, const double *h_times, int32_t n_times,
                            const lw_opts *opts, const void *d_out, bool *noop)
{
    const std::string w = who;
    *noop = false;
    if (!ctx || !opts) return fail(LW_E_INVALID, w + ": null context or options");
    if (n_charges < 1 || !h_charges) return fail(LW_E_INVALID, w + ": need at least one charge");
    if (n_pts < 0 || n_times < 0) return fail(LW_E_INVALID, w + ": negative size");
    if (opts->precision != LW_FP64 && opts->precision != LW_MIXED) return fail(LW_E_INVALID, w + ": unknown precision");
    if (opts->field_kind < LW_FIELD_TOTAL || opts->field_kind > LW_FIELD_RADIATION)
        return fail(LW_E_INVALID, w + ": unknown field kind");
    if (opts->max_iter < 0 || opts->max_iter > 100000 || std::isnan(opts->mask_radius))
        return fail(LW_E_INVALID, w + ": bad options");
    if ((opts->outputs & ~(LW_OUT_PHI | LW_OUT_A | LW_OUT_E | LW_OUT_B | LW_OUT_S)) != 0)
        return fail(LW_E_INVALID, w + ": unknown output bits");
    if (n_pts == 0 || n_times == 0) {
        *noop = true;
        return LW_OK;
    }
    if (!d_pts || !d_out || !h_times) return fail(LW_E_INVALID, w + ": null buffer");
    if (n_times > 65535 * 64) return fail(LW_E_INVALID, w + ": too many times");
    if (n_pts > ((int64_t)1 << 40)) return fail(LW_E_INVALID, w + ": too many points");
    double t_max = -INFINITY;
    for (int i = 0; i < n_times; ++i) {
        if (!std::isfinite(h_times[i])) return fail(LW_E_INVALID, w + ": non-finite time");
        t_max = std::max(t_max, h_times[i]);
    }
    for (int c = 0; c < n_charges; ++c) {
        lw_status st = check_traj(h_charges[c], c, t_max);
        if (st != LW_OK) return st;
    }
    return LW_OK;
}

// Stages charges and times and enqueues the record preparation; returns the
// device records.  extra_bytes of workspace follow the records (at *d_extra).
lw_status stage_records(lw_ctx *ctx, const lw_traj *h_charges, int32_t n_charges, const double *h_times,
                        int32_t n_times, uint32_t *d_flags, int64_t n_pts, size_t extra_bytes, hipStream_t s,
                        lw::SrcRec **d_recs_out, void **d_extra)
{
    const size_t ch_bytes = align_up(sizeof(lw_traj) * (size_t)n_charges, 256);
    const size_t tm_bytes = align_up(sizeof(double) * (size_t)n_times, 256);
    const size_t rec_bytes = align_up(lw::src_rec_bytes() * (size_t)n_charges * (size_t)n_times, 256);
    lw_status st = ensure_work(ctx, ch_bytes + tm_bytes + rec_bytes + extra_bytes, s);
    if (st != LW_OK) return st;
    st = acquire_stage(ctx, ch_bytes + tm_bytes);
    if (st != LW_OK) return st;
    char *stage = (char *)ctx->h_stage;
    std::memcpy(stage, h_charges, sizeof(lw_traj) * (size_t)n_charges);
    std::memcpy(stage + ch_bytes, h_times, sizeof(double) * (size_t)n_times);
    char *work = (char *)ctx->d_work;
    st = upload(ctx, work, ch_bytes + tm_bytes, s);
    if (st != LW_OK) return st;
    lw::SrcRec *d_recs = (lw::SrcRec *)(work + ch_bytes + tm_bytes);
    LW_HIP(lw::launch_prep((const lw_traj *)work, n_charges, (const double *)(work + ch_bytes), n_times, d_recs,
                           d_flags, n_pts, s));
    *d_recs_out = d_recs;
    if (d_extra) *d_extra = work + ch_bytes + tm_bytes + rec_bytes;
    return LW_OK;
}

}  // namespace

extern "C" {

lw_status lw_fields(lw_ctx *ctx, const lw_traj *h_charges, int32_t n_charges, const double *d_pts, int64_t n_pts,
                    const double *h_times, int32_t n_times, const lw_opts *opts, void *d_out, uint32_t *d_flags,
                    void *stream)
{
    bool noop = false;
    lw_status st0 = check_fields_args("lw_fields", ctx, h_charges, n_charges, d_pts, n_pts, h_times, n_times, opts,
                                      d_out, &noop);
    if (st0 != LW_OK || noop) return st0;
    LW_HIP(hipSetDevice(ctx->device));
    hipStream_t s = (hipStream_t)stream;
    lw::SrcRec *d_recs = nullptr;
    lw_status st = stage_records(ctx, h_charges, n_charges, h_times, n_times, d_flags, n_pts, 0, s, &d_recs, nullptr);
    if (st != LW_OK) return st;
    const double mask_r = opts->mask_radius < 0.0 ? 1e-10 : opts->mask_radius;
    const double tol_rel = opts->precision == LW_FP64 ? 4.0 * 2.220446049250313e-16 : 2.3283064365386963e-10;
    if (ctx->iter_hist) {
        LW_HIP(lw::launch_fields(d_recs, n_charges, d_pts, n_pts, n_times, *opts, tol_rel, mask_r, d_out, d_flags,
                                 ctx->field_launch, s, ctx->d_hist));
        return LW_OK;
    }
    lw::FieldLaunch L = ctx->field_launch;
    const std::string key = field_key(*opts, h_charges, n_charges, n_times, n_pts);
    auto it = ctx->tuned.find(key);
    if (it != ctx->tuned.end()) {
        L = it->second;
    } else if (ctx->autotune) {
        // time every candidate shape once (after one untimed launch) on this call's
        // own inputs; the final launch below writes the result
        hipEvent_t e0, e1;
        LW_HIP(hipEventCreate(&e0));
        LW_HIP(hipEventCreate(&e1));
        float best = 1e30f;
        for (int b : {64, 128, 256})
            for (int t : {1, 2, 4}) {
                if (t > 1 && t >= 2 * n_times) continue;
                const lw::FieldLaunch C{b, t};
                LW_HIP(lw::launch_fields(d_recs, n_charges, d_pts, n_pts, n_times, *opts, tol_rel, mask_r, d_out,
                                         nullptr, C, s));
                LW_HIP(hipEventRecord(e0, s));
                LW_HIP(lw::launch_fields(d_recs, n_charges, d_pts, n_pts, n_times, *opts, tol_rel, mask_r, d_out,
                                         nullptr, C, s));
                LW_HIP(hipEventRecord(e1, s));
                LW_HIP(hipEventSynchronize(e1));
                float ms = 0.f;
                LW_HIP(hipEventElapsedTime(&ms, e0, e1));
                if (ms < best) {
                    best = ms;
                    L = C;
                }
            }
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        ctx->tuned[key] = L;
        save_tune_entry(ctx, key, L);
    }
    LW_HIP(lw::launch_fields(d_recs, n_charges, d_pts, n_pts, n_times, *opts, tol_rel, mask_r, d_out, d_flags, L, s));
    return LW_OK;
}

lw_status lw_fields_noalloc(lw_ctx *ctx, const lw_traj *h_charges, int32_t n_charges, const double *d_pts,
                            int64_t n_pts, const double *h_times, int32_t n_times, const lw_opts *opts, void *d_out,
                            uint32_t *d_flags, void *stream)
{
    bool noop = false;
    lw_status st = check_fields_args("lw_fields_noalloc", ctx, h_charges, n_charges, d_pts, n_pts, h_times, n_times,
                                     opts, d_out, &noop);
    if (st != LW_OK || noop) return st;
    // the three parts of the scratch, each sized in a way that cannot overflow
    // (check_fields_args bounds n_times; n_charges is a positive int32)
    const size_t cap = LW_NOALLOC_SCRATCH_BYTES;
    const size_t ch_bytes = align_up(sizeof(lw_traj) * (size_t)n_charges, 256);
    const size_t tm_bytes = align_up(sizeof(double) * (size_t)n_times, 256);
    const size_t n_rec = (size_t)n_charges * (size_t)n_times;
    if (ch_bytes > cap || tm_bytes > cap || n_rec > cap / lw::src_rec_bytes() ||
        ch_bytes + tm_bytes + align_up(lw::src_rec_bytes() * n_rec, 256) > cap)
        return fail(LW_E_INVALID, "lw_fields_noalloc: " + std::to_string(n_charges) + " charges x " +
                                      std::to_string(n_times) + " times need more than the " +
                                      std::to_string(cap) + "-byte scratch (LW_NOALLOC_SCRATCH_BYTES)");
    LW_HIP(hipSetDevice(ctx->device));
    hipStream_t s = (hipStream_t)stream;
    void *base = g_scratch[ctx->device];
    if (!base) {
        st = scratch_setup(ctx->device);
        if (st != LW_OK) return st;
        base = g_scratch[ctx->device];
    }
    char *sc = (char *)base;
    LW_HIP(hipMemcpyAsync(sc, h_charges, sizeof(lw_traj) * (size_t)n_charges, hipMemcpyHostToDevice, s));
    LW_HIP(hipMemcpyAsync(sc + ch_bytes, h_times, sizeof(double) * (size_t)n_times, hipMemcpyHostToDevice, s));
    lw::SrcRec *d_recs = (lw::SrcRec *)(sc + ch_bytes + tm_bytes);
    // the prep kernel rewrites every record of this call and clears the flags
    LW_HIP(lw::launch_prep((const lw_traj *)sc, n_charges, (const double *)(sc + ch_bytes), n_times, d_recs, d_flags,
                           n_pts, s));
    const double mask_r = opts->mask_radius < 0.0 ? 1e-10 : opts->mask_radius;
    const double tol_rel = opts->precision == LW_FP64 ? 4.0 * 2.220446049250313e-16 : 2.3283064365386963e-10;
    LW_HIP(lw::launch_fields(d_recs, n_charges, d_pts, n_pts, n_times, *opts, tol_rel, mask_r, d_out, d_flags,
                             ctx->field_launch, s));
    return LW_OK;
}

lw_status lw_fields_vjp(lw_ctx *ctx, const lw_traj *h_charges, int32_t n_charges, const double *d_pts,
                        int64_t n_pts, const double *h_times, int32_t n_times, const lw_opts *opts, const void *d_cot,
                        double *d_grad, void *stream)
{
    bool noop = false;
    if (!d_grad) return fail(LW_E_INVALID, "lw_fields_vjp: null gradient buffer");
    lw_status st = check_fields_args("lw_fields_vjp", ctx, h_charges, n_charges, d_pts, n_pts, h_times, n_times, opts,
                                     d_cot, &noop);
    if (st != LW_OK) return st;
    LW_HIP(hipSetDevice(ctx->device));
    hipStream_t s = (hipStream_t)stream;
    if (opts->outputs & LW_OUT_S) return fail(LW_E_INVALID, "lw_fields_vjp: the Poynting vector has no adjoint here");
    if (noop) {
        LW_HIP(lw::launch_fill_zero(d_grad, (int64_t)n_charges * lw::vjp_params(), s));
        return LW_OK;
    }
    const int tchunk = 4;
    const size_t part_bytes = align_up(sizeof(double) * lw::vjp_partial_doubles(n_pts, n_times, n_charges, tchunk), 256);
    lw::SrcRec *d_recs = nullptr;
    void *d_partial = nullptr;
    st = stage_records(ctx, h_charges, n_charges, h_times, n_times, nullptr, n_pts, part_bytes, s, &d_recs, &d_partial);
    if (st != LW_OK) return st;
    const double mask_r = opts->mask_radius < 0.0 ? 1e-10 : opts->mask_radius;
    const double tol_rel = 4.0 * 2.220446049250313e-16;     // the adjoint recomputes the forward in FP64
    LW_HIP(lw::launch_fields_vjp(d_recs, n_charges, d_pts, n_pts, n_times, *opts, tol_rel, mask_r, d_cot,
                                 (double *)d_partial, tchunk, d_grad, s));
    return LW_OK;
}

// Validation of an oscillator run's arguments and its history depth: the ring
// of stored steps covers the longest retarded time.
static lw_status run_geometry(const char *who, const lw_dipole *h_dip, int32_t n_dip, const int32_t *h_inst_off,
                              int32_t n_inst, double dt, int64_t steps, const lw_run_opts *opts, int *ring_out)
{
    const std::string w = who;
    if (!opts || !h_dip || !h_inst_off) return fail(LW_E_INVALID, w + ": null argument");
    if (n_dip < 1 || n_inst < 1) return fail(LW_E_INVALID, w + ": need at least one dipole and instance");
    if (h_inst_off[0] != 0 || h_inst_off[n_inst] != n_dip)
        return fail(LW_E_INVALID, w + ": instance offsets must run from 0 to n_dip");
    if (!(dt > 0.0) || !std::isfinite(dt) || steps < 0) return fail(LW_E_INVALID, w + ": bad dt or steps");
    if (opts->precision != LW_FP64 && opts->precision != LW_MIXED)
        return fail(LW_E_INVALID, w + ": unknown precision");
    if (opts->dt_policy != LW_DT_STRICT && opts->dt_policy != LW_DT_EXTRAPOLATE)
        return fail(LW_E_INVALID, w + ": unknown dt policy");
    if (opts->out_stride < 1 || opts->ring_depth < 0 ||
        (opts->ring_depth & (opts->ring_depth - 1)) != 0 || !std::isfinite(opts->max_vel))
        return fail(LW_E_INVALID, w + ": bad options");
    for (int i = 0; i < n_dip; ++i) {
        const lw_dipole &D = h_dip[i];
        if (!finite3(D.origin) || !unit3(D.axis) || !(D.omega0 > 0.0) || !std::isfinite(D.omega0) ||
            !(D.q > 0.0) || !std::isfinite(D.q) || !(D.m1 > 0.0) || !(D.m2 > 0.0) || !std::isfinite(D.m1) ||
            !std::isfinite(D.m2) || !std::isfinite(D.d0) || !finite3(D.motion_amp) ||
            !std::isfinite(D.motion_omega) || !std::isfinite(D.motion_phase) ||
            !(std::fabs(D.motion_omega) * norm3(D.motion_amp) < 0.1 * C_LIGHT) ||
            (norm3(D.motion_amp) > 0.0 && D.motion_omega == 0.0))
            return fail(LW_E_INVALID, w + ": bad parameters for dipole " + std::to_string(i));
    }
    // separations inside each instance: distinct origins, the dt rule, and the
    // longest light travel time (history depth)
    // (squared distances for fixed pairs; moving origins (Sec. 4.3) stay within
    // their amplitudes of the mean position)
    std::vector<double> reach((size_t)n_dip);
    for (int i = 0; i < n_dip; ++i) reach[i] = motion_reach(h_dip[i]);
    const bool strict = opts->dt_policy == LW_DT_STRICT;
    const double cdt = C_LIGHT * dt, cdt2 = cdt * cdt;
    double max_sep = 0.0, max_r2 = 0.0;
    int bad_a = -1, bad_b = -1;
    lw_status bad = LW_OK;
    for (int k = 0; k < n_inst && bad == LW_OK; ++k) {
        const int a0 = h_inst_off[k], a1 = h_inst_off[k + 1];
        if (a1 < a0) return fail(LW_E_INVALID, w + ": decreasing instance offsets");
        for (int a = a0; a < a1 && bad == LW_OK; ++a) {
            const double *oa = h_dip[a].origin;
            for (int b = a + 1; b < a1; ++b) {
                const double *ob = h_dip[b].origin;
                const double dx = oa[0] - ob[0], dy = oa[1] - ob[1], dz = oa[2] - ob[2];
                const double r2 = dx * dx + dy * dy + dz * dz;
                const double swing = reach[a] + reach[b];
                if (swing == 0.0) {
                    max_r2 = std::max(max_r2, r2);
                    if (!(r2 > 0.0)) bad = LW_E_INVALID;
                    else if (strict && !(cdt2 < r2)) bad = LW_E_DT_TOO_LARGE;
                } else {
                    const double r = std::sqrt(r2);
                    max_sep = std::max(max_sep, r + swing);
                    if (!(r - swing > 0.0)) bad = LW_E_INVALID;
                    else if (strict && !(cdt < r - swing)) bad = LW_E_DT_TOO_LARGE;
                }
                if (bad != LW_OK) {
                    bad_a = a;
                    bad_b = b;
                    break;
                }
            }
        }
    }
    if (bad == LW_E_INVALID) return fail(LW_E_INVALID, w + ": two dipoles can share an origin");
    if (bad == LW_E_DT_TOO_LARGE)
        return fail(LW_E_DT_TOO_LARGE, w + ": c*dt is not below the separation of dipoles " +
                                           std::to_string(bad_a) + " and " + std::to_string(bad_b));
    max_sep = std::max(max_sep, std::sqrt(max_r2));
    // depth: the longest retarded time (plus the charges' own excursion) in
    // steps, two interpolation neighbours and one step of slack
    const double need = std::ceil(2.0 * max_sep / C_LIGHT / dt) + 3.0;
    if (need > (double)(1 << 24)) return fail(LW_E_INVALID, w + ": dt too small for the separations");
    int ring = 4;
    while (ring < (int)need) ring <<= 1;
    if (opts->ring_depth) {
        if (opts->ring_depth < (int)need)
            return fail(LW_E_INVALID, w + ": ring_depth below the longest retarded time");
        ring = opts->ring_depth;
    }
    *ring_out = ring;
    return LW_OK;
}

static lw_status dipole_run_impl(lw_ctx *ctx, const lw_dipole *h_dip, int32_t n_dip, const int32_t *h_inst_off,
                                 int32_t n_inst, double dt, int64_t steps, const lw_run_opts *opts,
                                 double *d_moment, double *d_dot, double *d_energy, double *d_drive, double *d_wabs,
                                 double *d_wrad, double *d_state, int64_t n_state, bool resume, void *stream);

// Stepped-path threshold (stepped_min_n) for a run's shape class: precision,
// moving origins, dt policy, history depth and the instance sizes by power of
// two.  Cached in the context (and the LW_TUNE_CACHE file); otherwise each
// threshold that splits the instances differently is timed on trial runs of
// the call's own dipoles, and the fastest is kept.  A trial's per-step cost is
// the difference of a 512-step and a 256-step run, so the per-call cost of
// staging and graph capture drops out.  Trials write two rows of moments into
// a context buffer and no run state; tuning synchronises the stream once.
static lw_status tune_stepped(lw_ctx *ctx, const lw_dipole *h_dip, int32_t n_dip, const int32_t *h_inst_off,
                              int32_t n_inst, double dt, const lw_run_opts *opts, int ring, hipStream_t s, int *out)
{
    bool moving = false;
    for (int i = 0; i < n_dip; ++i) moving = moving || motion_reach(h_dip[i]) > 0.0;
    std::map<int, int> sizes;                        // ceil(log2 n) -> instances
    int max_n = 0;
    for (int k = 0; k < n_inst; ++k) {
        const int n = h_inst_off[k + 1] - h_inst_off[k];
        if (n <= 0) continue;
        int b = 0;
        while ((1 << b) < n) ++b;
        ++sizes[b];
        max_n = std::max(max_n, n);
    }
    std::string key = "dipoles p" + std::to_string(opts->precision) + " m" + std::to_string(moving ? 1 : 0) + " d" +
                      std::to_string(opts->dt_policy) + " r" + std::to_string(ring) + " n";
    for (const auto &kv : sizes) key += " " + std::to_string(1 << kv.first) + ":" + std::to_string(kv.second);
    auto it = ctx->tuned_dip.find(key);
    if (it != ctx->tuned_dip.end()) {
        *out = it->second;
        return LW_OK;
    }
    *out = 16;
    if (!ctx->autotune) return LW_OK;
    // candidate thresholds: powers of two up to past the largest instance, one
    // per distinct split of the instances
    std::vector<int> cand;
    int last_split = -1;
    for (int T = 2; T <= 2 * std::max(max_n, 2); T <<= 1) {
        int stepped = 0;
        for (int k = 0; k < n_inst; ++k) {
            const int n = h_inst_off[k + 1] - h_inst_off[k];
            if (n > 0 && (n >= T || lw::ring_lds_bytes(n, ring) > 64 * 1024)) ++stepped;
        }
        if (stepped != last_split) cand.push_back(T);
        last_split = stepped;
    }
    const size_t need = sizeof(double) * 2 * (size_t)n_dip;
    if (ctx->trial_cap < need) {
        LW_HIP(hipStreamSynchronize(s));
        if (ctx->d_trial) LW_HIP(hipFree(ctx->d_trial));
        ctx->d_trial = nullptr;
        ctx->trial_cap = 0;
        if (hipMalloc((void **)&ctx->d_trial, need) != hipSuccess) return fail(LW_E_NOMEM, "tuner trial buffer");
        ctx->trial_cap = need;
    }
    // The trials run the call's own dipoles for up to 512 steps, which may latch an
    // error (speed limit, history) that the call itself, if shorter, never meets:
    // the error word a caller has not read yet is saved, each candidate runs on a
    // cleared word, a candidate whose trials latched anything is dropped, and the
    // saved word is put back.
    uint32_t saved_err = 0;
    const uint32_t zero_err = 0;
    LW_HIP(hipStreamSynchronize(s));
    LW_HIP(hipMemcpy(&saved_err, ctx->d_err, sizeof(uint32_t), hipMemcpyDeviceToHost));
    hipEvent_t ev[3];
    for (auto &e : ev) LW_HIP(hipEventCreate(&e));
    float best = 1e30f;
    lw_status st = LW_OK;
    for (int T : cand) {
        lw_run_opts o = *opts;
        o.stepped_min_n = T;
        float ms[2] = {0.f, 0.f};
        if (hipMemcpy(ctx->d_err, &zero_err, sizeof(uint32_t), hipMemcpyHostToDevice) != hipSuccess)
            st = fail(LW_E_HIP, "tuner error word");
        for (int r = 0; r < 2 && st == LW_OK; ++r) {
            const int64_t n_steps = 256 << r;
            o.out_stride = n_steps;
            if (hipEventRecord(ev[0], s) != hipSuccess) st = fail(LW_E_HIP, "tuner timing");
            if (st == LW_OK)
                st = dipole_run_impl(ctx, h_dip, n_dip, h_inst_off, n_inst, dt, n_steps, &o, ctx->d_trial, nullptr,
                                     nullptr, nullptr, nullptr, nullptr, nullptr, 0, false, (void *)s);
            if (st == LW_OK && (hipEventRecord(ev[1], s) != hipSuccess || hipEventSynchronize(ev[1]) != hipSuccess ||
                                hipEventElapsedTime(&ms[r], ev[0], ev[1]) != hipSuccess))
                st = fail(LW_E_HIP, "tuner timing");
        }
        if (st != LW_OK) break;
        uint32_t trial_err = 0;
        if (hipMemcpy(&trial_err, ctx->d_err, sizeof(uint32_t), hipMemcpyDeviceToHost) != hipSuccess) {
            st = fail(LW_E_HIP, "tuner error word");
            break;
        }
        if (trial_err) continue;                 // this threshold's trials did not run clean
        const float per_step = (ms[1] - ms[0]) / 256.0f;
        if (per_step < best) {
            best = per_step;
            *out = T;
        }
    }
    for (auto &e : ev) (void)hipEventDestroy(e);
    if (hipMemcpy(ctx->d_err, &saved_err, sizeof(uint32_t), hipMemcpyHostToDevice) != hipSuccess && st == LW_OK)
        st = fail(LW_E_HIP, "tuner error word");
    if (st != LW_OK) return st;
    // no candidate ran clean: keep the default and do not cache a choice
    if (best == 1e30f) {
        *out = 16;
        return LW_OK;
    }
    ctx->tuned_dip[key] = *out;
    save_tune_dip(ctx, key, *out);
    return LW_OK;
}

static lw_status dipole_run_impl(lw_ctx *ctx, const lw_dipole *h_dip, int32_t n_dip, const int32_t *h_inst_off,
                                 int32_t n_inst, double dt, int64_t steps, const lw_run_opts *opts,
                                 double *d_moment, double *d_dot, double *d_energy, double *d_drive, double *d_wabs,
                                 double *d_wrad, double *d_state, int64_t n_state, bool resume, void *stream)
{
    if (!ctx || !opts || !h_dip || !h_inst_off || !d_moment) return fail(LW_E_INVALID, "lw_dipole_run: null argument");
    int ring = 0;
    lw_status gst = run_geometry("lw_dipole_run", h_dip, n_dip, h_inst_off, n_inst, dt, steps, opts, &ring);
    if (gst != LW_OK) return gst;
    if (resume && !d_state) return fail(LW_E_INVALID, "lw_dipole_run: resume needs a run state");
    if (d_state && n_state < lw::state_doubles(n_dip, ring))
        return fail(LW_E_INVALID, "lw_dipole_run: the run state holds " + std::to_string(n_state) + " doubles, " +
                                      std::to_string(lw::state_doubles(n_dip, ring)) + " are needed");
    if (steps == 0 && !d_moment) return LW_OK;
    LW_HIP(hipSetDevice(ctx->device));
    hipStream_t s = (hipStream_t)stream;

    // small instances whose ring fits in LDS run whole in one workgroup each;
    // the others advance one launch per step with one workgroup per dipole
    const int lds_limit = 64 * 1024;
    int stepped_min = opts->stepped_min_n == 0 ? 16 : (opts->stepped_min_n < 0 ? (1 << 30) : opts->stepped_min_n);
    if (opts->stepped_min_n == LW_STEPPED_TUNE) {
        const lw_status tst = tune_stepped(ctx, h_dip, n_dip, h_inst_off, n_inst, dt, opts, ring, s, &stepped_min);
        if (tst != LW_OK) return tst;
    }
    std::vector<int32_t> lds_list, tgt, tgt_lo, tgt_n;
    std::vector<int64_t> tgt_base;
    int max_lds_n = 0;
    int64_t ring_doubles = 0;
    for (int k = 0; k < n_inst; ++k) {
        const int a0 = h_inst_off[k], n = h_inst_off[k + 1] - a0;
        if (n == 0) continue;
        if (n < stepped_min && lw::ring_lds_bytes(n, ring) <= lds_limit) {
            lds_list.push_back(k);
            max_lds_n = std::max(max_lds_n, n);
        } else {
            // a run state keeps every instance's ring at its place in the state
            const int64_t base = d_state ? lw::state_ring_off(a0, ring) - lw::STATE_HEAD : ring_doubles;
            for (int i = 0; i < n; ++i) {
                tgt.push_back(a0 + i);
                tgt_lo.push_back(a0);
                tgt_n.push_back(n);
                tgt_base.push_back(base);
            }
            ring_doubles += (int64_t)n * ring * 3;
        }
    }
    // largest instances first: their workgroups (n - 1 sources each) start in the
    // first waves of the dispatch and the small ones fill in behind them, which
    // shortens the step's tail; each instance's targets stay contiguous
    {
        std::vector<size_t> ord(tgt.size());
        for (size_t q = 0; q < ord.size(); ++q) ord[q] = q;
        std::stable_sort(ord.begin(), ord.end(), [&](size_t x, size_t y) { return tgt_n[x] > tgt_n[y]; });
        auto permute = [&](auto &v) {
            auto w = v;
            for (size_t q = 0; q < ord.size(); ++q) w[q] = v[ord[q]];
            v.swap(w);
        };
        permute(tgt);
        permute(tgt_lo);
        permute(tgt_n);
        permute(tgt_base);
    }
    const size_t n_tgt = tgt.size();

    const size_t in_bytes = align_up(sizeof(lw_dipole) * (size_t)n_dip, 256);
    const size_t off_bytes = align_up(sizeof(int32_t) * (size_t)(n_inst + 1), 256);
    const size_t list_bytes = align_up(sizeof(int32_t) * (lds_list.size() + 1), 256);
    const size_t t32_bytes = align_up(sizeof(int32_t) * (n_tgt + 1), 256);
    const size_t t64_bytes = align_up(sizeof(int64_t) * (n_tgt + 1), 256);
    const size_t stage_bytes = in_bytes + off_bytes + list_bytes + 3 * t32_bytes + t64_bytes;
    const size_t dev_bytes = align_up(lw::dip_dev_bytes(n_dip), 256);
    const size_t ecur_bytes = align_up(sizeof(double) * 3 * (size_t)n_dip, 256);   // E_d(t_n), then 2 energy sums
    const size_t step_bytes = 256;
    const size_t ring_bytes = d_state ? 256 : align_up(sizeof(double) * (size_t)std::max<int64_t>(ring_doubles, 1), 256);
    lw_status st = ensure_work(ctx, stage_bytes + dev_bytes + ecur_bytes + step_bytes + ring_bytes, s);
    if (st != LW_OK) return st;
    // the previous stepped run's graph is released once the stream has passed it
    if (ctx->graph_exec || ctx->graph) {
        LW_HIP(hipEventSynchronize(ctx->graph_done));
        if (ctx->graph_exec) (void)hipGraphExecDestroy(ctx->graph_exec);
        if (ctx->graph) (void)hipGraphDestroy(ctx->graph);
        ctx->graph_exec = nullptr;
        ctx->graph = nullptr;
    }
    st = acquire_stage(ctx, stage_bytes);
    if (st != LW_OK) return st;
    char *stage = (char *)ctx->h_stage;
    size_t o = 0;
    std::memcpy(stage + o, h_dip, sizeof(lw_dipole) * (size_t)n_dip);
    o += in_bytes;
    std::memcpy(stage + o, h_inst_off, sizeof(int32_t) * (size_t)(n_inst + 1));
    o += off_bytes;
    std::copy(lds_list.begin(), lds_list.end(), (int32_t *)(stage + o));
    o += list_bytes;
    std::copy(tgt.begin(), tgt.end(), (int32_t *)(stage + o));
    o += t32_bytes;
    std::copy(tgt_lo.begin(), tgt_lo.end(), (int32_t *)(stage + o));
    o += t32_bytes;
    std::copy(tgt_n.begin(), tgt_n.end(), (int32_t *)(stage + o));
    o += t32_bytes;
    std::copy(tgt_base.begin(), tgt_base.end(), (int64_t *)(stage + o));
    char *work = (char *)ctx->d_work;
    st = upload(ctx, work, stage_bytes, s);
    if (st != LW_OK) return st;
    o = 0;
    const lw_dipole *d_in = (const lw_dipole *)(work + o);
    o += in_bytes;
    const int32_t *d_off = (const int32_t *)(work + o);
    o += off_bytes;
    const int32_t *d_list = (const int32_t *)(work + o);
    o += list_bytes;
    const int32_t *d_tgt = (const int32_t *)(work + o);
    o += t32_bytes;
    const int32_t *d_tgt_lo = (const int32_t *)(work + o);
    o += t32_bytes;
    const int32_t *d_tgt_n = (const int32_t *)(work + o);
    o += t32_bytes;
    const int64_t *d_tgt_base = (const int64_t *)(work + o);
    o += t64_bytes;
    lw::DipDev *d_dev = (lw::DipDev *)(work + o);
    o += dev_bytes;
    double *d_Ecur = (double *)(work + o);
    double *d_W = d_Ecur + n_dip;
    o += ecur_bytes;
    int64_t *d_step = (int64_t *)(work + o);
    o += step_bytes;
    double *d_ring = (double *)(work + o);
    if (d_state) {
        // the stepped path works in the run state itself
        d_ring = d_state + lw::STATE_HEAD;
        d_Ecur = d_state + lw::state_ecur_off(n_dip, ring);
        d_W = d_state + lw::state_w_off(n_dip, ring);
    }

    const double max_vel = opts->max_vel > 0.0 ? opts->max_vel : C_LIGHT / 100.0;
    const int max_iter = 60;
    LW_HIP(lw::launch_dipole_prep(d_in, n_dip, d_dev, s));
    const lw::RunOut out{d_moment, d_dot, d_energy, d_drive, d_wabs, d_wrad, opts->out_stride, n_dip};
    // a resumed run's row 0 comes from its state, before either path updates it
    if (resume) LW_HIP(lw::launch_state_rows(d_dev, d_off, n_inst, d_state, ring, out, ctx->d_err, s));
    const bool both = !lds_list.empty() && n_tgt > 0;
    hipStream_t small_s = s;
    if (both) {
        if (!ctx->side) LW_HIP(hipStreamCreateWithFlags(&ctx->side, hipStreamNonBlocking));
        if (!ctx->join_a) LW_HIP(hipEventCreateWithFlags(&ctx->join_a, hipEventDisableTiming));
        if (!ctx->join_b) LW_HIP(hipEventCreateWithFlags(&ctx->join_b, hipEventDisableTiming));
        LW_HIP(hipEventRecord(ctx->join_a, s));
        LW_HIP(hipStreamWaitEvent(ctx->side, ctx->join_a, 0));
        small_s = ctx->side;
    }
    bool moving = false;
    for (int i = 0; i < n_dip; ++i) moving = moving || motion_reach(h_dip[i]) > 0.0;
    const bool mixed = opts->precision == LW_MIXED;
    LW_HIP(lw::launch_dipole_instances(d_dev, d_off, d_list, (int)lds_list.size(), max_lds_n, true, nullptr, nullptr,
                                       ring, steps, dt, max_vel, max_iter, out, moving, mixed, d_state, resume,
                                       ctx->d_err, small_s));
    if (n_tgt > 0) {
        if (!ctx->capture) LW_HIP(hipStreamCreateWithFlags(&ctx->capture, hipStreamNonBlocking));
        if (!ctx->graph_done) LW_HIP(hipEventCreateWithFlags(&ctx->graph_done, hipEventDisableTiming));
        const int chunk = 256;
        LW_HIP(lw::launch_dipole_steps(d_dev, d_tgt, d_tgt_lo, d_tgt_n, d_tgt_base, (int)n_tgt, d_ring, d_Ecur, d_W,
                                       d_step, ring, steps, dt, max_vel, max_iter, out, moving, mixed,
                                       resume ? d_state : nullptr, ctx->d_err, chunk, s, ctx->capture, &ctx->graph,
                                       &ctx->graph_exec));
        LW_HIP(hipEventRecord(ctx->graph_done, s));
    }
    if (both) {
        LW_HIP(hipEventRecord(ctx->join_b, ctx->side));
        LW_HIP(hipStreamWaitEvent(s, ctx->join_b, 0));
    }
    if (d_state) LW_HIP(lw::launch_state_header(d_state, ring, n_dip, steps, resume, s));
    return LW_OK;
}

lw_status lw_dipole_run(lw_ctx *ctx, const lw_dipole *h_dip, int32_t n_dip, const int32_t *h_inst_off,
                        int32_t n_inst, double dt, int64_t steps, const lw_run_opts *opts, double *d_moment,
                        double *d_dot, double *d_energy, double *d_drive, double *d_wabs, double *d_wrad,
                        double *h_gamma, double *h_domega, void *stream)
{
    lw_status st = dipole_run_impl(ctx, h_dip, n_dip, h_inst_off, n_inst, dt, steps, opts, d_moment, d_dot, d_energy,
                                   d_drive, d_wabs, d_wrad, nullptr, 0, false, stream);
    if (st != LW_OK || (!h_gamma && !h_domega)) return st;
    // collective rates and shift of the two-dipole instances (Sec. 2.4): wait for
    // the run (its latched errors are returned first), copy the moments back and
    // fit the normal modes after the transient of each pair
    st = lw_sync_status(ctx, stream);
    if (st != LW_OK) return st;
    const int64_t stride = opts->out_stride;
    const int64_t rows = steps / stride + 1;
    std::vector<double> mom((size_t)rows * (size_t)n_dip);
    LW_HIP(hipMemcpy(mom.data(), d_moment, sizeof(double) * mom.size(), hipMemcpyDeviceToHost));
    std::vector<double> w_ref((size_t)n_inst), modes(5 * (size_t)n_inst);
    std::vector<int64_t> skip((size_t)n_inst, 0);
    for (int k = 0; k < n_inst; ++k) {
        const int a = h_inst_off[k];
        w_ref[k] = h_inst_off[k + 1] > a ? h_dip[a].omega0 : 1.0;
        if (h_inst_off[k + 1] - a != 2) continue;
        double d[3];
        for (int i = 0; i < 3; ++i) d[i] = h_dip[a + 1].origin[i] - h_dip[a].origin[i];
        skip[k] = std::max<int64_t>(2000, (int64_t)std::ceil(3.0 * norm3(d) / (C_LIGHT * dt)));
    }
    st = lw_pair_modes(mom.data(), rows, n_dip, h_inst_off, n_inst, dt, stride, w_ref.data(), skip.data(),
                       modes.data());
    if (st != LW_OK) return st;
    for (int k = 0; k < n_inst; ++k) {
        if (h_gamma) {
            h_gamma[2 * k] = modes[5 * k];
            h_gamma[2 * k + 1] = modes[5 * k + 1];
        }
        if (h_domega) h_domega[k] = modes[5 * k + 4];
    }
    return LW_OK;
}

lw_status lw_dipole_run_state(lw_ctx *ctx, const lw_dipole *h_dip, int32_t n_dip, const int32_t *h_inst_off,
                              int32_t n_inst, double dt, int64_t steps, const lw_run_opts *opts, double *d_moment,
                              double *d_dot, double *d_energy, double *d_drive, double *d_wabs, double *d_wrad,
                              double *d_state, int64_t n_state, int32_t resume, void *stream)
{
    if (!d_state) return fail(LW_E_INVALID, "lw_dipole_run_state: null run state");
    return dipole_run_impl(ctx, h_dip, n_dip, h_inst_off, n_inst, dt, steps, opts, d_moment, d_dot, d_energy, d_drive,
                           d_wabs, d_wrad, d_state, n_state, resume != 0, stream);
}

lw_status lw_dipole_state_size(const lw_dipole *h_dip, int32_t n_dip, const int32_t *h_inst_off, int32_t n_inst,
                               double dt, const lw_run_opts *opts, int64_t *n_doubles)
{
    if (!n_doubles) return fail(LW_E_INVALID, "lw_dipole_state_size: null output");
    int ring = 0;
    const lw_status st = run_geometry("lw_dipole_state_size", h_dip, n_dip, h_inst_off, n_inst, dt, 0, opts, &ring);
    if (st != LW_OK) return st;
    *n_doubles = lw::state_doubles(n_dip, ring);
    return LW_OK;
}

// The backward sweep of the oscillator adjoint, over segments of K steps from
// the last to the first.  Sweeping a segment needs its history window (the
// segment and the look-back before it) and the reverse of the detector
// snapshots whose newest sample lies in it.  A side stream prepares the next
// (earlier) segment while the caller's stream sweeps the current one, so the
// latency-bound backward steps (a few workgroups per launch) overlap with the
// detector reverse and, when checkpointed, with the segment's recomputation.
//
// whole = true: the forward run stores every step, the history ring holds the
// whole run, and every snapshot is reversed in one launch before the sweep.
//
// whole = false (checkpointing): the forward pass keeps a run state every K
// steps; preparing a segment runs it again from its state with every step
// stored and copies the state's ring and the new rows into the history ring,
// which holds two windows (the one being swept and the one being prepared,
// 2K + depth steps).  Each sample is written once, by the latest window that
// holds it, so the preparation never rewrites a sample the sweep reads; the
// preparation of window g - 1 starts only once the sweep of window g + 1 has
// ended, whose ring slots it reuses.  Detector cotangents of window g - 1 go
// to samples the sweep of window g neither reads nor clears.
static lw_status vjp_pipelined(lw_ctx *ctx, const lw_dipole *h_dip, int32_t n_dip, const int32_t *h_inst_off,
                               int32_t n_inst, double dt, int64_t steps, const lw_run_opts *opts,
                               const double *d_det_pts, int64_t n_det, const double *h_snap_times, int32_t n_snap,
                               bool whole, int64_t K, double *d_grad_pos, double *h_J, void *stream)
{
    hipStream_t s = (hipStream_t)stream;
    int ring_geo = 0;
    lw_status st = run_geometry("lw_dipole_run_vjp", h_dip, n_dip, h_inst_off, n_inst, dt, steps, opts, &ring_geo);
    if (st != LW_OK) return st;
    int ring_fwd = ring_geo;
    int64_t ring_h = 1;
    if (whole) {
        while (ring_h < steps + 1) ring_h <<= 1;
        if (ring_h > (1 << 26)) return fail(LW_E_INVALID, "lw_dipole_run_vjp: run too long for the stored history");
    } else {
        // the detector's look-back: an upper bound on the light time from a
        // detector point to an origin (the farthest corner of the points'
        // bounding box), doubled and padded as for the drive pairs
        std::vector<double> P((size_t)(3 * n_det));
        LW_HIP(hipMemcpyAsync(P.data(), d_det_pts, sizeof(double) * P.size(), hipMemcpyDeviceToHost, s));
        LW_HIP(hipStreamSynchronize(s));
        double lo[3], hi[3];
        for (int c = 0; c < 3; ++c) {
            const double *x = P.data() + c * n_det;
            lo[c] = *std::min_element(x, x + n_det);
            hi[c] = *std::max_element(x, x + n_det);
            if (!std::isfinite(lo[c]) || !std::isfinite(hi[c]))
                return fail(LW_E_INVALID, "lw_dipole_run_vjp: detector points must be finite");
        }
        double reach2 = 0.0;
        for (int i = 0; i < n_dip; ++i) {
            double r2 = 0.0;
            for (int c = 0; c < 3; ++c) {
                const double e = std::max(std::fabs(lo[c] - h_dip[i].origin[c]), std::fabs(hi[c] - h_dip[i].origin[c]));
                r2 += e * e;
            }
            reach2 = std::max(reach2, r2);
        }
        const double w_det = std::ceil(2.0 * std::sqrt(reach2) / C_LIGHT / dt) + 3.0;
        if (!(w_det < (double)(1 << 24))) return fail(LW_E_INVALID, "lw_dipole_run_vjp: detector too far for dt");
        ring_fwd = 4;
        while (ring_fwd < std::max<int64_t>(ring_geo, (int64_t)w_det + 6)) ring_fwd <<= 1;
        ring_h = 4;
        while (ring_h < 2 * K + ring_fwd + 4) ring_h <<= 1;
        if (ring_h > (1 << 26)) return fail(LW_E_INVALID, "lw_dipole_run_vjp: checkpoint interval too long");
    }
    const int64_t n_seg = (steps + K - 1) / K;
    const int64_t sd = whole ? 0 : lw::state_doubles(n_dip, ring_fwd);
    const int64_t out_rows = whole ? steps + 1 : K + 1;
    // drive pairs per step (2 stages x n targets x (n-1) sources x 2 charges) and of E_d(0)
    std::vector<int64_t> pair_off(n_inst + 1, 0), pair_off0(n_inst + 1, 0);
    for (int k = 0; k < n_inst; ++k) {
        const int64_t n = h_inst_off[k + 1] - h_inst_off[k];
        pair_off[k + 1] = pair_off[k] + 4 * n * (n - 1);
        pair_off0[k + 1] = pair_off0[k] + 2 * n * (n - 1);
    }
    const int64_t n_pairs = pair_off[n_inst], n_pairs0 = pair_off0[n_inst];
    // snapshots by segment: snapshot k is reversed before the step that consumes
    // its newest sample, min(floor(t_k / dt), steps - 1); sorted latest first,
    // the snapshots of one segment are contiguous
    std::vector<int64_t> due(n_snap);
    std::vector<int> order(n_snap);
    for (int k = 0; k < n_snap; ++k) {
        due[k] = std::min<int64_t>((int64_t)std::floor(h_snap_times[k] / dt), steps - 1);
        order[k] = k;
    }
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return due[x] > due[y]; });
    std::vector<int> snap_end(n_seg + 1, 0);      // sorted snapshots of segment g: [snap_end[g+1], snap_end[g])
    for (int r = 0; r < n_snap; ++r) snap_end[due[order[r]] / K] = r + 1;
    for (int64_t g = n_seg - 1; g >= 0; --g) snap_end[g] = std::max(snap_end[g], snap_end[g + 1]);
    // with the whole history every snapshot can be reversed at once, before the
    // sweep: one launch wide enough to fill the chip
    if (whole)
        for (int64_t g = 0; g < n_seg; ++g) snap_end[g] = n_snap;
    int64_t n_jpart = 0;                           // J partials: one per 256 lanes of each segment's launch
    for (int64_t g = 0; g < n_seg; ++g) n_jpart += (n_det * (snap_end[g] - snap_end[g + 1]) + 255) / 256;
    const size_t ck_b = align_up(sizeof(double) * (size_t)(sd * n_seg + 1), 256);
    const size_t ws_b = align_up(sizeof(double) * (size_t)(sd + 1), 256);
    const size_t out_b = align_up(sizeof(double) * (size_t)(out_rows * n_dip), 256);
    const size_t hist_b = align_up(sizeof(double) * (size_t)(ring_h * n_dip * 3), 256);
    const size_t jp_b = align_up(sizeof(double) * (size_t)(n_jpart + 1), 256);
    const size_t dip_b = align_up(sizeof(lw_dipole) * (size_t)n_dip, 256);
    const size_t off_b = align_up(sizeof(int32_t) * (size_t)(n_inst + 1), 256);
    const size_t po_b = align_up(sizeof(int64_t) * (size_t)(n_inst + 1), 256);
    const size_t tm_b = align_up(sizeof(double) * (size_t)n_snap, 256);
    const size_t dev_b = align_up(lw::dip_dev_bytes(n_dip), 256);
    const size_t adj_b = align_up(sizeof(double) * 8 * (size_t)n_dip, 256);   // two cotangent states
    const size_t rbp_b = align_up(sizeof(double) * 3 * (size_t)std::max<int64_t>(n_pairs, 1), 256);
    const size_t rbp0_b = align_up(sizeof(double) * 3 * (size_t)std::max<int64_t>(n_pairs0, 1), 256);
    const size_t taup_b = align_up(sizeof(double) * (size_t)std::max<int64_t>(n_pairs, 1), 256);
    const size_t stage_b = dip_b + off_b + 2 * po_b + tm_b;
    st = ensure_work2(ctx, ck_b + ws_b + 3 * out_b + 2 * hist_b + jp_b + 256 + stage_b + dev_b + adj_b + rbp_b +
                               rbp0_b + taup_b + 256, s);
    if (st != LW_OK) return st;
    char *w2 = (char *)ctx->d_work2;
    size_t o = 0;
    auto take = [&](size_t bytes) { char *p = w2 + o; o += bytes; return p; };
    double *d_ckpt = (double *)take(ck_b);
    double *d_ws = (double *)take(ws_b);
    double *d_D = (double *)take(out_b);
    double *d_V = (double *)take(out_b);
    double *d_Ed = (double *)take(out_b);
    double *d_hist = (double *)take(hist_b);
    double *d_hbar = (double *)take(hist_b);
    double *d_Jpart = (double *)take(jp_b);
    double *d_J = (double *)take(256);
    char *stage_dev = take(stage_b);
    lw::DipDev *d_dev = (lw::DipDev *)take(dev_b);
    double *d_adj = (double *)take(adj_b);
    double *d_rbp = (double *)take(rbp_b);
    double *d_rbp0 = (double *)take(rbp0_b);
    double *d_taup = (double *)take(taup_b);
    int64_t *d_step = (int64_t *)take(256);
    // records, offsets, pair offsets and the sorted snapshot times
    st = acquire_stage(ctx, stage_b);
    if (st != LW_OK) return st;
    char *stage = (char *)ctx->h_stage;
    std::memcpy(stage, h_dip, sizeof(lw_dipole) * (size_t)n_dip);
    std::memcpy(stage + dip_b, h_inst_off, sizeof(int32_t) * (size_t)(n_inst + 1));
    std::memcpy(stage + dip_b + off_b, pair_off.data(), sizeof(int64_t) * (size_t)(n_inst + 1));
    std::memcpy(stage + dip_b + off_b + po_b, pair_off0.data(), sizeof(int64_t) * (size_t)(n_inst + 1));
    double *st_times = (double *)(stage + dip_b + off_b + 2 * po_b);
    for (int r = 0; r < n_snap; ++r) st_times[r] = h_snap_times[order[r]];
    st = upload(ctx, stage_dev, stage_b, s);
    if (st != LW_OK) return st;
    const lw_dipole *d_in = (const lw_dipole *)stage_dev;
    const int32_t *d_off = (const int32_t *)(stage_dev + dip_b);
    const int64_t *d_pair_off = (const int64_t *)(stage_dev + dip_b + off_b);
    const int64_t *d_pair_off0 = (const int64_t *)(stage_dev + dip_b + off_b + po_b);
    const double *d_times = (const double *)(stage_dev + dip_b + off_b + 2 * po_b);
    LW_HIP(lw::launch_dipole_prep(d_in, n_dip, d_dev, s));
    lw_run_opts fo = *opts;
    if (whole) {
        // forward run with every step stored, then the whole history
        fo.out_stride = 1;
        st = lw_dipole_run(ctx, h_dip, n_dip, h_inst_off, n_inst, dt, steps, &fo, d_D, d_V, nullptr, d_Ed, nullptr,
                           nullptr, nullptr, nullptr, stream);
        if (st != LW_OK) return st;
        LW_HIP(lw::launch_hist_rows(d_dev, d_D, d_V, d_Ed, n_dip, steps + 1, 0, (int)ring_h, d_hist, s));
    } else {
        // forward pass: a run state every K steps (outputs: two rows per segment, discarded)
        fo.ring_depth = ring_fwd;
        for (int64_t g = 0; g < n_seg; ++g) {
            const int64_t a = g * K, ks = std::min(K, steps - a);
            if (g > 0)
                LW_HIP(hipMemcpyAsync(d_ckpt + g * sd, d_ws, sizeof(double) * sd, hipMemcpyDeviceToDevice, s));
            fo.out_stride = ks;
            st = lw_dipole_run_state(ctx, h_dip, n_dip, h_inst_off, n_inst, dt, ks, &fo, d_D, nullptr, nullptr,
                                     nullptr, nullptr, nullptr, d_ws, sd, g > 0 ? 1 : 0, stream);
            if (st != LW_OK) return st;
        }
        fo.out_stride = 1;
    }
    LW_HIP(lw::launch_vjp_begin(n_dip, n_pairs, steps, d_hbar, ring_h * n_dip * 3, d_grad_pos, d_rbp, d_taup, d_adj,
                                d_step, s));
    if (!ctx->adj_side) LW_HIP(hipStreamCreateWithFlags(&ctx->adj_side, hipStreamNonBlocking));
    if (!ctx->adj_built) LW_HIP(hipEventCreateWithFlags(&ctx->adj_built, hipEventDisableTiming));
    if (!ctx->adj_swept) LW_HIP(hipEventCreateWithFlags(&ctx->adj_swept, hipEventDisableTiming));
    hipStream_t t = ctx->adj_side;
    // segment g on the side stream: (checkpointed) the segment run again with
    // every step stored and the samples only this window holds; then the
    // reverse of its snapshots
    int64_t jp_next = 0;
    auto prepare = [&](int64_t g) -> lw_status {
        const int64_t a = g * K, ks = std::min(K, steps - a);
        if (!whole) {
            const int64_t top = g + 1 < n_seg ? a + K - ring_fwd : a + ks;   // newest sample written here
            if (top >= a) {      // (with K below the look-back, later windows hold every row)
                if (g > 0)
                    LW_HIP(hipMemcpyAsync(d_ws, d_ckpt + g * sd, sizeof(double) * sd, hipMemcpyDeviceToDevice, t));
                const lw_status r = lw_dipole_run_state(ctx, h_dip, n_dip, h_inst_off, n_inst, dt, ks, &fo, d_D, d_V,
                                                        nullptr, d_Ed, nullptr, nullptr, d_ws, sd, g > 0 ? 1 : 0, t);
                if (r != LW_OK) return r;
                LW_HIP(lw::launch_hist_rows(d_dev, d_D, d_V, d_Ed, n_dip, std::min(ks, top - a) + 1, a, (int)ring_h,
                                            d_hist, t));
            }
            if (g > 0)
                LW_HIP(lw::launch_hist_from_state(d_ckpt + g * sd, d_off, n_inst, n_dip, ring_fwd,
                                                  std::max<int64_t>(a - ring_fwd + 1, 0), std::min(a - 1, top),
                                                  (int)ring_h, d_hist, t));
        }
        const int r0 = snap_end[g + 1], cnt = snap_end[g] - r0;
        if (cnt > 0) {
            // the window's newest sample bounds what the snapshots read
            LW_HIP(lw::launch_vjp_detector(d_dev, n_dip, d_hist, d_hbar, (int)ring_h, a + ks, dt, d_det_pts, n_det,
                                           d_times + r0, cnt, n_snap, d_grad_pos, d_Jpart + jp_next, ctx->d_err, t));
            jp_next += (n_det * cnt + 255) / 256;
        }
        LW_HIP(hipEventRecord(ctx->adj_built, t));
        return LW_OK;
    };
    // backward steps replay a captured chunk of C launches (each chunk moves the
    // device step base by C): C divides K where a divisor in [16, 64] exists
    int64_t C = 32;
    for (int64_t c = 64; c >= 16; --c)
        if (K % c == 0) {
            C = c;
            break;
        }
    struct StepGraph {           // released once the stream has passed it, on every way out
        hipStream_t s;
        hipGraph_t graph = nullptr;
        hipGraphExec_t exec = nullptr;
        ~StepGraph()
        {
            if (exec) {
                (void)hipStreamSynchronize(s);
                (void)hipGraphExecDestroy(exec);
            }
            if (graph) (void)hipGraphDestroy(graph);
        }
    } sg{s};
    if (!ctx->capture) LW_HIP(hipStreamCreateWithFlags(&ctx->capture, hipStreamNonBlocking));
    if (K >= C) {
        LW_HIP(hipStreamBeginCapture(ctx->capture, hipStreamCaptureModeThreadLocal));
        const hipError_t ce = lw::launch_vjp_steps(d_dev, d_off, d_pair_off, n_inst, n_dip, d_hist, d_hbar,
                                                   (int)ring_h, dt, d_adj, d_rbp, d_taup, d_step, C, steps,
                                                   ctx->d_err, ctx->capture);
        const hipError_t ee = hipStreamEndCapture(ctx->capture, &sg.graph);
        LW_HIP(ce);
        LW_HIP(ee);
        LW_HIP(hipGraphInstantiate(&sg.exec, sg.graph, nullptr, nullptr, 0));
    }
    // on failure both streams are drained before returning (the graph is
    // released on the way out)
    auto bail = [&](lw_status r) {
        (void)hipStreamSynchronize(t);
        (void)hipStreamSynchronize(s);
        return r;
    };
    LW_HIP(hipEventRecord(ctx->adj_swept, s));
    LW_HIP(hipStreamWaitEvent(t, ctx->adj_swept, 0));
    st = prepare(n_seg - 1);
    if (st != LW_OK) return bail(st);
    for (int64_t g = n_seg - 1; g >= 0; --g) {
        const int64_t a = g * K, ks = std::min(K, steps - a);
        if (hipStreamWaitEvent(s, ctx->adj_built, 0) != hipSuccess) return bail(fail(LW_E_HIP, "hipStreamWaitEvent"));
        if (g > 0) {
            st = prepare(g - 1);
            if (st != LW_OK) return bail(st);
        }
        // backward steps a + ks - 1 .. a
        const int64_t reps = sg.exec ? ks / C : 0;
        for (int64_t r = 0; r < reps; ++r)
            if (hipGraphLaunch(sg.exec, s) != hipSuccess) return bail(fail(LW_E_HIP, "backward steps"));
        if (lw::launch_vjp_steps(d_dev, d_off, d_pair_off, n_inst, n_dip, d_hist, d_hbar, (int)ring_h, dt, d_adj,
                                 d_rbp, d_taup, d_step, ks - reps * C, steps, ctx->d_err, s) != hipSuccess)
            return bail(fail(LW_E_HIP, "backward steps"));
        if (hipEventRecord(ctx->adj_swept, s) != hipSuccess || hipStreamWaitEvent(t, ctx->adj_swept, 0) != hipSuccess)
            return bail(fail(LW_E_HIP, "hipEventRecord"));
    }
    LW_HIP(lw::launch_vjp_end(d_dev, d_off, d_pair_off, d_pair_off0, n_inst, n_pairs0, n_dip, d_hist, d_hbar,
                              (int)ring_h, dt, d_adj, d_rbp, d_rbp0, d_grad_pos, d_Jpart, jp_next, d_J, ctx->d_err,
                              s));
    double J = 0.0;
    LW_HIP(hipMemcpyAsync(&J, d_J, sizeof(double), hipMemcpyDeviceToHost, s));
    st = lw_sync_status(ctx, stream);
    *h_J = J;
    return st;
}

lw_status lw_dipole_run_vjp(lw_ctx *ctx, const lw_dipole *h_dip, int32_t n_dip, const int32_t *h_inst_off,
                            int32_t n_inst, double dt, int64_t steps, const lw_run_opts *opts, const double *d_det_pts,
                            int64_t n_det, const double *h_snap_times, int32_t n_snap, int32_t ckpt_every,
                            double *d_grad_pos, double *h_J, void *stream)
{
    if (!ctx || !opts || !h_dip || !h_inst_off || !d_det_pts || !h_snap_times || !d_grad_pos || !h_J)
        return fail(LW_E_INVALID, "lw_dipole_run_vjp: null argument");
    if (n_det < 1 || n_snap < 1 || n_dip < 1 || n_inst < 1 || steps < 1)
        return fail(LW_E_INVALID, "lw_dipole_run_vjp: empty detector, snapshots, dipoles or run");
    for (int k = 0; k < n_snap; ++k)
        if (!(h_snap_times[k] >= 0.0 && h_snap_times[k] <= (double)steps * dt))
            return fail(LW_E_INVALID, "lw_dipole_run_vjp: snapshot times must lie in [0, steps dt]");
    int max_n = 0;
    for (int k = 0; k < n_inst; ++k) max_n = std::max(max_n, h_inst_off[k + 1] - h_inst_off[k]);
    if (max_n > 1024) return fail(LW_E_INVALID, "lw_dipole_run_vjp: instances of more than 1024 dipoles");
    if (opts->precision != LW_FP64) return fail(LW_E_INVALID, "lw_dipole_run_vjp: the oscillator adjoint is FP64 only");
    for (int i = 0; i < n_dip; ++i)
        if (motion_reach(h_dip[i]) > 0.0)
            return fail(LW_E_INVALID, "lw_dipole_run_vjp: moving dipoles have no adjoint here");
    if (n_det * (int64_t)n_snap > ((int64_t)1 << 36)) return fail(LW_E_INVALID, "lw_dipole_run_vjp: detector too large");
    if (ckpt_every < 0) return fail(LW_E_INVALID, "lw_dipole_run_vjp: negative checkpoint interval");
    LW_HIP(hipSetDevice(ctx->device));
    // without checkpoints the sweep is still taken in segments, so that the
    // detector reverse of earlier snapshots overlaps with the later steps
    const bool whole = ckpt_every == 0 || ckpt_every >= steps;
    const int64_t K = whole ? std::max<int64_t>(256, ((steps + 15) / 16 + 63) / 64 * 64) : ckpt_every;
    return vjp_pipelined(ctx, h_dip, n_dip, h_inst_off, n_inst, dt, steps, opts, d_det_pts, n_det, h_snap_times,
                         n_snap, whole, K, d_grad_pos, h_J, stream);
}

// ---------------------------------------------------------------------------
// host-side mode extraction (Sec. 2.4)
// ---------------------------------------------------------------------------

static void prony2(const std::vector<double> &x, int lag, double delta, double &gamma, double &omega)
{
    gamma = omega = NAN;
    const int64_t N = (int64_t)x.size();
    const int64_t L = lag;
    if (N < 2 * L + 2) return;
    // least squares for x[k+2L] = c1 x[k+L] + c0 x[k] via the 2x2 normal equations
    long double saa = 0, sab = 0, sbb = 0, say = 0, sby = 0;
    for (int64_t k = 0; k + 2 * L < N; ++k) {
        const long double a = x[k + L], b = x[k], y = x[k + 2 * L];
        saa += a * a;
        sab += a * b;
        sbb += b * b;
        say += a * y;
        sby += b * y;
    }
    const long double det = saa * sbb - sab * sab;
    if (!(det != 0)) return;
    const long double c1 = (say * sbb - sby * sab) / det;
    const long double c0 = (saa * sby - sab * say) / det;
    const long double disc = c1 * c1 + 4 * c0;
    if (!(disc < 0)) return;
    const long double r = std::sqrt(-c0);
    const long double th = std::atan2(std::sqrt(-disc) / 2, c1 / 2);
    gamma = (double)(-2.0L * std::log(r) / (L * (long double)delta));
    omega = (double)(th / (L * (long double)delta));
}

lw_status lw_pair_modes(const double *h_moment, int64_t n_rows, int32_t n_dip, const int32_t *h_inst_off,
                        int32_t n_inst, double dt, int64_t out_stride, const double *h_omega_ref,
                        const int64_t *h_skip_steps, double *h_out)
{
    if (!h_moment || !h_inst_off || !h_omega_ref || !h_skip_steps || !h_out || n_rows < 1 || n_dip < 1 ||
        n_inst < 1 || !(dt > 0.0) || out_stride < 1)
        return fail(LW_E_INVALID, "lw_pair_modes: bad argument");
    const double delta = dt * (double)out_stride;
    for (int k = 0; k < n_inst; ++k) {
        double *o = h_out + 5 * k;
        for (int q = 0; q < 5; ++q) o[q] = NAN;
        const int a = h_inst_off[k];
        if (h_inst_off[k + 1] - a != 2 || a < 0 || a + 1 >= n_dip) continue;
        const int64_t k0 = (h_skip_steps[k] + out_stride - 1) / out_stride;
        if (k0 >= n_rows) continue;
        std::vector<double> sp, am;
        sp.reserve(n_rows - k0);
        am.reserve(n_rows - k0);
        long double ss = 0, sa = 0;
        for (int64_t r = k0; r < n_rows; ++r) {
            const double d1 = h_moment[r * n_dip + a], d2 = h_moment[r * n_dip + a + 1];
            sp.push_back(d1 + d2);
            am.push_back(d1 - d2);
            ss += (long double)sp.back() * sp.back();
            sa += (long double)am.back() * am.back();
        }
        const double w0 = h_omega_ref[k];
        int lag = (int)std::lround(PI / (2.0 * w0 * delta));
        if (lag < 1) lag = 1;
        const double rs = std::sqrt((double)(ss / sp.size())), ra = std::sqrt((double)(sa / am.size()));
        if (rs > 1e-6 * ra) prony2(sp, lag, delta, o[0], o[2]);
        if (ra > 1e-6 * rs) prony2(am, lag, delta, o[1], o[3]);
        if (std::isfinite(o[2]) && std::isfinite(o[3])) o[4] = 0.5 * (o[2] - o[3]);
        else if (std::isfinite(o[2])) o[4] = o[2] - w0;
        else if (std::isfinite(o[3])) o[4] = w0 - o[3];
    }
    return LW_OK;
}

}  // extern "C"
