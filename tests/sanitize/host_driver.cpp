// Test driver for the host code of the HIP library under AddressSanitizer and
// UndefinedBehaviorSanitizer.
//
// Test infrastructure: built by tests/sanitize/build.py, with hipcc compiling the
// library's sources and this file into one executable and the sanitizers applied to
// the host pass only (the device code is built as usual and never launched here).  It
// runs on a machine without a GPU: it calls the entry points that work on the host
// alone (the Green's-function and normal-mode helpers, the two-dipole mode fit, the
// dipole run's argument and geometry checks) and the argument checks every other entry
// point makes before it touches a device.  Input arrays are read from raw files into
// allocations of exactly the file's size.
//
// Modes (files are raw native-endian arrays):
//   theory            lines on stdin: "gamma0 q m omega0", "gf R[3] p1[3] p2[3] omega0",
//                     "modes R[3] p[3] q m omega0"; prints status and outputs per line
//   pair_modes M N_DIP OFF DT STRIDE OMEGA_REF SKIP OUT
//                     lw_pair_modes on moments M ([rows][n_dip]), int32 offsets, FP64
//                     omega_ref and int64 skip per instance; writes OUT ([n_inst][5])
//   state_size DIP OFF DT PRECISION POLICY STRIDE MAX_VEL RING_DEPTH
//                     lw_dipole_state_size on lw_dipole records; prints status, size
//                     and the error message
//   null_ctx          every entry point that takes a context, called without one
//   create            lw_create on device 0 (on a machine without a GPU: its error
//                     path); destroys the context if one was made
#include <cinttypes>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <iostream>
#include <sstream>
#include <string>
#include <vector>

#include "lw.h"

namespace {

std::vector<unsigned char> slurp(const char *path)
{
    FILE *f = std::fopen(path, "rb");
    if (!f) {
        std::fprintf(stderr, "cannot open %s\n", path);
        std::exit(2);
    }
    std::fseek(f, 0, SEEK_END);
    const long n = std::ftell(f);
    std::fseek(f, 0, SEEK_SET);
    std::vector<unsigned char> buf((size_t)n);
    if (n > 0 && std::fread(buf.data(), 1, (size_t)n, f) != (size_t)n) {
        std::fprintf(stderr, "cannot read %s\n", path);
        std::exit(2);
    }
    std::fclose(f);
    return buf;
}

// exact-size heap copy of a file (a std::vector's capacity may exceed its size)
template <class T>
T *read_exact(const char *path, size_t *count)
{
    const std::vector<unsigned char> buf = slurp(path);
    *count = buf.size() / sizeof(T);
    T *p = static_cast<T *>(std::malloc(buf.size() > 0 ? buf.size() : 1));
    if (!p) std::exit(2);
    if (!buf.empty()) std::memcpy(p, buf.data(), buf.size());
    return p;
}

void print_status(const char *what, lw_status st)
{
    std::printf("%s %d %s\n", what, (int)st, st == LW_OK ? "" : lw_last_error());
}

int mode_theory()
{
    std::string line;
    while (std::getline(std::cin, line)) {
        std::istringstream in(line);
        std::string op;
        in >> op;
        if (op == "gamma0") {
            double q, m, w;
            in >> q >> m >> w;
            std::printf("gamma0 %.17g\n", lw_gamma0(q, m, w));
        } else if (op == "gf") {
            double R[3], p1[3], p2[3], w, out[2] = {0.0, 0.0};
            for (double &x : R) in >> x;
            for (double &x : p1) in >> x;
            for (double &x : p2) in >> x;
            in >> w;
            const lw_status st = lw_gf_pair(R, p1, p2, w, out);
            std::printf("gf %d %.17g %.17g\n", (int)st, out[0], out[1]);
        } else if (op == "modes") {
            double R[3], p[3], q, m, w, out[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
            for (double &x : R) in >> x;
            for (double &x : p) in >> x;
            in >> q >> m >> w;
            const lw_status st = lw_exact_modes(R, p, q, m, w, out);
            std::printf("modes %d %.17g %.17g %.17g %.17g %.17g\n", (int)st, out[0], out[1], out[2], out[3], out[4]);
        } else if (!op.empty()) {
            std::fprintf(stderr, "unknown theory line: %s\n", line.c_str());
            return 2;
        }
    }
    return 0;
}

int mode_pair_modes(char **a)
{
    size_t n_m, n_off, n_w, n_skip;
    double *m = read_exact<double>(a[0], &n_m);
    const int32_t n_dip = std::atoi(a[1]);
    int32_t *off = read_exact<int32_t>(a[2], &n_off);
    double *w = read_exact<double>(a[5], &n_w);
    int64_t *skip = read_exact<int64_t>(a[6], &n_skip);
    const int32_t n_inst = (int32_t)n_off - 1;
    if (n_dip < 1 || n_inst < 0 || n_w != (size_t)n_inst || n_skip != (size_t)n_inst) {
        std::fprintf(stderr, "inconsistent pair_modes inputs\n");
        return 2;
    }
    double *out = static_cast<double *>(std::malloc(sizeof(double) * 5 * (size_t)(n_inst > 0 ? n_inst : 1)));
    const lw_status st = lw_pair_modes(m, (int64_t)(n_m / (size_t)n_dip), n_dip, off, n_inst, std::atof(a[3]),
                                       std::atoll(a[4]), w, skip, out);
    print_status("pair_modes", st);
    FILE *f = std::fopen(a[7], "wb");
    if (!f || std::fwrite(out, sizeof(double), 5 * (size_t)n_inst, f) != 5 * (size_t)n_inst) return 2;
    std::fclose(f);
    std::free(m);
    std::free(off);
    std::free(w);
    std::free(skip);
    std::free(out);
    return 0;
}

int mode_state_size(char **a)
{
    size_t n_dip, n_off;
    lw_dipole *dip = read_exact<lw_dipole>(a[0], &n_dip);
    int32_t *off = read_exact<int32_t>(a[1], &n_off);
    lw_run_opts o;
    std::memset(&o, 0, sizeof o);
    o.precision = std::atoi(a[3]);
    o.dt_policy = std::atoi(a[4]);
    o.out_stride = std::atoll(a[5]);
    o.max_vel = std::atof(a[6]);
    o.ring_depth = std::atoi(a[7]);
    int64_t size = -1;
    const lw_status st = lw_dipole_state_size(dip, (int32_t)n_dip, off, (int32_t)n_off - 1, std::atof(a[2]), &o,
                                              &size);
    std::printf("state_size %d %" PRId64 " %s\n", (int)st, size, st == LW_OK ? "" : lw_last_error());
    std::free(dip);
    std::free(off);
    return 0;
}

int mode_null_ctx()
{
    lw_traj ch;
    std::memset(&ch, 0, sizeof ch);
    ch.q = 1.0;
    lw_opts fo;
    std::memset(&fo, 0, sizeof fo);
    lw_dipole dip[2];
    std::memset(dip, 0, sizeof dip);
    for (int i = 0; i < 2; ++i) {
        dip[i].origin[0] = 1e-8 * i;
        dip[i].axis[2] = 1.0;
        dip[i].omega0 = 1e15;
        dip[i].q = 1.602176634e-19;
        dip[i].m1 = dip[i].m2 = 1.8218767403e-27;
        dip[i].d0 = 1e-31;
    }
    int32_t off[2] = {0, 2};
    lw_run_opts ro;
    std::memset(&ro, 0, sizeof ro);
    ro.out_stride = 1;
    double t = 0.0, J = 0.0, gamma[2], domega[1];
    int64_t n_state = 0;
    print_status("sync_status", lw_sync_status(nullptr, nullptr));
    print_status("set_autotune", lw_set_autotune(nullptr, 1));
    print_status("fields", lw_fields(nullptr, &ch, 1, nullptr, 1, &t, 1, &fo, nullptr, nullptr, nullptr));
    print_status("fields_noalloc", lw_fields_noalloc(nullptr, &ch, 1, nullptr, 1, &t, 1, &fo, nullptr, nullptr, nullptr));
    print_status("fields_vjp", lw_fields_vjp(nullptr, &ch, 1, nullptr, 1, &t, 1, &fo, nullptr, nullptr, nullptr));
    print_status("dipole_run", lw_dipole_run(nullptr, dip, 2, off, 1, 1e-17, 10, &ro, nullptr, nullptr, nullptr,
                                             nullptr, nullptr, nullptr, gamma, domega, nullptr));
    print_status("dipole_state_size_null_out", lw_dipole_state_size(dip, 2, off, 1, 1e-17, &ro, nullptr));
    print_status("dipole_state_size", lw_dipole_state_size(dip, 2, off, 1, 1e-17, &ro, &n_state));
    print_status("dipole_run_state", lw_dipole_run_state(nullptr, dip, 2, off, 1, 1e-17, 10, &ro, nullptr, nullptr,
                                                         nullptr, nullptr, nullptr, nullptr, nullptr, n_state, 0,
                                                         nullptr));
    print_status("dipole_run_vjp", lw_dipole_run_vjp(nullptr, dip, 2, off, 1, 1e-17, 10, &ro, nullptr, 1, &t, 1, 0,
                                                     nullptr, &J, nullptr));
    uint64_t bins[LW_ITER_BINS];
    print_status("set_iteration_histogram", lw_set_iteration_histogram(nullptr, 1));
    print_status("iteration_histogram", lw_iteration_histogram(nullptr, bins, LW_ITER_BINS, 0, nullptr));
    print_status("destroy", lw_destroy(nullptr));
    return 0;
}

int mode_create()
{
    lw_ctx *ctx = nullptr;
    const lw_status st = lw_create(&ctx, 0);
    print_status("create", st);
    if (st == LW_OK) print_status("destroy", lw_destroy(ctx));
    return 0;
}

}  // namespace

int main(int argc, char **argv)
{
    if (argc == 2 && !std::strcmp(argv[1], "theory")) return mode_theory();
    if (argc == 10 && !std::strcmp(argv[1], "pair_modes")) return mode_pair_modes(argv + 2);
    if (argc == 10 && !std::strcmp(argv[1], "state_size")) return mode_state_size(argv + 2);
    if (argc == 2 && !std::strcmp(argv[1], "null_ctx")) return mode_null_ctx();
    if (argc == 2 && !std::strcmp(argv[1], "create")) return mode_create();
    std::fprintf(stderr, "usage: see the header of host_driver.cpp\n");
    return 2;
}
