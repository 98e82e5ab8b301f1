// Drives the host side of libls -- argument checks of every C-ABI entry point, the workspace
// sizing (arena carves for the sketch, the lists, the QR and the pass), and the served stream's
// bookkeeping -- through host-only contexts and servers (device -1), for a build of the library
// with AddressSanitizer and UndefinedBehaviorSanitizer on the host code.  No device work is done.
#include <cstdint>
#include <cstdio>

#include "ls.h"

static int failures = 0;
static void check(bool ok, const char *what)
{
    if (!ok) {
        std::fprintf(stderr, "FAILED: %s\n", what);
        ++failures;
    }
}

int main()
{
    // fake, aligned, never dereferenced device pointers: every call below stops before device work
    double *P = reinterpret_cast<double *>(uintptr_t(0x10000));
    float *Pf = reinterpret_cast<float *>(uintptr_t(0x10000));
    int32_t *Pi = reinterpret_cast<int32_t *>(uintptr_t(0x10000));
    int8_t *Pb = reinterpret_cast<int8_t *>(uintptr_t(0x10000));
    ls_ctx *ctx = nullptr, *bad = nullptr;
    check(ls_create(-1, &ctx) == LS_OK && ctx, "host-only context");
    ls_destroy(ctx);
    // no GPU here: a device index is refused; with a GPU, device 0 would make a real context
    const ls_status st_bad = ls_create(-2, &bad);
    check(st_bad == LS_ERR_DEVICE && bad == nullptr, "bad device index");
    check(ls_create(-1, &ctx) == LS_OK, "host-only context again");
    int64_t iv = 0;
    double dv = 0.0;
    for (int key = 1; key <= 12; ++key) check(ls_get_option(ctx, key, &iv, &dv) == LS_OK, "get option");
    check(ls_set_option(ctx, LS_OPT_ZETA, 0, 0.0) == LS_ERR_ARG, "zeta 0");
    check(ls_set_option(ctx, 99, 0, 0.0) == LS_ERR_ARG, "unknown option");
    check(ls_last_error(ctx) != nullptr && ls_last_error(nullptr) != nullptr, "last error");
    // valid arguments stop at "no device"; invalid ones are refused first
    check(ls_sketch_embedding(ctx, nullptr, 1000, 100, 8, 1, Pi, Pb) == LS_ERR_DEVICE, "embedding");
    check(ls_sketch_embedding(ctx, nullptr, 1000, 100, 200, 1, Pi, Pb) == LS_ERR_ARG, "embedding zeta > d");
    check(ls_sketch_csr(ctx, nullptr, 1000, 100, 8, 1, Pi, Pi) == LS_ERR_DEVICE, "csr");
    check(ls_sketch(ctx, nullptr, 100000, 500, P, 500, P, 10000, 8, 1, P, 500, P) == LS_ERR_DEVICE, "sketch");
    check(ls_sketch(ctx, nullptr, 100000, 500, P, 499, P, 10000, 8, 1, P, 500, P) == LS_ERR_ARG, "sketch lda");
    check(ls_sketch(ctx, nullptr, 100000, 500, P, 500, P, 10000, 8, 1, P, 500, nullptr) == LS_ERR_ARG, "sketch b/Sb");
    check(ls_sketch_f32(ctx, nullptr, 100000, 500, P, 500, P, 10000, 8, 1, Pf, 500, Pf) == LS_ERR_DEVICE, "sketch f32");
    check(ls_qr_sketch(ctx, nullptr, 10000, 500, P, 500, P, P, 500, P) == LS_ERR_DEVICE, "qr");
    check(ls_qr_sketch(ctx, nullptr, 400, 500, P, 500, P, P, 500, P) == LS_ERR_ARG, "qr d < n");
    check(ls_qr_sketch_f32(ctx, nullptr, 10000, 500, Pf, 500, Pf, Pf, 500, P) == LS_ERR_DEVICE, "qr f32");
    check(ls_gradient(ctx, nullptr, 1000, 10, P, 10, P, P, P, nullptr) == LS_ERR_DEVICE, "gradient");
    check(ls_gradient_noalloc(ctx, nullptr, 1000, 10, P, 10, P, P, P, nullptr) == LS_ERR_DEVICE, "gradient noalloc");
    check(ls_gradient(ctx, nullptr, 1000, 4096, P, 4096, P, P, P, nullptr) == LS_ERR_UNSUPPORTED, "gradient n");
    check(ls_precond_solve(ctx, nullptr, 10, P, 10, P, P) == LS_ERR_DEVICE, "precond");
    check(ls_precond_solve_f32(ctx, nullptr, 10, Pf, 10, P, P) == LS_ERR_DEVICE, "precond f32");
    check(ls_iterate(ctx, nullptr, 1000, 10, P, 10, P, P, 10, P, 3, nullptr) == LS_ERR_DEVICE, "iterate");
    check(ls_iterate(ctx, nullptr, 1000, 10, P, 10, P, P, 10, P, -1, nullptr) == LS_ERR_ARG, "iterate q < 0");
    check(ls_solve(ctx, nullptr, 1000, 10, P, 10, P, 200, 5, P) == LS_ERR_DEVICE, "solve");
    check(ls_solve(ctx, nullptr, 1000, 10, P, 10, P, 0, 5, P) == LS_ERR_DEVICE, "solve, d from eq. dimension");
    check(ls_solve(ctx, nullptr, 5, 10, P, 10, P, 200, 5, P) == LS_ERR_ARG, "solve m < n");
    int64_t du = 0;
    int32_t steps = 0, prec = 0;
    check(ls_solve_info(ctx, &du, &steps, nullptr, nullptr, &prec) == LS_OK, "solve info");
    check(ls_sync(ctx, nullptr) == LS_ERR_DEVICE, "sync");
    double ms = 0.0;
    int64_t launches = 0;
    check(ls_profile(ctx, &ms, &launches, 1) == LS_ERR_DEVICE, "profile");
    ls_destroy(ctx);
    ls_destroy(nullptr);

    // served stream: host-only server, footprints of many shapes (arena sizing of every buffer)
    ls_server *sv = nullptr;
    check(ls_server_create(-1, int64_t(1) << 40, 64, &sv) == LS_OK && sv, "host-only server");
    const int64_t shapes[][3] = {{4000, 32, 640}, {200000, 256, 5120}, {2000000, 500, 10000},
                                 {1000000, 1000, 20000}, {4000000, 2000, 40000}, {70001, 2048, 41000}};
    const int32_t precs[] = {LS_PRECISION_FP64, LS_PRECISION_MIXED};
    for (int32_t prec : precs) {
        check(ls_server_set_precision(sv, prec) == LS_OK, "set precision");
        for (const auto &sh : shapes) {
            int64_t res = 0, su = 0;
            check(ls_server_footprint(sv, sh[0], sh[1], sh[2], &res, &su) == LS_OK && res > 0 && su > 0, "footprint");
            int64_t t = 0;
            check(ls_server_submit(sv, sh[0], sh[1], P, sh[1], P, sh[2], 40, 1, P, &t) == LS_ERR_DEVICE, "submit");
        }
    }
    check(ls_server_set_precision(sv, 7) == LS_ERR_ARG, "bad precision");
    int32_t used = 0;
    check(ls_server_request_precision(sv, 7, &used) == LS_ERR_ARG, "unknown ticket precision");
    int64_t st[8] = {0};
    check(ls_server_stats(sv, st) == LS_OK && st[0] == 0, "stats");
    ls_status r = LS_OK;
    check(ls_server_wait(sv, 7, 0.0, &r) == LS_ERR_ARG, "unknown ticket");
    double times[4];
    check(ls_server_request_info(sv, 7, times) == LS_ERR_ARG, "unknown ticket info");
    check(ls_server_last_error(sv) != nullptr, "server last error");
    ls_server_destroy(sv);
    ls_server_destroy(nullptr);
    if (failures) return 1;
    std::printf("host driver: all calls clean\n");
    return 0;
}
