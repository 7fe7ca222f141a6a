// abi_check.cpp -- a caller of libsphfilt that uses nothing but the C-ABI and
// the HIP runtime (no Python, no PyTorch), as a C, C++ or Fortran evolution
// code would.  It checks properties that hold exactly or to round-off for the
// double FFT filter of arXiv:2305.01537 (Sec. II.A):
//   - the adjoint is the transpose: <F x, y> = <x, F^T y> to 1e-13;
//   - linearity with an exact scale: F(2 x) = 2 F(x) bit for bit (every step
//     is a sum of products with the data, and scaling by 2 is exact);
//   - in place equals out of place, bit for bit;
//   - a batch of the same patch equals the plan, bit for bit, and the
//     allocation-free batch call equals the batch call;
//   - hybrid fields: replaying recorded decisions gives the recorded field bit
//     for bit, and the adjoint that replays a forward call's decisions is its
//     transpose (<F_D x, y> = <x, F_D^T y> to 1e-13);
//   - argument errors come back as status codes before any device work.
// Prints one line per check and "abi_check: ok"; exits non-zero on failure.
#include "../../include/sphfilt.h"

#include <hip/hip_runtime_api.h>

#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <vector>

namespace {

int failures = 0;

void expect(bool ok, const char *what)
{
    std::printf("%s: %s\n", what, ok ? "ok" : "FAILED");
    if (!ok) ++failures;
}

bool hip_ok(hipError_t e, const char *what)
{
    if (e == hipSuccess) return true;
    std::printf("%s: %s\n", what, hipGetErrorString(e));
    ++failures;
    return false;
}

// Deterministic values in [-1, 1) (a 64-bit linear congruential sequence).
void fill(std::vector<double> &v, uint64_t seed)
{
    uint64_t s = seed * 6364136223846793005ULL + 1442695040888963407ULL;
    for (double &x : v) {
        s = s * 6364136223846793005ULL + 1442695040888963407ULL;
        x = (double)(s >> 11) * 0x1p-52 - 1.0;
    }
}

double dot(const std::vector<double> &a, const std::vector<double> &b)
{
    long double s = 0.0L;
    for (size_t i = 0; i < a.size(); ++i) s += (long double)a[i] * (long double)b[i];
    return (double)s;
}

}  // namespace

int main()
{
    // lines of 128 (theta) and 256 (phi) points: no fused shells, so plan and
    // batch run the same two-pass workers
    const int n_r = 6, n_theta = 64, n_phi = 256, n_fields = 3;
    const size_t n = (size_t)n_fields * n_r * n_theta * n_phi;
    const int parity[n_fields] = {1, -1, 1};
    const double L[n_fields] = {3.0, 0.8, 12.0};
    const int kind[n_fields] = {SPHFILT_EXP, SPHFILT_GAUSS, SPHFILT_SHARP};
    const sphfilt_cutoff cut = {nullptr, L, kind, 2.0, 0.0, 0.0};

    // argument errors: reported before any device work
    sphfilt_plan bad = nullptr;
    expect(sphfilt_plan_create(&bad, n_r, n_theta, 127, n_fields, parity, &cut) == SPHFILT_EINVAL &&
               bad == nullptr,
           "odd n_phi is SPHFILT_EINVAL");
    expect(sphfilt_plan_create(&bad, n_r, 100, 200, n_fields, parity, &cut) == SPHFILT_EUNSUPPORTED,
           "lines of 200 points are SPHFILT_EUNSUPPORTED");
    const int bad_parity[n_fields] = {1, 0, 1};
    expect(sphfilt_plan_create(&bad, n_r, n_theta, n_phi, n_fields, bad_parity, &cut) == SPHFILT_EINVAL,
           "parity 0 is SPHFILT_EINVAL");
    expect(sphfilt_apply(nullptr, nullptr, nullptr, nullptr) == SPHFILT_EINVAL, "NULL plan is SPHFILT_EINVAL");
    expect(sphfilt_status_string(SPHFILT_EINVAL) != nullptr && sphfilt_version() != nullptr,
           "status strings and version");

    sphfilt_plan plan = nullptr;
    const int rc = sphfilt_plan_create(&plan, n_r, n_theta, n_phi, n_fields, parity, &cut);
    expect(rc == SPHFILT_OK, "sphfilt_plan_create");
    if (rc != SPHFILT_OK) return 1;

    std::vector<double> x(n), y(n), x2(n);
    fill(x, 1);
    fill(y, 2);
    for (size_t i = 0; i < n; ++i) x2[i] = 2.0 * x[i];
    const size_t bytes = n * sizeof(double);
    double *dx = nullptr, *dy = nullptr, *dfx = nullptr, *dfty = nullptr, *dx2 = nullptr, *db = nullptr;
    bool ok = hip_ok(hipMalloc((void **)&dx, bytes), "hipMalloc") &&
              hip_ok(hipMalloc((void **)&dy, bytes), "hipMalloc") &&
              hip_ok(hipMalloc((void **)&dfx, bytes), "hipMalloc") &&
              hip_ok(hipMalloc((void **)&dfty, bytes), "hipMalloc") &&
              hip_ok(hipMalloc((void **)&dx2, bytes), "hipMalloc") &&
              hip_ok(hipMalloc((void **)&db, bytes), "hipMalloc");
    hipStream_t s = nullptr;
    ok = ok && hip_ok(hipStreamCreate(&s), "hipStreamCreate");
    ok = ok && hip_ok(hipMemcpy(dx, x.data(), bytes, hipMemcpyHostToDevice), "hipMemcpy") &&
         hip_ok(hipMemcpy(dy, y.data(), bytes, hipMemcpyHostToDevice), "hipMemcpy") &&
         hip_ok(hipMemcpy(dx2, x2.data(), bytes, hipMemcpyHostToDevice), "hipMemcpy") &&
         hip_ok(hipMemcpy(db, x.data(), bytes, hipMemcpyHostToDevice), "hipMemcpy");
    if (!ok) return 1;

    // out of place: F x, F^T y; in place: F (2 x)
    expect(sphfilt_apply(plan, dx, dfx, s) == SPHFILT_OK, "sphfilt_apply");
    expect(sphfilt_apply_adjoint(plan, dy, dfty, s) == SPHFILT_OK, "sphfilt_apply_adjoint");
    expect(sphfilt_apply(plan, dx2, dx2, s) == SPHFILT_OK, "sphfilt_apply in place");

    // a batch of the same patch, in place on a copy of x
    sphfilt_patch_desc desc;
    desc.n_r = n_r;
    desc.n_theta = n_theta;
    desc.n_phi = n_phi;
    desc.n_fields = n_fields;
    desc.parity = parity;
    desc.cut = cut;
    sphfilt_batch batch = nullptr;
    expect(sphfilt_batch_create(&batch, 1, &desc, nullptr) == SPHFILT_OK, "sphfilt_batch_create");
    const double *ins[1] = {db};
    double *outs[1] = {db};
    expect(sphfilt_batch_apply(batch, ins, outs, 0, s) == SPHFILT_OK, "sphfilt_batch_apply");
    ok = hip_ok(hipStreamSynchronize(s), "hipStreamSynchronize");
    int dev_err = -1;
    expect(sphfilt_batch_status(batch, &dev_err) == SPHFILT_OK && dev_err == 0, "batch device error word");

    std::vector<double> fx(n), fty(n), f2x(n), fb(n), xin(n);
    ok = ok && hip_ok(hipMemcpy(fx.data(), dfx, bytes, hipMemcpyDeviceToHost), "hipMemcpy") &&
         hip_ok(hipMemcpy(fty.data(), dfty, bytes, hipMemcpyDeviceToHost), "hipMemcpy") &&
         hip_ok(hipMemcpy(f2x.data(), dx2, bytes, hipMemcpyDeviceToHost), "hipMemcpy") &&
         hip_ok(hipMemcpy(fb.data(), db, bytes, hipMemcpyDeviceToHost), "hipMemcpy") &&
         hip_ok(hipMemcpy(xin.data(), dx, bytes, hipMemcpyDeviceToHost), "hipMemcpy");
    if (!ok) return 1;

    const double a = dot(fx, y), b = dot(x, fty);
    const double rel = std::fabs(a - b) / std::fmax(std::fabs(a), std::fabs(b));
    std::printf("dot test: <Fx,y> = %.17g, <x,F^T y> = %.17g, relative difference %.3g\n", a, b, rel);
    expect(rel <= 1e-13, "adjoint is the transpose");

    bool exact = true, moved = false;
    for (size_t i = 0; i < n; ++i) {
        exact &= f2x[i] == 2.0 * fx[i];
        moved |= fx[i] != x[i];
    }
    expect(exact, "F(2x) = 2 F(x) bit for bit (in place against out of place)");
    expect(moved, "the filter changes the field");
    expect(std::memcmp(xin.data(), x.data(), bytes) == 0, "out of place leaves the input untouched");
    expect(std::memcmp(fb.data(), fx.data(), bytes) == 0, "batch equals plan bit for bit");

    // the allocation-free call on the same batch, in place on another copy of x
    ok = hip_ok(hipMemcpy(db, x.data(), bytes, hipMemcpyHostToDevice), "hipMemcpy");
    expect(sphfilt_batch_apply_noalloc(batch, ins, outs, 0, s) == SPHFILT_OK, "sphfilt_batch_apply_noalloc");
    std::vector<double> fn(n);
    ok = ok && hip_ok(hipStreamSynchronize(s), "hipStreamSynchronize") &&
         hip_ok(hipMemcpy(fn.data(), db, bytes, hipMemcpyDeviceToHost), "hipMemcpy");
    expect(ok && std::memcmp(fn.data(), fb.data(), bytes) == 0, "allocation-free call equals the batch call");

    // hybrid fields 0 and 2: field 0 is a level of 2 with a jump to zero on
    // every shell's first rows, field 2 keeps the signed noise
    const int kind_h[n_fields] = {SPHFILT_HYBRID, SPHFILT_EXP, SPHFILT_HYBRID};
    const sphfilt_cutoff cut_h = {nullptr, L, kind_h, 2.0, 0.0, 0.0};
    sphfilt_plan hp = nullptr;
    expect(sphfilt_plan_create(&hp, n_r, n_theta, n_phi, n_fields, parity, &cut_h) == SPHFILT_OK,
           "hybrid sphfilt_plan_create");
    std::vector<double> xh = x;
    const size_t shell = (size_t)n_theta * n_phi;
    for (int i = 0; i < n_r; ++i)
        for (size_t k = 0; k < shell; ++k) xh[i * shell + k] = k < shell / 8 ? 0.0 : 2.0 + 0.1 * x[i * shell + k];
    const size_t n_th = (size_t)n_fields * n_r * (n_phi / 2), n_ph = (size_t)n_fields * n_r * n_theta;
    unsigned char *dth = nullptr, *dph = nullptr;
    double *dxh = nullptr, *drec = nullptr, *drep = nullptr, *dadj = nullptr;
    ok = hip_ok(hipMalloc((void **)&dth, n_th), "hipMalloc") && hip_ok(hipMalloc((void **)&dph, n_ph), "hipMalloc") &&
         hip_ok(hipMalloc((void **)&dxh, bytes), "hipMalloc") && hip_ok(hipMalloc((void **)&drec, bytes), "hipMalloc") &&
         hip_ok(hipMalloc((void **)&drep, bytes), "hipMalloc") && hip_ok(hipMalloc((void **)&dadj, bytes), "hipMalloc") &&
         hip_ok(hipMemset(dth, 0, n_th), "hipMemset") && hip_ok(hipMemset(dph, 0, n_ph), "hipMemset") &&
         hip_ok(hipMemcpy(dxh, xh.data(), bytes, hipMemcpyHostToDevice), "hipMemcpy");
    if (!ok) return 1;
    expect(sphfilt_apply_ex(hp, dxh, drec, 0, dth, dph, 0, s) == SPHFILT_OK, "hybrid forward, recording");
    expect(sphfilt_apply_ex(hp, dxh, drep, 0, dth, dph, 1, s) == SPHFILT_OK, "hybrid forward, replaying");
    expect(sphfilt_apply_ex(hp, dy, dadj, 1, dth, dph, 1, s) == SPHFILT_OK, "hybrid adjoint, replaying");
    std::vector<double> rec(n), rep(n), adj(n);
    std::vector<unsigned char> th(n_th), ph(n_ph);
    ok = hip_ok(hipStreamSynchronize(s), "hipStreamSynchronize") &&
         hip_ok(hipMemcpy(rec.data(), drec, bytes, hipMemcpyDeviceToHost), "hipMemcpy") &&
         hip_ok(hipMemcpy(rep.data(), drep, bytes, hipMemcpyDeviceToHost), "hipMemcpy") &&
         hip_ok(hipMemcpy(adj.data(), dadj, bytes, hipMemcpyDeviceToHost), "hipMemcpy") &&
         hip_ok(hipMemcpy(th.data(), dth, n_th, hipMemcpyDeviceToHost), "hipMemcpy") &&
         hip_ok(hipMemcpy(ph.data(), dph, n_ph, hipMemcpyDeviceToHost), "hipMemcpy");
    if (!ok) return 1;
    size_t fired = 0;
    for (unsigned char c : th) fired += c;
    for (unsigned char c : ph) fired += c;
    std::printf("hybrid: %zu of %zu hybrid lines took the Gaussian\n", fired, (n_th + n_ph) * 2 / 3);
    expect(fired > 0 && fired < (n_th + n_ph) * 2 / 3, "the detector fires on some hybrid lines, not all");
    expect(std::memcmp(rec.data(), rep.data(), bytes) == 0, "replayed decisions give the recorded field");
    const double ah = dot(rec, y), bh = dot(xh, adj);
    const double relh = std::fabs(ah - bh) / std::fmax(std::fabs(ah), std::fabs(bh));
    std::printf("hybrid dot test: relative difference %.3g\n", relh);
    expect(relh <= 1e-13, "the adjoint with a forward call's decisions is its transpose");
    sphfilt_plan_destroy(hp);
    for (double *p : {dxh, drec, drep, dadj}) (void)hipFree(p);
    (void)hipFree(dth);
    (void)hipFree(dph);

    sphfilt_batch_destroy(batch);
    sphfilt_plan_destroy(plan);
    (void)hipStreamDestroy(s);
    for (double *p : {dx, dy, dfx, dfty, dx2, db}) (void)hipFree(p);
    std::printf("abi_check: %s\n", failures ? "FAILED" : "ok");
    return failures ? 1 : 0;
}
