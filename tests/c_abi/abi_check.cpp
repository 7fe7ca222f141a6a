// abi_check.cpp -- a caller of libsphfilt that uses nothing but the C-ABI and
// the HIP runtime (no Python, no PyTorch), as a C, C++ or Fortran evolution
// code would.  It checks properties that hold exactly or to round-off for the
// double FFT filter of arXiv:2305.01537 (Sec. II.A):
//   - the adjoint is the transpose: <F x, y> = <x, F^T y> to 1e-13;
//   - linearity with an exact scale: F(2 x) = 2 F(x) bit for bit (every step
//     is a sum of products with the data, and scaling by 2 is exact);
//   - in place equals out of place, bit for bit;
//   - a batch of the same patch equals the plan, bit for bit;
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

    sphfilt_batch_destroy(batch);
    sphfilt_plan_destroy(plan);
    (void)hipStreamDestroy(s);
    for (double *p : {dx, dy, dfx, dfty, dx2, db}) (void)hipFree(p);
    std::printf("abi_check: %s\n", failures ? "FAILED" : "ok");
    return failures ? 1 : 0;
}
