// plan.cpp -- host side of the sphfilt C-ABI (include/sphfilt.h).
//
// A plan turns the filter's parameters into device tables once:
//   * one item per shell (field, radius) for the theta-pass, carrying
//     l_max = max(floor, 2 rho L) (Sec. II.B, l_max equation);
//   * one item per ring pair (j, n_theta-1-j) for the phi-pass, carrying
//     m_max = max(floor, 2 rho sin(theta_j) L) (Sec. II.B, m_max equation);
//   * twiddle tables exp(-2 pi i j / N) for both line lengths.
// Items whose mask is 1 on every mode (cutoff >= N/2 for the exponential and
// sharp filters) are sorted after the others: an in-place call launches over
// the non-identity prefix only, an out-of-place call over all items and the
// identity ones are copied.
#include "../../include/sphfilt.h"
#include "sphfilt_internal.h"

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <new>
#include <vector>

using namespace sphfilt;

namespace {

constexpr double kPi = 3.14159265358979323846264338327950288;

struct DeviceTables {
    ThetaItem *theta = nullptr;
    PhiItem *phi = nullptr;
    Twiddle *tw_theta = nullptr;
    Twiddle *tw_phi = nullptr;
    double *eneg = nullptr;
};

struct HostTables {
    std::vector<ThetaItem> theta;   // active first, then identity
    std::vector<PhiItem> phi;
    int theta_active = 0;
    int phi_active = 0;
};

bool fault(const char *what)
{
    const char *e = std::getenv("SPHFILT_FAULT");
    return e && std::strcmp(e, what) == 0;
}

bool supported_line(int n) { return n == 32 || n == 64 || n == 128 || n == 256; }

// cos and sin of 2 pi j / N, reducing the angle to the first octant with
// integer arithmetic so the table is accurate to the last bit or so.
void unit_root(long long j, long long N, double *c, double *s)
{
    j %= N;
    if (j < 0) j += N;
    if (N % 8 != 0) {
        const double a = 2.0 * kPi * (double)j / (double)N;
        *c = std::cos(a);
        *s = std::sin(a);
        return;
    }
    bool neg_s = false, neg_c = false, swap = false;
    if (2 * j > N) { j = N - j; neg_s = true; }          // theta -> 2pi - theta
    if (4 * j > N) { j = N / 2 - j; neg_c = true; }      // theta -> pi - theta
    if (8 * j > N) { j = N / 4 - j; swap = true; }       // theta -> pi/2 - theta
    const double a = 2.0 * kPi * (double)j / (double)N;
    double cc = std::cos(a), ss = std::sin(a);
    if (swap) { double t = cc; cc = ss; ss = t; }
    if (neg_c) cc = -cc;
    if (neg_s) ss = -ss;
    *c = cc;
    *s = ss;
}

std::vector<Twiddle> twiddles(int N)
{
    std::vector<Twiddle> t((size_t)N);
    for (int j = 0; j < N; ++j) {
        double c, s;
        unit_root(j, N, &c, &s);
        t[(size_t)j] = Twiddle{c, -s};
    }
    return t;
}

// e^{-k}, k in [0, kExpTable): the exponential mask above its cutoff.
std::vector<double> exp_table()
{
    std::vector<double> e((size_t)kExpTable);
    for (int k = 0; k < kExpTable; ++k) e[(size_t)k] = std::exp(-(double)k);
    return e;
}

int validate(int n_r, int n_theta, int n_phi, int n_fields, const int *parity,
             const sphfilt_cutoff *cut)
{
    if (n_r <= 0 || n_theta <= 0 || n_phi <= 0 || n_fields <= 0) return SPHFILT_EINVAL;
    if (n_phi % 2 != 0) return SPHFILT_EINVAL;
    if (!parity || !cut || !cut->L) return SPHFILT_EINVAL;
    if (!std::isfinite(cut->floor_modes) || cut->floor_modes < 0.0) return SPHFILT_EINVAL;
    for (int f = 0; f < n_fields; ++f) {
        if (parity[f] != 1 && parity[f] != -1) return SPHFILT_EINVAL;
        if (!std::isfinite(cut->L[f]) || !(cut->L[f] > 0.0)) return SPHFILT_EINVAL;
        if (cut->kind && (cut->kind[f] < SPHFILT_EXP || cut->kind[f] > SPHFILT_SHARP))
            return SPHFILT_EINVAL;
    }
    if (cut->rho)
        for (int i = 0; i < n_r; ++i)
            if (!std::isfinite(cut->rho[i]) || !(cut->rho[i] > 0.0)) return SPHFILT_EINVAL;
    // ring ids are 32-bit on the device
    if ((long long)n_fields * n_r * n_theta > 0x7fffffffLL) return SPHFILT_EUNSUPPORTED;
    if (!supported_line(2 * n_theta) || !supported_line(n_phi)) return SPHFILT_EUNSUPPORTED;
    return SPHFILT_OK;
}

void build_items(int n_r, int n_theta, int n_phi, int n_fields, const int *parity,
                 const sphfilt_cutoff *cut, HostTables *h)
{
    std::vector<ThetaItem> ta, ti;
    std::vector<PhiItem> pa, pi;
    for (int f = 0; f < n_fields; ++f) {
        const int kind = cut->kind ? cut->kind[f] : SPHFILT_EXP;
        const int base_flags = kind | (parity[f] < 0 ? kFlagOddParity : 0);
        const double L = cut->L[f];
        for (int i = 0; i < n_r; ++i) {
            const double rho = cut->rho ? cut->rho[i] : (double)i + 0.5;
            double c = 2.0 * rho * L;
            if (!(c > cut->floor_modes)) c = cut->floor_modes;
            const bool ident = kind != SPHFILT_GAUSS && c >= (double)n_theta;
            const ThetaItem t{f * n_r + i, base_flags | (ident ? kFlagIdentity : 0), c};
            (ident ? ti : ta).push_back(t);
            for (int j = 0; j < n_theta / 2; ++j) {
                const double s = std::sin(((double)j + 0.5) * kPi / (double)n_theta);
                double m = 2.0 * rho * s * L;
                if (!(m > cut->floor_modes)) m = cut->floor_modes;
                const bool pid = kind != SPHFILT_GAUSS && m >= (double)(n_phi / 2);
                const PhiItem p{(f * n_r + i) * n_theta + j, base_flags | (pid ? kFlagIdentity : 0), m};
                (pid ? pi : pa).push_back(p);
            }
        }
    }
    h->theta_active = (int)ta.size();
    h->phi_active = (int)pa.size();
    h->theta = std::move(ta);
    h->theta.insert(h->theta.end(), ti.begin(), ti.end());
    h->phi = std::move(pa);
    h->phi.insert(h->phi.end(), pi.begin(), pi.end());
}

void fill_stats(int n_r, int n_theta, int n_phi, int n_fields, const HostTables &h, sphfilt_stats *s)
{
    std::memset(s, 0, sizeof(*s));
    const long long shell_pts = (long long)n_theta * n_phi;
    s->n_points = (long long)n_fields * n_r * shell_pts;
    s->theta_shells_total = (long long)n_fields * n_r;
    s->theta_shells_active = h.theta_active;
    s->theta_lines_total = s->theta_shells_total * (n_phi / 2);
    s->theta_lines_active = (long long)h.theta_active * (n_phi / 2);
    s->phi_rings_total = (long long)n_fields * n_r * n_theta;
    s->phi_rings_active = 2LL * h.phi_active;
    const long long th_act = (long long)h.theta_active * shell_pts;   // points
    const long long ph_act = s->phi_rings_active * n_phi;
    s->bytes_forward_inplace = 16 * (th_act + ph_act);
    s->bytes_forward_outofplace = 16 * (s->n_points + ph_act);
    s->bytes_adjoint_inplace = 16 * (ph_act + th_act);
    s->bytes_adjoint_outofplace = 16 * (s->n_points + th_act);
}

}  // namespace

struct sphfilt_plan_s {
    int n_r, n_theta, n_phi, n_fields;
    int device;
    HostTables host;
    DeviceTables dev;
    int theta_cols, phi_lines;
};

namespace {

void free_device(DeviceTables *d)
{
    if (d->theta) (void)hipFree(d->theta);
    if (d->phi) (void)hipFree(d->phi);
    if (d->tw_theta) (void)hipFree(d->tw_theta);
    if (d->tw_phi) (void)hipFree(d->tw_phi);
    if (d->eneg) (void)hipFree(d->eneg);
    *d = DeviceTables{};
}

template <typename T>
int upload(T **dst, const std::vector<T> &src)
{
    const size_t bytes = sizeof(T) * (src.empty() ? 1 : src.size());
    hipError_t e = hipMalloc((void **)dst, bytes);
    if (e == hipErrorOutOfMemory) { *dst = nullptr; return SPHFILT_ENOMEM; }
    if (e != hipSuccess) { *dst = nullptr; return SPHFILT_EDEVICE; }
    if (!src.empty() && hipMemcpy(*dst, src.data(), sizeof(T) * src.size(), hipMemcpyHostToDevice) != hipSuccess)
        return SPHFILT_EDEVICE;
    return SPHFILT_OK;
}

// Make the plan's device current for the duration of one call.
struct DeviceGuard {
    int prev = -1;
    bool ok = true;
    explicit DeviceGuard(int dev)
    {
        if (hipGetDevice(&prev) != hipSuccess) { ok = false; return; }
        if (prev != dev && hipSetDevice(dev) != hipSuccess) ok = false;
    }
    ~DeviceGuard()
    {
        int cur;
        if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
    }
};

enum class Pass { Theta, Phi };

int run_pass(sphfilt_plan p, Pass which, const double *in, double *out, bool all_items, hipStream_t s)
{
    hipError_t e;
    if (which == Pass::Theta) {
        const int n = all_items ? (int)p->host.theta.size() : p->host.theta_active;
        e = launch_theta(2 * p->n_theta, p->theta_cols, in, out, p->dev.theta, n, p->n_theta,
                         p->n_phi, p->dev.tw_theta, p->dev.eneg, s);
    } else {
        const int n = all_items ? (int)p->host.phi.size() : p->host.phi_active;
        e = launch_phi(p->n_phi, p->phi_lines, in, out, p->dev.phi, n, p->n_theta, p->dev.tw_phi,
                       p->dev.eneg, s);
    }
    return e == hipSuccess ? SPHFILT_OK : SPHFILT_EDEVICE;
}

int check_call(sphfilt_plan p, const double *in, double *out)
{
    if (!p || !in || !out) return SPHFILT_EINVAL;
    const size_t bytes = sizeof(double) * (size_t)p->n_fields * p->n_r * p->n_theta * p->n_phi;
    const uintptr_t a = (uintptr_t)in, b = (uintptr_t)out;
    if (a != b && a < b + bytes && b < a + bytes) return SPHFILT_EINVAL;   // partial overlap
    if (fault("launch")) return SPHFILT_EDEVICE;
    return SPHFILT_OK;
}

// Two passes in the given order.  Out of place, the first pass runs over all
// items (copying identity lines) and the second works in place on `out`.
int apply_two(sphfilt_plan p, Pass first, Pass second, const double *in, double *out, void *stream)
{
    int rc = check_call(p, in, out);
    if (rc) return rc;
    DeviceGuard g(p->device);
    if (!g.ok) return SPHFILT_EDEVICE;
    hipStream_t s = (hipStream_t)stream;
    const bool inplace = in == out;
    rc = run_pass(p, first, in, out, !inplace, s);
    if (rc) return rc;
    return run_pass(p, second, out, out, false, s);
}

int apply_one(sphfilt_plan p, Pass which, const double *in, double *out, void *stream)
{
    int rc = check_call(p, in, out);
    if (rc) return rc;
    DeviceGuard g(p->device);
    if (!g.ok) return SPHFILT_EDEVICE;
    return run_pass(p, which, in, out, in != out, (hipStream_t)stream);
}

}  // namespace

extern "C" {

int sphfilt_workload_stats(int n_r, int n_theta, int n_phi, int n_fields, const int *parity,
                           const sphfilt_cutoff *cut, sphfilt_stats *out)
{
    if (!out) return SPHFILT_EINVAL;
    int rc = validate(n_r, n_theta, n_phi, n_fields, parity, cut);
    if (rc) return rc;
    try {
        HostTables h;
        build_items(n_r, n_theta, n_phi, n_fields, parity, cut, &h);
        fill_stats(n_r, n_theta, n_phi, n_fields, h, out);
    } catch (const std::bad_alloc &) {
        return SPHFILT_ENOMEM;
    }
    return SPHFILT_OK;
}

int sphfilt_plan_create(sphfilt_plan *out, int n_r, int n_theta, int n_phi, int n_fields,
                        const int *parity, const sphfilt_cutoff *cut)
{
    if (!out) return SPHFILT_EINVAL;
    *out = nullptr;
    int rc = validate(n_r, n_theta, n_phi, n_fields, parity, cut);
    if (rc) return rc;
    if (fault("alloc")) return SPHFILT_ENOMEM;
    sphfilt_plan p = new (std::nothrow) sphfilt_plan_s();
    if (!p) return SPHFILT_ENOMEM;
    p->n_r = n_r;
    p->n_theta = n_theta;
    p->n_phi = n_phi;
    p->n_fields = n_fields;
    p->theta_cols = default_theta_cols(n_phi);
    p->phi_lines = default_phi_lines(n_phi);
    try {
        build_items(n_r, n_theta, n_phi, n_fields, parity, cut, &p->host);
        if (hipGetDevice(&p->device) != hipSuccess) rc = SPHFILT_EDEVICE;
        if (!rc) rc = upload(&p->dev.theta, p->host.theta);
        if (!rc) rc = upload(&p->dev.phi, p->host.phi);
        if (!rc) rc = upload(&p->dev.tw_theta, twiddles(2 * n_theta));
        if (!rc) rc = upload(&p->dev.tw_phi, twiddles(n_phi));
        if (!rc) rc = upload(&p->dev.eneg, exp_table());
    } catch (const std::bad_alloc &) {
        rc = SPHFILT_ENOMEM;
    }
    if (rc) {
        free_device(&p->dev);
        delete p;
        return rc;
    }
    *out = p;
    return SPHFILT_OK;
}

int sphfilt_plan_destroy(sphfilt_plan plan)
{
    if (!plan) return SPHFILT_OK;
    {
        DeviceGuard g(plan->device);
        free_device(&plan->dev);
    }
    delete plan;
    return SPHFILT_OK;
}

int sphfilt_apply(sphfilt_plan plan, const double *in, double *out, void *stream)
{
    return apply_two(plan, Pass::Theta, Pass::Phi, in, out, stream);
}

int sphfilt_apply_adjoint(sphfilt_plan plan, const double *in, double *out, void *stream)
{
    return apply_two(plan, Pass::Phi, Pass::Theta, in, out, stream);
}

int sphfilt_apply_theta(sphfilt_plan plan, const double *in, double *out, void *stream)
{
    return apply_one(plan, Pass::Theta, in, out, stream);
}

int sphfilt_apply_phi(sphfilt_plan plan, const double *in, double *out, void *stream)
{
    return apply_one(plan, Pass::Phi, in, out, stream);
}

int sphfilt_plan_stats(sphfilt_plan plan, sphfilt_stats *out)
{
    if (!plan || !out) return SPHFILT_EINVAL;
    fill_stats(plan->n_r, plan->n_theta, plan->n_phi, plan->n_fields, plan->host, out);
    return SPHFILT_OK;
}

int sphfilt_plan_set_schedule(sphfilt_plan plan, int theta_cols, int phi_lines)
{
    if (!plan) return SPHFILT_EINVAL;
    const int tc = theta_cols ? theta_cols : plan->theta_cols;
    const int pl = phi_lines ? phi_lines : plan->phi_lines;
    if (!theta_shape_ok(2 * plan->n_theta, tc, plan->n_phi) || !phi_shape_ok(plan->n_phi, pl))
        return SPHFILT_EINVAL;
    plan->theta_cols = tc;
    plan->phi_lines = pl;
    return SPHFILT_OK;
}

int sphfilt_plan_get_schedule(sphfilt_plan plan, int *theta_cols, int *phi_lines)
{
    if (!plan) return SPHFILT_EINVAL;
    if (theta_cols) *theta_cols = plan->theta_cols;
    if (phi_lines) *phi_lines = plan->phi_lines;
    return SPHFILT_OK;
}

const char *sphfilt_status_string(int status)
{
    switch (status) {
    case SPHFILT_OK: return "ok";
    case SPHFILT_EINVAL: return "invalid argument";
    case SPHFILT_ENOMEM: return "out of memory";
    case SPHFILT_EDEVICE: return "HIP device or launch error";
    case SPHFILT_EUNSUPPORTED: return "size not supported by this build";
    default: return "unknown status";
    }
}

const char *sphfilt_version(void) { return "0.1.0"; }

}  // extern "C"
