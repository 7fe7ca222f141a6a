// host_tables.cpp -- host-side tables shared by plans and batches:
// validation, the per-shell / per-ring-pair item lists with their cutoffs
// (arXiv:2305.01537, Sec. II.A, the l_max / m_max equations), twiddles and
// the e^{-k} table of the exponential mask.
#include "host_tables.h"

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdlib>
#include <cstring>

namespace sphfilt {

constexpr double kPi = 3.14159265358979323846264338327950288;

bool fault(const char *what)
{
    const char *e = std::getenv("SPHFILT_FAULT");
    return e && std::strcmp(e, what) == 0;
}

bool supported_line(int n)
{
    return n == 32 || n == 48 || n == 64 || n == 80 || n == 96 || n == 128 || n == 160 ||
           n == 192 || n == 256;
}

// cos and sin of 2 pi j / N, reducing the angle to the first octant with
// integer arithmetic so the table is accurate to the last bit or so.
static void unit_root(long long j, long long N, double *c, double *s)
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
    if (!std::isfinite(cut->detector_eps) || cut->detector_eps < 0.0) return SPHFILT_EINVAL;
    if (!std::isfinite(cut->detector_threshold) || cut->detector_threshold < 0.0) return SPHFILT_EINVAL;
    for (int f = 0; f < n_fields; ++f) {
        if (parity[f] != 1 && parity[f] != -1) return SPHFILT_EINVAL;
        if (!std::isfinite(cut->L[f]) || !(cut->L[f] > 0.0)) return SPHFILT_EINVAL;
        if (cut->kind && (cut->kind[f] < SPHFILT_EXP || cut->kind[f] > SPHFILT_HYBRID))
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

// Items [0, k) of the first n are hybrid and the rest of them are not: k, or
// n when hybrid items come later (then every item takes the hybrid kernel).
template <typename T>
static int hybrid_prefix(const std::vector<T> &items, int n)
{
    int k = 0;
    while (k < n && (items[(size_t)k].flags & kKindMask) == SPHFILT_HYBRID) ++k;
    for (int i = k; i < n; ++i)
        if ((items[(size_t)i].flags & kKindMask) == SPHFILT_HYBRID) return n;
    return k;
}

void build_items(int n_r, int n_theta, int n_phi, int n_fields, const int *parity,
                 const sphfilt_cutoff *cut, HostTables *h)
{
    const bool fusable = shell_fusable(n_theta, n_phi);
    std::vector<ThetaItem> tf, ta, ti;     // fused, other active, identity shells
    std::vector<PhiItem> pa, pi, ra, ri;   // all rings; rings of unfused shells
    std::vector<PhiItem> rings;
    // hybrid fields first: every list then starts with the hybrid items, which
    // the hybrid-capable kernels take, and the plain kernels take the rest
    std::vector<int> order;
    for (int pass = 0; pass < 2; ++pass)
        for (int f = 0; f < n_fields; ++f)
            if ((cut->kind && cut->kind[f] == SPHFILT_HYBRID) == (pass == 0)) order.push_back(f);
    for (const int f : order) {
        const int kind = cut->kind ? cut->kind[f] : SPHFILT_EXP;
        const int base_flags = kind | (parity[f] < 0 ? kFlagOddParity : 0);
        const double L = cut->L[f];
        for (int i = 0; i < n_r; ++i) {
            const double rho = cut->rho ? cut->rho[i] : (double)i + 0.5;
            double c = 2.0 * rho * L;
            if (!(c > cut->floor_modes)) c = cut->floor_modes;
            // Gaussian and hybrid lines always act (the Gaussian damps every l != 0)
            const bool may_skip = kind == SPHFILT_EXP || kind == SPHFILT_SHARP;
            const bool ident = may_skip && c >= (double)n_theta;
            const ThetaItem t{f * n_r + i, base_flags | (ident ? kFlagIdentity : 0), c};
            rings.clear();
            bool all_rings = true;
            for (int j = 0; j < n_theta / 2; ++j) {
                const double s = std::sin(((double)j + 0.5) * kPi / (double)n_theta);
                double m = 2.0 * rho * s * L;
                if (!(m > cut->floor_modes)) m = cut->floor_modes;
                const bool pid = may_skip && m >= (double)(n_phi / 2);
                all_rings = all_rings && !pid;
                const PhiItem p{(f * n_r + i) * n_theta + j, base_flags | (pid ? kFlagIdentity : 0), m};
                rings.push_back(p);
                (pid ? pi : pa).push_back(p);
            }
            const bool fuse = fusable && !ident && all_rings;
            if (fuse) {
                tf.push_back(t);
                for (const PhiItem &p : rings) h->fused_c.push_back(p.c);
            } else {
                (ident ? ti : ta).push_back(t);
                if (ident)
                    for (const PhiItem &p : rings) ((p.flags & kFlagIdentity) ? ri : ra).push_back(p);
                else
                    for (const PhiItem &p : rings)
                        if (!(p.flags & kFlagIdentity)) h->phi_in.push_back(p);
            }
        }
    }
    h->n_fused = (int)tf.size();
    h->theta_active = (int)(tf.size() + ta.size());
    h->phi_active = (int)pa.size();
    h->theta = std::move(tf);
    h->theta.insert(h->theta.end(), ta.begin(), ta.end());
    h->theta.insert(h->theta.end(), ti.begin(), ti.end());
    h->phi = std::move(pa);
    h->phi.insert(h->phi.end(), pi.begin(), pi.end());
    h->phi_rest_active = (int)ra.size();
    h->phi_rest = std::move(ra);
    h->phi_rest.insert(h->phi_rest.end(), ri.begin(), ri.end());
    h->theta_hyb = hybrid_prefix(h->theta, h->theta_active);
    h->phi_hyb = hybrid_prefix(h->phi, h->phi_active);
    h->fused_hyb = hybrid_prefix(h->theta, h->n_fused);
    h->phi_in_hyb = hybrid_prefix(h->phi_in, (int)h->phi_in.size());
}

HybridArgs hybrid_args(const sphfilt_cutoff *cut, int n_fields)
{
    HybridArgs h{};
    h.eps = cut->detector_eps > 0.0 ? cut->detector_eps : 1e-12;
    h.threshold = cut->detector_threshold > 0.0 ? cut->detector_threshold : 0.95;
    for (int f = 0; f < n_fields && cut->kind; ++f) h.present |= cut->kind[f] == SPHFILT_HYBRID;
    return h;
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
    // every ring of a fused shell is filtered: fusing saves its phi round trip
    s->shells_fused = h.n_fused;
    s->bytes_fused_inplace = s->bytes_forward_inplace - 16LL * h.n_fused * shell_pts;
}

}  // namespace sphfilt
