// sphfilt_internal.h -- types shared by the host plan and the kernels.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace sphfilt {

// Item flags: low two bits are the filter kind (SPHFILT_EXP / GAUSS / SHARP).
enum : int {
    kKindMask = 3,
    kFlagOddParity = 4,    // axis parity sign -1
    kFlagIdentity = 8,     // mask is 1 for every mode of the line: copy only
};

// One shell (field f, radius i) of the theta-pass: every meridian pair of the
// shell shares l_max.  shell = f * n_r + i.
struct ThetaItem {
    int32_t shell;
    int32_t flags;
    double c;              // l_max
};

// One ring pair (j, n_theta-1-j) of the phi-pass; both rings have the same
// m_max because sin(theta) is evaluated on the mirror-symmetric colatitude.
// ring = (f * n_r + i) * n_theta + j with j < n_theta / 2.
struct PhiItem {
    int32_t ring;
    int32_t flags;
    double c;              // m_max
};

// Hybrid-filter arguments of a pass (the automatic exponential/Gaussian
// switch of Sec. II.A).  dec: one byte per real line, 1 = Gaussian; with
// replay the decisions are read from it, otherwise they are detected and,
// if dec is not null, recorded.  present: the launch has hybrid lines.
struct HybridArgs {
    double eps, threshold;
    unsigned char *dec;
    int replay;
    int present;
};

// Length of the e^{-k} table: covers k <= N/2 for every supported N.
constexpr int kExpTable = 512;

struct Twiddle {
    double re, im;         // exp(-2 pi i j / N)
};

// Launchers (kernels_theta.hip, kernels_phi.hip, kernels.hip).  All return
// hipSuccess or the launch error.
// theta: n_items shells, each split in tiles of 2*cols meridian columns.
// eneg: e^{-k} for k in [0, kExpTable), used by the exponential mask.
hipError_t launch_theta(int n_line, int cols, const double *in, double *out,
                        const ThetaItem *items, int n_items, int n_theta, int n_phi,
                        const Twiddle *tw, const double *eneg, const HybridArgs &h,
                        hipStream_t stream);
// phi: n_items ring pairs, `lines` of them per workgroup.
hipError_t launch_phi(int n_line, int lines, const double *in, double *out, const PhiItem *items,
                      int n_items, int n_theta, const Twiddle *tw, const double *eneg,
                      const HybridArgs &h, hipStream_t stream);

// Fused shells: both passes of n_shells shells (every line of which is
// filtered), in the order given by `adjoint`, and in the same launch the phi
// pass of n_rings ring pairs of other shells (256/N2 per workgroup; identity
// rings are copied when in != out).  Needs shell_fusable(n_theta, n_phi).
// ring_c: the n_theta/2 phi cutoffs (j ascending) of each shell.  ht / hp:
// hybrid arguments of the theta and phi passes.  The twiddle table is the one
// of length n_phi (= 2 n_theta).
// mfma: the fused shells' theta pass as the circulant product (plain kinds,
// needs theta_gemm_ok; a launch with hybrid shells must pass false).
hipError_t launch_shell_phi(bool adjoint, int n_theta, int n_phi, const double *in, double *out,
                            const ThetaItem *shells, const double *ring_c, int n_shells,
                            const PhiItem *rings, int n_rings, const Twiddle *tw,
                            const double *eneg, const HybridArgs &ht, const HybridArgs &hp,
                            hipStream_t stream, bool mfma = false);
// The theta pass as the circulant product on the matrix cores, over active
// shells of plain kinds, on grids with theta_gemm_ok (n_phi = 2 n_theta in
// {32, 64}); tw: the twiddle table of length n_phi.
bool theta_gemm_ok(int n_theta, int n_phi);
hipError_t launch_theta_gemm(int n_theta, int n_phi, const double *in, double *out,
                             const ThetaItem *items, int n_items, const Twiddle *tw,
                             const double *eneg, hipStream_t stream);
// n_phi = 2 n_theta in {32, 64, 128}: whole shells per 256-lane workgroup.
bool shell_fusable(int n_theta, int n_phi);
int shells_per_group(int n_phi);

// Launch shapes (kernels.hip).  A theta workgroup has 256 lanes holding
// theta_lines_per_group(N) complex lines, split in sub-tiles of `cols` lines,
// one shell per sub-tile (the plan's plain theta kernel runs 128-lane
// workgroups at some N, see kernels_theta.hip); a phi workgroup holds `lines`
// ring pairs.
int lanes_per_line(int n_line);
int ilog2_int(int v);
int theta_lines_per_group(int n_line);
bool theta_shape_ok(int n_line, int cols, int n_phi);
bool phi_shape_ok(int n_line, int lines);
int default_theta_cols(int n_line, int n_phi);
int default_phi_lines(int n_line);

}  // namespace sphfilt
