// Internal layout shared by the host side (api.hip) and the kernels (kernels.hip).
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

#include "rbl_nrtv2.h"

namespace rbl {

constexpr int kMaxDet = 3;
constexpr int kWfTaylorF2 = 0;  // RBL_TAYLORF2
constexpr int kWfNrtv2 = 1;     // RBL_PHENOMD_NRTV2
constexpr int kNodeTile = 64;  // node tables are padded to a multiple of the wavefront
constexpr int kPhasorN = 512;  // entries of the unit-phasor table exp(2 pi i k / kPhasorN)

// Per-chain record produced by the setup kernels (FP64, 64 doubles, 512 B).
//   [0]        status: 1 valid, 0 outside the physical domain, NaN if theta has a NaN
//   [1..10]    dc_b  = c_b(theta) - c_b(theta0), TaylorF2 basis coefficients, in table units
//              (kPhasorN rev: an exact power-of-two scaling)
//   [11..16]   P_d = C_d / C_d0, (re, im) per detector (the likelihood kernels form K_d = P_d G)
//   [17..19]   dtau_d = (tc + dt_d) - (tc0 + dt_d0), times kPhasorN  [s]
//   [20..21]   G = (dL0/dL)(Mc/Mc0)^(5/6) exp(2i (phic - phic0)) exp(-2 pi i dc_const), (re, im)
//   [22]       dL
//   [24..52]   NrtParams<double> of the chain (IMRPhenomD_NRTidalv2 events; dc and the
//              constant phase are then unused: the edge phase is taken absolutely)
constexpr int kRecStride = 64;
constexpr int kRecStatus = 0;
constexpr int kRecDc = 1;
constexpr int kRecK = 11;
constexpr int kRecTau = 17;
constexpr int kRecG = 20;
constexpr int kRecDl = 22;
constexpr int kRecNrt = 24;

// Partial derivatives stored per chain for the gradient (FP64, 200 doubles):
//   [0, 162)   intrinsic block, rows of 6 (d/d(Mc, q, chi1, chi2, Lambda1, Lambda2)):
//              TaylorF2: rows 0-9 dc_b, row 10 dc_const, row 11 ln amp;
//              IMRPhenomD_NRTidalv2: rows 0-25 the node parameters in adjoint order
//              (see nrt_node_adjoint), row 26 ln amp
//   [162, 198) d(Re P_d, Im P_d, dt_d)/d(iota, psi, ra, dec), [3 det][3][4]
// The remaining dependencies (dL, tc, phic) are applied in closed form.
constexpr int kJacStride = 200;
constexpr int kJacInt = 0;
constexpr int kJacExt = 162;
constexpr int kJacAmpTf2 = 11;
constexpr int kJacAmpNrt = kNrtAdj;

// Reference (fiducial) constants computed once per event on the device.
struct RefConsts {
    double c0[kTf2Basis];     // reference basis coefficients [rev]
    double c0_const;          // reference constant phase [rev]
    double amp0;              // reference amplitude scale (see Tf2Coeffs::amp)
    double mc0, dl0, phic0, tc0;
    double invC0_re[kMaxDet], invC0_im[kMaxDet];   // 1 / C_d0
    double tau0[kMaxDet];                          // tc0 + dt_d0
    double h0fac_re[kMaxDet], h0fac_im[kMaxDet];   // (C_d0/dL0) exp(2i phic0) exp(-2 pi i c0_const)
    int32_t status;                                 // 1 if theta0 is valid
    int32_t waveform;                               // RBL_TAYLORF2 or RBL_PHENOMD_NRTV2
    NrtParams<double> nrt;                          // theta0 coefficients (IMRPhenomD_NRTidalv2; c0_const = 0)
    NrtConsts nc;                                   // parameter-independent matching constants
};

// Detector network description passed by value to kernels.
struct Network {
    int32_t n_det;
    double gmst;
    double D[kMaxDet][9];
    double r[kMaxDet][3];
};

// Device pointers of a resident event.
//
// Edge ("node") tables use a lane-contiguous layout: with L = ceil(n_nodes / 64)
// edges per lane, edge j belongs to lane j / L at step k = j % L and is stored at
// k * 64 + lane.  A wavefront that walks k = 0..L-1 therefore reads each table
// row with one coalesced access, and every lane sees consecutive edges (only the
// first edge of a lane needs a neighbour from another lane).
struct EventDev {
    int32_t n_det, n_bins, n_nodes, n_nodes_pad, L;
    int32_t waveform;
    int64_t n_freq;
    double f_low, delta_f;
    // node tables [n_nodes_pad][2]: (f, x = f^(1/3)) and (1/x, ln x) (padding: f = 0,
    // x = 1/x = 1, ln x = 0); a wavefront reads a step's four columns with two contiguous
    // 16-byte-per-lane loads
    const double* node_fx;
    const double* node_il;
    // per (det, node) tables, [n_det][n_nodes_pad]: gamma ([2]: re, im), mu, and the cross
    // coefficients xL_j = -nu(bin j-1), xR_j = -nu(bin j) = xL_{j+1}: the weights of
    // Re(r_{j-1} r_j*) and Re(r_j r_{j+1}*) in 2 lnL
    const double* g;
    const double* mu;
    const double* xL;
    const double* xR;
    // FP32 copies for the mixed-precision kernels
    const float* g32;
    const float* mu32;
    const float* xL32;
    const float* xR32;
    // IMRPhenomD_NRTidalv2 events: reference phase [rev] and inverse amplitude factor per edge
    const double* phi0;
    const double* ia0;
    const float* ia0_32;
    const double* node_x578;  // x^5.78 per edge (IMRPhenomD_NRTidalv2 tidal amplitude)
    // per detector: Gs_d = sum_j |gamma_dj|, Hs_d = sum_j (|mu_dj| + |xL_dj|)  [2 * kMaxDet]
    // (a chain's binned-sum magnitude is at most sum_d |K_d| Gs_d + |K_d|^2 Hs_d)
    const double* scales;
    // [kPhasorN][2]: cos and sin of 2 pi k / kPhasorN (read into LDS by the likelihood kernels)
    const double* phasor;
    // [kMaxDet]: M_d = sum_j mu_dj.  A TaylorF2 ratio has |r_dj| = |K_d| at every edge, so its
    // quadratic term is sum_j mu_dj |r_dj|^2 = |K_d|^2 M_d.
    const double* mu_sum;
};

// Mixed precision is used for a chain while the magnitude bound of its binned sum,
// M = sum_d |K_d| Gs_d + |K_d|^2 Hs_d, stays below this value; larger chains take the
// FP64 path.  Measured on the 3-detector TaylorF2 workload (1024 chains, all forced to
// the mixed path), the mixed-path error stayed below 2.2e-8 M in every range of M from
// 1e3 to 1e7, so M <= 5e4 keeps it under 1.1e-3, nine times inside the 1e-2 bound.
constexpr double kMixedScaleMax = 5.0e4;

}  // namespace rbl
