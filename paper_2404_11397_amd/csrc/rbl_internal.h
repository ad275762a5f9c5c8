// Internal layout shared by the host side (api.hip) and the kernels (kernels.hip).
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

#include "rbl_physics.h"

namespace rbl {

constexpr int kMaxDet = 3;
constexpr int kNodeTile = 64;  // node tables are padded to a multiple of the wavefront

// Per-chain record produced by the setup kernel (FP64, 32 doubles, 256 B).
//   [0]        status: 1 valid, 0 outside the physical domain, NaN if theta has a NaN
//   [1..10]    dc_b  = c_b(theta) - c_b(theta0), TaylorF2 basis coefficients [rev]
//   [11..16]   K_d   = (C_d/C_d0)(dL0/dL)(Mc/Mc0)^(5/6) exp(2i dphic) exp(-2 pi i dc_const), (re, im) per d
//   [17..19]   dtau_d = (tc + dt_d) - (tc0 + dt_d0)  [s]
constexpr int kRecStride = 32;
constexpr int kRecStatus = 0;
constexpr int kRecDc = 1;
constexpr int kRecK = 11;
constexpr int kRecTau = 17;
constexpr int kRecUsed = 20;                 // entries 1..19 are differentiable
constexpr int kJacRows = kRecUsed - 1;       // rows of d(record)/d(theta), record entries 1..19

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
};

// Detector network description passed by value to kernels.
struct Network {
    int32_t n_det;
    double gmst;
    double D[kMaxDet][9];
    double r[kMaxDet][3];
};

// Device pointers of a resident event.
struct EventDev {
    int32_t n_det, n_bins, n_nodes, n_nodes_pad;
    int64_t n_freq;
    double f_low, delta_f;
    // node tables, each [n_nodes_pad] (padding: f = 0, x = ix = 1, lx = 0)
    const double* node_f;
    const double* node_x;
    const double* node_ix;
    const double* node_lx;
    // per (det, node) tables, [n_det][n_nodes_pad]: gamma (re, im), mu, nuL, nuR
    const double* g_re;
    const double* g_im;
    const double* mu;
    const double* nuL;
    const double* nuR;
};

}  // namespace rbl
