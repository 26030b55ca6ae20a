// Host-side launchers of the kvb kernels (internal to libkvb.so).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/kvb.h"

namespace kvb {

// Error model of the MFMA selection scores (see knn_mfma.hip).
struct ErrModel {
    double gamma;   // accumulation bound (K + 4) 2^-24
    double norm;    // relative error of the folded |y_j|^2
    double cross;   // relative bound of the cross term |2 y_i.y_j - computed|
    double center;  // relative rounding of the centred coordinates
};

struct TuneResult {
    double chi[256];
    double e_star;
    double dim;
    int g_star;
    int pad;
};

// k-NN
hipError_t launch_select_direct(const float* X, int n, int m, int kp, uint64_t* keys, float* slast,
                                hipStream_t st);
hipError_t launch_refine(const float* X, int n, int m, int k, int kp, int kstride, const uint64_t* keys,
                         const float* slast, float lb_scale, int32_t* idx, float* d2, int32_t* flags,
                         int* fb_count, int* fb_list, int force_period, hipStream_t st);
hipError_t launch_fallback(const float* X, int n, int m, int k, const int* fb_count, const int* fb_list,
                           int32_t* idx, float* d2, hipStream_t st);

hipError_t launch_prep(const float* X, int n, int m, int split, int kpad, double* colpart, int colblocks,
                       double* mu, void* Aq, void* Bc, float* ynorm2, unsigned* rmax_bits, hipStream_t st);
int mfma_kstep(int split);
int mfma_pick_ksteps(int split, int needed);
hipError_t launch_select_mfma(int split, const void* Aq, const void* Bc, int n, int kpad, int kp, const float* ynorm2,
                              const unsigned* rmax, ErrModel em, uint64_t* lists, int cap, float* lb, hipStream_t st);

// passes
hipError_t launch_adhoc_bandwidth(const float* d2, int n, int k, int k0, float* b, hipStream_t st);
hipError_t launch_density(const int32_t* idx, const float* d2, int n, int k, const float* b, double e, double d,
                          double beta, float* rho, float* psi, hipStream_t st);
int chi_num_blocks(int64_t nnz);
hipError_t launch_chi(const int32_t* idx, const float* d2, const float* rho, int64_t nnz, int k, int G,
                      double log_emin, double log_emax, double* partial, TuneResult* out, hipStream_t st);
int logsum_num_blocks(int n);
hipError_t launch_grid_scale(const float* ref, const float* rho, int n, double* partial, double* out,
                             hipStream_t st);
hipError_t launch_qpass(const int32_t* idx, const float* d2, int n, int k, const float* rho, double e,
                        double alpha, double d, double* qa, hipStream_t st);
hipError_t launch_assemble(const int32_t* idx, const float* d2, int n, int k, const float* rho, double e,
                           const double* qa, int out_kind, int64_t* rowptr, int32_t* col, float* val,
                           double* P, double* D, hipStream_t st);

}  // namespace kvb
