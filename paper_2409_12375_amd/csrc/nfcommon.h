// Declarations shared by the near-field assembly and the surrogate.
#pragma once

#include "common.h"

namespace xrl {

struct NFRules {
    double gx[40], gw[40];  // Gauss-Legendre on [0,1], n_touch points
    double tx[40], tw[40];  // the same nodes through the sigmoidal map u^3/(u^3+(1-u)^3), weights times its derivative
    // near-singular pairs, by class c (r >= 1.5, 0.75 <= r < 1.5, r < 0.75):
    // an ns_n[c] x ns_n[c] conical rule on 4^ns_lev[c] sub-triangles
    double nx[3][8], nw[3][8];
    int ns_n[3], ns_lev[3];
    double rx4[8], rw4[8];  // regular, n_hi points
    double rx3[8], rw3[8];  // regular, n_lo points
    int n_touch, n_hi, n_lo;
};

struct NFArgs {
    const int32_t *leaf_box, *box_beg, *box_end, *near_rows, *near_src, *leaf_tpad, *pvid;
    const int64_t *val_off;
    const double *pv, *cen, *diam;
    double r_near, r_mid;
    int64_t n_leaves;
    unsigned long long *counters;  // [0] self [1] touch [2] near-singular [3] regular
    int64_t *work;                 // special entries: value index
    int32_t *work_meta;            // packed (k, l)
    unsigned long long *work_n;    // [0] touching count, [1] near-singular count (separate halves)
    int64_t work_cap;
};

struct CheapRule {
    double x[3], w[3];
};

// Surrogate weights on the device: packed FP32 (biases used from here) and
// bf16 copies of the three weight matrices, padded for the MFMA tiles.
struct MlpDevice {
    int H = 0;
    DevBuf<float> w32;
    DevBuf<short> w1, w2, w3;
};

void gauss_legendre01(int n, double *x, double *w);
void mlp_prepare_host(MlpDevice &m, const xrl_mlp *h, hipStream_t s);
void mlp_infer(const MlpDevice &m, const float *X, int64_t n, float *out, hipStream_t s);
// features and cheap values of queued near-singular entries (queue positions
// cap - 1 - i, i < n)
void ns_features(const NFArgs &a, int64_t n, float *feat, double *cheap, hipStream_t s);

}  // namespace xrl
