// Declarations shared by the near-field assembly and the surrogate.
#pragma once

#include "common.h"

namespace xrl {

struct NFRules {
    double gx[40], gw[40];  // Gauss-Legendre on [0,1], n_touch points
    double tx[40], tw[40];  // the same nodes through the sigmoidal map u^3/(u^3+(1-u)^3), weights times its derivative
    // touching pairs in the FP32 storage modes (touch_graded): one-sided
    // grading u -> u^2 toward the shared vertex (s = 0; n_gs points, n_gse
    // when the panels share an edge) and toward the shared side (t = 0;
    // n_gt points)
    int touch_graded, n_gs, n_gse, n_gt;
    double gs_x[16], gs_w[16], gse_x[16], gse_w[16], gt_x[16], gt_w[16];
    // near-singular pairs, by class c (r >= 1.5, 0.75 <= r < 1.5, r < 0.75):
    // an ns_n[c] x ns_n[c] conical rule on 4^ns_lev[c] sub-triangles
    double nx[3][8], nw[3][8];
    int ns_n[3], ns_lev[3];
    // ns_sym[c]: class c takes the 16-point symmetric triangle rule (exact to
    // degree 8) on each sub-triangle instead of the conical rule
    int ns_sym[3];
    double ns16_b[16][3], ns16_w[16];
    double rx4[8], rw4[8];  // regular, n_hi points
    double rx3[8], rw3[8];  // regular, n_lo points
    int n_touch, n_hi, n_lo;
    // regular pairs in the FP32 pass: symmetric triangle rules, barycentric
    // points and weights summing to one: 12 points (exact to degree 6)
    // below r_mid, 6 points (degree 4) above
    double sym_b[18][3], sym_w[18];
};

struct NFArgs {
    const int32_t *leaf_box, *box_beg, *box_end, *near_rows, *near_src, *leaf_tpad, *pvid;
    const int64_t *val_off;
    const double *pv, *cen, *diam;
    double r_near, r_mid;
    int64_t n_leaves;
    unsigned long long *counters;  // [0] self [1] touch [2] near-singular [3] regular [4] regular below r_mid
    // Queued entries, one contiguous range per queue (kQTouch, kQNs0..2):
    // work[pos] = value index, work_meta[2 pos], [2 pos + 1] = (k, l).
    // q_off[4 li + q]: first position of leaf li in queue q (exclusive scan
    // of the per-leaf counts, the queue's base included).
    int64_t *work;
    int32_t *work_meta;
    const int64_t *q_off;
    // P_kl = P_lk: a queued entry with k < l is integrated once and also
    // written to the block of leaf(l) (work_mirror[pos], -1 if that entry is
    // not stored); entries with k > l whose mirror is stored are not queued.
    int64_t *work_mirror;
    // [n_near_rows]: the mirror of every source row (row_mirror), written by
    // the counting pass and read by the filling passes
    int64_t *row_mir;
    const int32_t *panel_leaf;  // [N] leaf of each sorted panel
    // Reference point of the FP32 classification: every leaf classifies its
    // entries from centroids relative to this one point, so (k, l) and
    // (l, k) get the same class bit for bit in any two leaves (the mirror of
    // an entry skipped above is then always integrated and written).
    double cref[3];
};

// Near-field entry classes: the queues of pass 2 (touching; near-singular of
// rule class 0, 1, 2 for r >= 1.5, 0.75 <= r < 1.5, r < 0.75), regular, self.
enum { kQTouch = 0, kQNs0 = 1, kQNs1 = 2, kQNs2 = 3, kNQueues = 4, kRegular = 4, kSelf = 5 };

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
// base + i, i < n)
void ns_features(const NFArgs &a, int64_t base, int64_t n, float *feat, double *cheap, hipStream_t s);

}  // namespace xrl
