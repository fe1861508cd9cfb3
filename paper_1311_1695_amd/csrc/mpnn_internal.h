// The warm-start network behind lap_mpnn_* (mpnn.hip): a small
// message-passing network over the plan's graph whose output columns serve
// as JD's start block.  All work areas are row-major FP32 in plan order.
#pragma once

#include "block_kernels.h"

struct lap_mpnn {
    lap_mpnn_config cfg{};
    int device = 0;
    // weight matrix l: wr[l] x wc[l], column-major at params + woff[l]; bias at boff[l]
    std::vector<int> wr, wc;
    std::vector<long long> woff, boff;
    long long nparams = 0;
    lapeig::DevBuf<float> params, grad, adam_m, adam_v;
    long long step = 0;
    // work areas for the largest graph seen
    int n_alloc = 0;
    std::vector<lapeig::DevBuf<float>> hc;  // layers + 1 buffers [h | D^{-1}A h], n x 2F
    std::vector<lapeig::DevBuf<float>> zp;  // pre-activations of the hidden layers, n x H
    lapeig::DevBuf<float> yx;               // [Yh | X], n x (p + kmax)
    lapeig::DevBuf<float> gy, ghc, gh, tmp, ones;
    lapeig::DevBuf<float> small;            // [S | C], the gradient coefficients, column sums, W'
    lapeig::DevBuf<double> loss;
    lapeig::BlockScratch bs;
};

namespace lapeig {

constexpr int kMpnnMaxCols = 32;  // out_cols + target columns, and the hidden width

void mpnn_init(lap_mpnn *m, const lap_mpnn_config &cfg);
// Forward pass on plan P; leaves Yh (plan order) in the first out_cols
// columns of m->yx.
void mpnn_forward(lap_mpnn *m, const lap_plan &P, uint64_t feature_seed, hipStream_t s);
// Loss against X (device, n x kx column-major, caller order) and the
// gradient in m->grad; returns the loss.
double mpnn_loss_grad(lap_mpnn *m, const lap_plan &P, uint64_t feature_seed, const double *X, int kx,
                      hipStream_t s);
void mpnn_adam(lap_mpnn *m, float lr, hipStream_t s);
// V0 (device, n x out_cols column-major, caller order) = Yh.
void mpnn_output(lap_mpnn *m, const lap_plan &P, double *V0, hipStream_t s);

}  // namespace lapeig
