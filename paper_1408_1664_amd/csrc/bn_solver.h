// Host-side plan of one solve: tile sizes and the workspace layout.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include <vector>

#include "../../include/bn.h"
#include "bn_kernels.h"

namespace bnk {

// LDS histogram limit of the local-score kernel (parent configurations x
// child values of the largest family).
constexpr int kMaxBins = 16384;

struct Plan {
    int n, m, d, N;
    uint32_t K;                 // parent sets per node
    int bA, bL, bG, aG, W;      // tile bits
    bool two_level;             // Gamma high bits in two passes
    uint32_t KG, KA;
    bool x32;
    int max_bins;
    int lin_mode;                 // linear tiles: 0 off, 1 on, 2 every tile to the fallback
    GammaGeom gg;                 // per-endpoint Gamma geometry
    uint64_t y1_elems, y2_elems;
    std::vector<uint32_t> tiles;  // C(n - bL, h), h = 0..n-bL
    size_t o_binom, o_lorder, o_loff, o_pat, o_seed, o_famask, o_seedA, o_items, o_ordC, o_arity, o_rho, o_q, o_logp,
        o_beta, o_qt, o_gexp, o_alpha_f, o_alpha_b, o_L_f, o_L_b, o_R_f, o_R_b, o_Y1, o_Y2,
        o_gam, o_part, o_layer, o_resid, o_diag, o_cnt, o_post, o_data, o_scores_end, o_fbA,
        o_fbG, o_rtG, o_betal, o_anc, o_linok, o_Zs, o_ps, o_bits;
    uint32_t KS;                  // K(13, d - 1)
    bool alpha_lin;               // linear alpha tiles (seeds in o_Zs)
    bool fused;                   // alpha never materialised (9-bit block seeds)
    uint32_t KS9;                 // K(9, d - 1): stored seeds per block
    size_t o_zw9, o_emax, o_flin, o_hord, o_glo;
    size_t total;
};

bn_status validate(const bn_problem *p, bool host_data, bool check_values);
Plan make_plan(int n, int d, int m, bn_precision prec, bool with_data, bool with_post);
bn_status enqueue_solve(const Plan &P, const bn_problem *p, const uint8_t *dev_data, char *ws,
                        hipStream_t st, double *dev_post, double *dev_diag, PhaseEvents *ev,
                        double *dev_ps = nullptr);

}  // namespace bnk
