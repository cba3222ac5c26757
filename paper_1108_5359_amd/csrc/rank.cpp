// Target-rank estimation (Sec. 3.6): a host loop over the FP64 seed solver
// that grows the seed block until its rank passes eq. rank_test, or stops at
// the size limit of eq. rank_test1.
#include "rpca_internal.h"

#include <algorithm>
#include <string>
#include <vector>

namespace {

// Whether `order` (host, count entries) is a permutation of 0..count-1.
bool is_permutation(const int64_t *order, int64_t count)
{
    std::vector<unsigned char> seen((size_t)count, 0);
    for (int64_t i = 0; i < count; ++i) {
        const int64_t v = order[i];
        if (v < 0 || v >= count || seen[(size_t)v]) return false;
        seen[(size_t)v] = 1;
    }
    return true;
}

// Sorted copy of order[first .. first + count).
std::vector<int64_t> sorted_slice(const int64_t *order, int64_t first, int64_t count)
{
    std::vector<int64_t> v(order + first, order + first + count);
    std::sort(v.begin(), v.end());
    return v;
}

} // namespace

extern "C" int rpca_estimate_rank(rpca_ctx_t ctx, const float *M, int64_t m, int64_t n,
                                  int64_t ldm, int32_t r0, const rpca_opts *opts,
                                  const int64_t *row_order, const int64_t *col_order,
                                  int32_t cross_validate, rpca_rank_info *info)
{
    if (!ctx) return RPCA_ERR_ARG;
    ctx->last_error.clear();
    if (!M || !opts || !row_order || !col_order || !info)
        return set_status(ctx, RPCA_ERR_ARG, "estimate_rank: NULL argument");
    if (m < 1 || n < 1 || ldm < m) return set_status(ctx, RPCA_ERR_ARG, "estimate_rank: bad sizes of M");
    int st = check_opts(ctx, *opts);
    if (st != RPCA_OK) return st;
    const int64_t sr = opts->os_r, sc = opts->os_c;
    // eq. rank_test1 on the first block too: a guess whose block already
    // exceeds half of M is outside what l1 filtering is for
    if (r0 < 1 || 2 * sr * r0 > m || 2 * sc * r0 > n)
        return set_status(ctx, RPCA_ERR_ARG, "estimate_rank: need r0 >= 1 with os_r*r0 <= m/2 and os_c*r0 <= n/2");
    if (!is_permutation(row_order, m) || !is_permutation(col_order, n))
        return set_status(ctx, RPCA_ERR_ARG, "estimate_rank: row_order / col_order must be permutations");
    RPCA_HIP_TRY(ctx, hipSetDevice(ctx->device));

    // workspace: the block's indices (int64) and the seed's factors at the
    // largest block of the loop (p, q <= half of M, rank <= min(p, q))
    const int64_t pmax = m / 2, qmax = n / 2, kmax = std::min(pmax, qmax);
    const size_t bytes = (size_t)(pmax + qmax) * 8 + (size_t)((pmax + qmax) * kmax + kmax) * 8 + 256;
    if ((st = ensure_buf(ctx, ctx->rank_ws, bytes)) != RPCA_OK) return st;
    int64_t *dI = static_cast<int64_t *>(ctx->rank_ws.ptr);
    int64_t *dJ = dI + pmax;
    double *U = reinterpret_cast<double *>(dJ + qmax);
    double *V = U + pmax * kmax;
    double *sg = V + qmax * kmax;

    // rank r' of the seed PCP on rows row_order[r_first ..) x cols col_order[c_first ..)
    auto seed_rank = [&](int64_t r_first, int64_t p, int64_t c_first, int64_t q, int *rank) -> int {
        const std::vector<int64_t> I = sorted_slice(row_order, r_first, p);
        const std::vector<int64_t> J = sorted_slice(col_order, c_first, q);
        RPCA_HIP_TRY(ctx, hipMemcpy(dI, I.data(), (size_t)p * 8, hipMemcpyHostToDevice));
        RPCA_HIP_TRY(ctx, hipMemcpy(dJ, J.data(), (size_t)q * 8, hipMemcpyHostToDevice));
        SeedOut so;
        // target rank min(p, q): nothing is truncated, so_rank_found is r'
        const int s = run_seed(ctx, M, ldm, dI, p, dJ, q, (int32_t)std::min(p, q), *opts, U, sg, V,
                               &so, nullptr);
        *rank = so.rank_found;
        return s;
    };

    *info = rpca_rank_info{};
    info->cv_rank = -1;
    int worst = RPCA_OK;
    std::string worst_msg;
    int64_t p = sr * r0, q = sc * r0;
    for (int round = 0;; ++round) {
        if (round == RPCA_RANK_MAX_ROUNDS)
            return set_status(ctx, RPCA_WARN_RANK, "estimate_rank: round limit reached");
        int rk = 0;
        const int s = seed_rank(0, p, 0, q, &rk);
        if (s < 0) return s;
        if (s == RPCA_WARN_NOT_CONVERGED && worst == RPCA_OK) {
            worst = s;
            worst_msg = "estimate_rank: a seed missed seed_tol";
        }
        info->ranks[round] = rk;
        info->ps[round] = p;
        info->qs[round] = q;
        info->rounds = round + 1;
        info->r_est = rk;
        info->p = p;
        info->q = q;
        if (rk == 0) return set_status(ctx, RPCA_ERR_SEED, "estimate_rank: the recovered seed has rank 0");
        if (p >= sr * rk && q >= sc * rk) {          // eq. rank_test
            info->accepted = 1;
            break;
        }
        const int64_t p2 = sr * rk, q2 = sc * rk;
        if (2 * p2 > m || 2 * q2 > n)                  // eq. rank_test1
            return set_status(ctx, RPCA_WARN_RANK,
                              "estimate_rank: a seed of rank " + std::to_string(rk) +
                                  " needs a block beyond half of M (eq. rank_test1)");
        p = p2;
        q = q2;
    }
    if (cross_validate && 2 * p <= m && 2 * q <= n) {
        int rk = 0;
        const int s = seed_rank(p, p, q, q, &rk);
        if (s < 0) return s;
        info->cv_rank = rk;
        if (rk != info->r_est)
            return set_status(ctx, RPCA_WARN_RANK,
                              "estimate_rank: the cross-validation block has rank " +
                                  std::to_string(rk) + ", the accepted seed " +
                                  std::to_string(info->r_est));
    }
    if (worst != RPCA_OK) return set_status(ctx, worst, worst_msg);
    return RPCA_OK;
}
