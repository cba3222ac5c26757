// Dispatch of the l1 filtering kernels (see filter_kernel.h): picks the
// built (PT, KS) class for (p, r), packs up to two families of regressions
// (column and row filtering, Sec. 3.3: independent steps) into one launch.
#include "filter_kernel.h"

#include <algorithm>
#include <climits>
#include <string>

namespace filterk {
extern template int launch_filter_pt<1>(rpca_ctx *, int, const FilterLaunch &, int, bool, hipStream_t);
extern template int launch_filter_pt<2>(rpca_ctx *, int, const FilterLaunch &, int, bool, hipStream_t);
extern template int launch_filter_pt<3>(rpca_ctx *, int, const FilterLaunch &, int, bool, hipStream_t);
extern template int launch_filter_pt<4>(rpca_ctx *, int, const FilterLaunch &, int, bool, hipStream_t);
extern template int launch_filter_pt<5>(rpca_ctx *, int, const FilterLaunch &, int, bool, hipStream_t);
extern template int launch_filter_pt<7>(rpca_ctx *, int, const FilterLaunch &, int, bool, hipStream_t);
extern template int launch_filter_pt<8>(rpca_ctx *, int, const FilterLaunch &, int, bool, hipStream_t);
extern template int launch_filter_pt<10>(rpca_ctx *, int, const FilterLaunch &, int, bool, hipStream_t);
extern template int launch_filter_pt<13>(rpca_ctx *, int, const FilterLaunch &, int, bool, hipStream_t);
extern template int launch_filter_pt<16>(rpca_ctx *, int, const FilterLaunch &, int, bool, hipStream_t);
extern template int launch_filter_pt<19>(rpca_ctx *, int, const FilterLaunch &, int, bool, hipStream_t);
extern template int launch_filter_pt<26>(rpca_ctx *, int, const FilterLaunch &, int, bool, hipStream_t);
extern template int launch_filter_pt<32>(rpca_ctx *, int, const FilterLaunch &, int, bool, hipStream_t);
} // namespace filterk

using namespace filterk;

namespace {

// Smallest built class >= need, or -1.
int pick_from(const int *list, int count, int need)
{
    for (int i = 0; i < count; ++i)
        if (list[i] >= need) return list[i];
    return -1;
}

// Both forms share the tile classes up to PT = 19; beyond, the FP32 form
// takes the quarter-tile shape too (FP32 contractions).
int pick_pt(int p, int /*precision*/) { return pick_from(kPTh, kNumPTh, (p + 15) / 16); }

// The quarter-tile shape serves the precision form from PT = 19 and the FP32
// form beyond the FP32 tile classes.
bool quarter_form(int PT, int precision) { return half_form(PT) && (precision == 1 || PT > 19); }
int pick_ks(int r) { return pick_from(kKS, kNumKS, (r + 3) / 4); }

size_t lds_limit(rpca_ctx *ctx) { return ctx->max_lds ? ctx->max_lds : 65536; }

// Smallest p whose regressions use FP16 contractions in the precision form:
// below it the LAD fixed point reached by the ADM moves by more than the
// tolerance under FP16 products (measured: p = 30 -> 2e-3, p = 50 -> 1.5e-7).
constexpr int kMinPHalf = 48;

// Automatic choice of the FP32 kernel form for `tiles` 16-regression tiles
// of class (PT, KS) on `ncu` compute units.  The tile form gives each SIMD
// whole tiles (a workgroup of four tile waves per CU slot), the split form a
// quarter of a tile per wave (one tile per workgroup).  Compare the
// contraction work of the busiest SIMD: ceil(tiles / 4 / ncu) tiles of PT
// element tiles against ceil(tiles / ncu) waves of ceil(PT / 4); the split
// form must win by a quarter to pay for its exchange and barrier per step.
bool choose_split(int PT, int KS, int64_t tiles, int ncu)
{
    if (!split_built(PT, KS) || ncu < 1 || tiles < 1) return false;
    const int64_t tile_blocks = (tiles + kWavesPerBlock - 1) / kWavesPerBlock;
    const int64_t busiest_tile = (tile_blocks + ncu - 1) / ncu * PT;
    const int64_t busiest_split = (tiles + ncu - 1) / ncu * ((PT + kWavesPerBlock - 1) / kWavesPerBlock);
    return 5 * busiest_split <= 4 * busiest_tile;
}

} // namespace

bool filter_supported(rpca_ctx *ctx, int p, int r, int precision)
{
    if (p < 1 || r < 1) return false;
    if (precision == 1 && p < kMinPHalf) precision = 0;
    const int PT = pick_pt(p, precision), KS = pick_ks(r);
    if (PT < 0 || KS < 0) return false;
    if (precision == 1)
        return (half_form(PT) ? lds_bytes_f16q(PT, KS, 1) : lds_bytes_f16(PT, KS, false)) <= lds_limit(ctx);
    return (quarter_form(PT, 0) ? lds_bytes_q32(PT, KS, 1) : lds_bytes(PT, KS)) <= lds_limit(ctx);
}

int filter_form_of(rpca_ctx *ctx, int p, int r, int precision, int form, int64_t regs)
{
    if (precision == 1 && p >= kMinPHalf) return 0;
    const int PT = pick_pt(p, 0), KS = pick_ks(r);
    if (PT >= 0 && quarter_form(PT, 0)) return 3;
    if (PT < 0 || KS < 0 || form == 1 || !split_built(PT, KS)) return 1;
    if (form == 2) return 2;
    return choose_split(PT, KS, (regs + 15) / 16, ctx->num_cu) ? 2 : 1;
}

bool filter_same_class(int p0, int r0, int p1, int r1)
{
    // one class list serves both modes
    return pick_pt(p0, 1) == pick_pt(p1, 1) && pick_ks(r0) == pick_ks(r1);
}

int launch_filter(rpca_ctx *ctx, const FilterSide *sides, int nsides, const FilterConsts &c_in,
                  hipStream_t stream)
{
    if (nsides < 1 || nsides > 2) return set_status(ctx, RPCA_ERR_ARG, "filter: bad side count");
    // Two sides in one launch: the side whose tiles hold neighbouring
    // regressions (row regressions: 16 adjacent rows, so each gathered line
    // serves a whole tile) takes the low workgroup indices, which start first.
    // The first round of workgroups then waits on the cheap gather, and the
    // scattered one (a line per element of a column regression) runs beside
    // work already in progress.  Each side carries its own outputs, and a
    // result does not depend on where its tile sits in the grid.
    FilterSide ord[2];
    if (nsides == 2 && sides[1].reg_stride < sides[0].reg_stride) {
        ord[0] = sides[1];
        ord[1] = sides[0];
        sides = ord;
    }
    // FP16 contractions only where they keep the FP32 accuracy (p >= kMinPHalf);
    // smaller regressions stay FP32 in the precision form too.
    FilterConsts c = c_in;
    if (c.precision == 1 && sides[0].p < kMinPHalf) c.precision = 0;
    if (nsides == 2 && c_in.precision == 1 && (sides[0].p < kMinPHalf) != (sides[1].p < kMinPHalf)) {
        int st = launch_filter(ctx, &sides[0], 1, c_in, stream);
        if (st != RPCA_OK) return st;
        return launch_filter(ctx, &sides[1], 1, c_in, stream);
    }
    const int PT = pick_pt(sides[0].p, c.precision);
    const int KS = pick_ks(sides[0].r);
    for (int s = 0; s < nsides; ++s) {
        if (!filter_supported(ctx, sides[s].p, sides[s].r, c.precision))
            return set_status(ctx, RPCA_ERR_UNSUPPORTED,
                              "filter: p = " + std::to_string(sides[s].p) + ", r = " +
                                  std::to_string(sides[s].r) + " outside the built kernel classes");
        if (pick_pt(sides[s].p, c.precision) != PT || pick_ks(sides[s].r) != KS)
            return set_status(ctx, RPCA_ERR_ARG, "filter: fused sides must share a class");
    }
    FilterLaunch L{};
    L.c = c;
    L.frag32[0] = L.frag32[1] = nullptr;
    // workspace for x in fragment order: 16 PT floats per regression (padded to
    // tiles, and to tile pairs: the quarter-tile form keeps one x slot per tile
    // slot of its workgroups)
    size_t xoff[2] = {0, 0}, xtotal = 0;
    for (int s = 0; s < nsides; ++s) {
        xoff[s] = xtotal;
        xtotal += (size_t)((sides[s].nreg + 31) / 32 * 2) * PT * 256;
    }
    {
        int st = ensure_buf(ctx, ctx->xbuf_ws, xtotal * sizeof(float));
        if (st != RPCA_OK) return st;
    }
    const bool quarter = quarter_form(PT, c.precision);
    if (quarter || (c.precision == 1 && lds_bytes_f16(PT, KS, true) > lds_limit(ctx))) {
        // FP32 refresh fragments (and, in the FP32 quarter-tile form, those of
        // v = A w) do not fit next to the staged ones: build them in HBM
        const int RT = (KS + 3) / 4;
        const size_t per = (size_t)PT * RT * 256;
        int st = ensure_buf(ctx, ctx->frag_ws, per * nsides * sizeof(float));
        if (st != RPCA_OK) return st;
        for (int s = 0; s < nsides; ++s) {
            float *dst = static_cast<float *>(ctx->frag_ws.ptr) + per * s;
            hipLaunchKernelGGL(prep_frag32, dim3((unsigned)((per + 255) / 256)), dim3(256), 0, stream,
                               sides[s].A, sides[s].lda, sides[s].p, sides[s].r, PT, RT, dst);
            RPCA_HIP_TRY(ctx, hipGetLastError());
            L.frag32[s] = dst;
        }
        if (nsides == 1) L.frag32[1] = L.frag32[0];
    }
    // FP32 kernel form: the caller's choice, else from the tile count of the
    // whole call (plan_regs) or of this launch; beyond the tile classes always
    // the quarter-tile form (its grid is sized for it below), also where a
    // split class is built (PT 26, 32 at r <= 16)
    bool split = false;
    if (c.precision == 0 && c.form != 1 && split_built(PT, KS) && !quarter) {
        if (c.form == 2) {
            split = true;
        } else {
            int64_t tiles = 0;
            if (c.plan_regs > 0) tiles = (c.plan_regs + 15) / 16;
            else
                for (int s = 0; s < nsides; ++s) tiles += (sides[s].nreg + 15) / 16;
            split = choose_split(PT, KS, tiles, ctx->num_cu);
        }
    }
    // quarter-tile forms: persistent, one workgroup per CU, the CUs shared
    // between the sides in proportion to their tiles; two tiles per workgroup
    // where their LDS fits and the element indices fit 32 bits
    L.qtiles = 1;
    const size_t lds2 = c.precision == 1 ? lds_bytes_f16q(PT, KS, 2) : lds_bytes_q32(PT, KS, 2);
    if (quarter && lds2 <= lds_limit(ctx)) {
        bool fits = true;
        for (int s = 0; s < nsides; ++s) fits = fits && sides[s].elem_bound <= INT_MAX;
        if (fits) L.qtiles = 2;
    }
    int64_t all_units = 0;
    for (int s = 0; s < nsides; ++s) all_units += (sides[s].nreg + 16 * L.qtiles - 1) / (16 * L.qtiles);
    const int64_t ncu = ctx->num_cu > 0 ? ctx->num_cu : 256;
    int nblocks = 0;
    for (int s = 0; s < nsides; ++s) {
        L.side[s] = sides[s];
        L.side[s].xbuf = static_cast<float *>(ctx->xbuf_ws.ptr) + xoff[s];
        const int64_t tiles = (sides[s].nreg + 15) / 16;
        int64_t blocks;
        if (quarter) {
            // units of qtiles tiles
            const int64_t units = (sides[s].nreg + 16 * L.qtiles - 1) / (16 * L.qtiles);
            blocks = std::min<int64_t>(units, std::max<int64_t>(1, (ncu * units + all_units / 2) / std::max<int64_t>(all_units, 1)));
        } else {
            // tiles per workgroup: 1 (split form) or 4
            const int64_t per = split ? 1 : kWavesPerBlock;
            blocks = (tiles + per - 1) / per;
        }
        if (blocks > INT_MAX / 2) return set_status(ctx, RPCA_ERR_UNSUPPORTED, "filter: too many regressions");
        if (s == 0) L.nblocks0 = (int)blocks;
        nblocks += (int)blocks;
    }
    if (nsides == 1) L.side[1] = sides[0];
    if (nblocks == 0) return RPCA_OK;
    switch (PT) {
    case 1: return launch_filter_pt<1>(ctx, KS, L, nblocks, split, stream);
    case 2: return launch_filter_pt<2>(ctx, KS, L, nblocks, split, stream);
    case 3: return launch_filter_pt<3>(ctx, KS, L, nblocks, split, stream);
    case 4: return launch_filter_pt<4>(ctx, KS, L, nblocks, split, stream);
    case 5: return launch_filter_pt<5>(ctx, KS, L, nblocks, split, stream);
    case 7: return launch_filter_pt<7>(ctx, KS, L, nblocks, split, stream);
    case 8: return launch_filter_pt<8>(ctx, KS, L, nblocks, split, stream);
    case 10: return launch_filter_pt<10>(ctx, KS, L, nblocks, split, stream);
    case 13: return launch_filter_pt<13>(ctx, KS, L, nblocks, split, stream);
    case 16: return launch_filter_pt<16>(ctx, KS, L, nblocks, split, stream);
    case 19: return launch_filter_pt<19>(ctx, KS, L, nblocks, split, stream);
    case 26: return launch_filter_pt<26>(ctx, KS, L, nblocks, split, stream);
    case 32: return launch_filter_pt<32>(ctx, KS, L, nblocks, split, stream);
    default: return set_status(ctx, RPCA_ERR_UNSUPPORTED, "filter: p class not built");
    }
}
