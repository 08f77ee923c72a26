// The paper's whole system on a batch of stereo pairs of uneven sizes
// (Sec. III and Sec. IV-A): per pair, the reduction of both views, the
// coarse matcher -- ZNCC + SGM (Eqs. (1)-(6)), the paper's main one, or
// census + SGM --, optionally the single matching phase and the 3 x 3 median
// (Eq. (7), Sec. III-A3), and the Table I network.  Every launch of every
// pair goes onto the caller's stream in pair order, with no allocation and no
// host synchronisation, so that a call can be captured in one hipGraph and
// replayed; the pairs reuse one workspace sized for the largest pair.
#include "kernels.h"

namespace sv {
namespace {

struct PbLayout {
    size_t low_l, low_r, cen_l, cen_r, disp, disp2, sgm, smp, net, total;
    size_t sgm_bytes, smp_bytes, net_bytes;
};

PbLayout pb_layout(const sv_paper_desc &d, int H, int W, int D) {
    PbLayout L{};
    const int h = cdiv(H, d.factor), w = cdiv(W, d.factor);
    const size_t px = (size_t)h * w;
    size_t o = 0;
    L.low_l = o; o = align256(o + px);
    L.low_r = o; o = align256(o + px);
    L.cen_l = o; o = align256(o + px * 8);
    L.cen_r = o; o = align256(o + px * 8);
    L.disp = o;  o = align256(o + px);
    L.disp2 = o; o = align256(o + px);
    L.sgm_bytes = sv_sgm_workspace_bytes(1, h, w, D);
    L.sgm = o;   o = align256(o + L.sgm_bytes);
    L.smp_bytes = sv_smp_workspace_bytes(1, h, w);
    L.smp = o;   o = align256(o + L.smp_bytes);
    L.net_bytes = sv_tvae_workspace_bytes(d.dtype, d.factor, 1, H, W);
    L.net = o;   o = align256(o + L.net_bytes);
    L.total = o;
    return L;
}

sv_status pb_check(const sv_paper_desc *d) {
    if (!d) return SV_ERR_NULL;
    if (d->matcher != SV_MATCH_ZNCC_SGM && d->matcher != SV_MATCH_CENSUS_SGM) return SV_ERR_RANGE;
    if (d->factor < 1 || d->factor > 8 || d->median < 0 || d->median > 1) return SV_ERR_RANGE;
    if (d->dtype != SV_F32 && d->dtype != SV_BF16 && d->dtype != SV_F16) return SV_ERR_DTYPE;
    if (d->win_w < 1 || d->win_h < 1 || d->win_w % 2 == 0 || d->win_h % 2 == 0) return SV_ERR_RANGE;
    const int nbits = d->win_w * d->win_h - 1;
    if (nbits < 1 || nbits > 64 || d->win_w > 17 || d->win_h > 17) return SV_ERR_RANGE;
    if (d->P1 < 0 || d->P2 < d->P1) return SV_ERR_RANGE;
    if (d->matcher == SV_MATCH_ZNCC_SGM) {
        if (64 + d->P2 > 255) return SV_ERR_RANGE;
        if (!zncc_window_supported(d->win_w, d->win_h)) return SV_ERR_UNSUPPORTED;
    } else if (nbits + 1 + d->P2 > 255) {
        return SV_ERR_RANGE;
    }
    return SV_OK;
}

}  // namespace
}  // namespace sv

using namespace sv;

extern "C" {

size_t sv_paper_batch_workspace_bytes(const sv_paper_desc *desc, int max_H, int max_W, int max_D) {
    if (pb_check(desc) != SV_OK || max_H <= 0 || max_W <= 0 || max_D < 1 || max_D > 256) return 0;
    const PbLayout L = pb_layout(*desc, max_H, max_W, max_D);
    if (L.net_bytes == 0) return 0;
    return L.total;
}

sv_status sv_paper_batch(const sv_paper_desc *desc, const sv_pair *pairs, int n, const void *packed_w,
                         void *workspace, size_t ws_bytes, void *stream) {
    sv_status r = pb_check(desc);
    if (r != SV_OK) return r;
    if (!pairs || !packed_w || !workspace) return SV_ERR_NULL;
    if (n < 0) return SV_ERR_SHAPE;
    if ((uintptr_t)workspace % 256) return SV_ERR_RANGE;
    const sv_paper_desc &d = *desc;
    // every pair is checked before the first launch
    for (int i = 0; i < n; ++i) {
        const sv_pair &p = pairs[i];
        if (!p.left || !p.right || !p.out) return SV_ERR_NULL;
        if (p.H <= 0 || p.W <= 0 || p.H > 16384 || p.W > 16384 || p.D < 1 || p.D > 256) return SV_ERR_SHAPE;
        const PbLayout L = pb_layout(d, p.H, p.W, p.D);
        if (L.net_bytes == 0) return SV_ERR_SHAPE;
        if (L.total > ws_bytes) return SV_ERR_WORKSPACE;
    }
    char *ws = (char *)workspace;
    const hipStream_t st = (hipStream_t)stream;
    for (int i = 0; i < n; ++i) {
        const sv_pair &p = pairs[i];
        const PbLayout L = pb_layout(d, p.H, p.W, p.D);
        const int h = cdiv(p.H, d.factor), w = cdiv(p.W, d.factor);
        uint8_t *low_l = (uint8_t *)(ws + L.low_l), *low_r = (uint8_t *)(ws + L.low_r);
        uint64_t *cen_l = (uint64_t *)(ws + L.cen_l), *cen_r = (uint64_t *)(ws + L.cen_r);
        uint8_t *disp = (uint8_t *)(ws + L.disp);
        uint8_t *coarse = p.disp_low ? p.disp_low : (uint8_t *)(ws + L.disp2);
        // reduction of both views (and their census words, for census + SGM)
        r = launch_reduce_census(p.left, p.right, 1, p.H, p.W, p.W, d.factor, d.win_w, d.win_h, low_l, low_r,
                                 cen_l, cen_r, st);
        if (r != SV_OK) return r;
        uint8_t *matched = d.median ? disp : coarse;
        if (d.matcher == SV_MATCH_ZNCC_SGM)
            r = sv_zncc_sgm(low_l, low_r, 1, h, w, p.D, d.win_w, d.win_h, d.P1, d.P2, matched, ws + L.sgm,
                            L.sgm_bytes, stream);
        else
            r = sv_sgm(cen_l, cen_r, 1, h, w, p.D, d.win_w * d.win_h - 1, d.P1, d.P2, matched, ws + L.sgm,
                       L.sgm_bytes, stream);
        if (r != SV_OK) return r;
        if (d.median) {
            r = sv_smp_median(disp, 1, h, w, p.D, coarse, ws + L.smp, L.smp_bytes, stream);
            if (r != SV_OK) return r;
        }
        r = sv_tvae_forward(d.dtype, d.factor, packed_w, coarse, low_l, 1, p.H, p.W, nullptr, p.out, nullptr,
                            ws + L.net, L.net_bytes, stream);
        if (r != SV_OK) return r;
    }
    return SV_OK;
}

}  // extern "C"
