// Batches of uneven pairs through the whole path, and the tile autotuner.
//
// A plan owns flattened per-level buffers sized for max_n pairs of the largest
// size, a pinned host copy and a device copy of the pair table, and a hipGraph
// of the 12 stage launches (census, cost + WTA, 9 network convolutions, final
// gather).  Every launch is persistent: a fixed grid walks that stage's tiles
// of all pairs through the table's prefix sums, so the same graph serves any
// mix of sizes up to the plan's maxima.  A call writes the table for its
// pairs, copies it to the device on the caller's stream and replays the graph.
#include <errno.h>
#include <math.h>
#include <sys/stat.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <string>
#include <vector>

#include "net.h"
#include "prof.h"

namespace sv {

int cost_wta_split_for(int B, int h, int w, int D);
void cost_wta_split_tuned(int B, int h, int w, int D, int d);
int cost_wta_split_override();

static const int kStageGridMax = 1024;

// Pinned host copies of the pair table a plan cycles through: a call waits
// on the host only when the copy it takes is still being uploaded by the call
// SV_TAB_RING calls earlier.
#define SV_TAB_RING 4

}  // namespace sv

using namespace sv;

struct sv_batch_plan {
    NetShape ns;
    sv_vae_desc desc;
    int max_n, max_H, max_W, max_D, win_w, win_h, nbits;
    int dsplit;
    int cen_th;  // census tile height (4 or 16)
    int fin_th;  // final gather tile height (16, 32 or 64)
    int cfg[NLAYERS];
    int grid[BS_NSTAGES];
    size_t cap[4];
    void *dev;
    PairTable *tab_dev;
    PairTable *tab_host[SV_TAB_RING];    // pinned staging copies, used in turn
    hipEvent_t tab_done[SV_TAB_RING];    // recorded after the upload from that copy
    bool tab_pending[SV_TAB_RING];
    unsigned long long calls;
    uint64_t *cl, *cr;
    uint8_t *low, *disp;
    void *E1, *E2, *E3, *G3, *G2, *G1, *G0;
    float *ML;
    hipStream_t cap_stream;
    hipGraph_t graph;
    hipGraphExec_t exec;
    const void *graph_w;
};

namespace sv {

// ---------------------------------------------------------------------------
// Autotune cache: a text file, one entry per line
//   gfx950|dt<dtype>|c<c1>,<c2>,<c3>|L<latent>|f<factor>|B<batch>|<H>x<W> <dsplit> <name0>,...,<name8>
// with the layers' configurations by name (sv_conv_cfg_name), loaded once per
// process into memory; lookups take the entry of the same network and image
// size with the nearest batch size.  A line that does not parse, or names a
// configuration this library does not have, is ignored.
// ---------------------------------------------------------------------------
struct TuneEntry {
    int dt, c1, c2, c3, L, f, B, H, W, dsplit, cfg[NLAYERS];
};
static std::mutex g_tune_mu;
static std::vector<TuneEntry> g_tune;
static bool g_tune_loaded = false;

static std::string cache_path() {
    const char *e = getenv("SV_AUTOTUNE_CACHE");
    if (e && *e) return e;
    const char *home = getenv("HOME");
    return std::string(home ? home : "/tmp") + "/.cache/sv_autotune.tsv";
}

static int cfg_by_name(const std::string &name) {
    for (int c = 0; c < conv_num_cfgs(); ++c)
        if (name == conv_cfg_name(c)) return c;
    return -1;
}

static bool parse_entry(const char *line, TuneEntry &t) {
    char names[400];
    const int m = sscanf(line, "gfx950|dt%d|c%d,%d,%d|L%d|f%d|B%d|%dx%d %d %399s", &t.dt, &t.c1, &t.c2,
                         &t.c3, &t.L, &t.f, &t.B, &t.H, &t.W, &t.dsplit, names);
    if (m != 11) return false;
    bool ok = (t.dsplit == 1 || t.dsplit == 2 || t.dsplit == 4 || t.dsplit == 8) && t.B > 0;
    std::string rest(names);
    size_t pos = 0;
    for (int i = 0; i < NLAYERS && ok; ++i) {
        const size_t comma = rest.find(',', pos);
        const bool last = i == NLAYERS - 1;
        if (last != (comma == std::string::npos)) return false;
        t.cfg[i] = cfg_by_name(rest.substr(pos, last ? std::string::npos : comma - pos));
        ok = t.cfg[i] >= 0;
        pos = comma + 1;
    }
    return ok;
}

static void format_entry(const TuneEntry &t, char *buf, size_t n) {
    int k = snprintf(buf, n, "gfx950|dt%d|c%d,%d,%d|L%d|f%d|B%d|%dx%d\t%d\t", t.dt, t.c1, t.c2, t.c3,
                     t.L, t.f, t.B, t.H, t.W, t.dsplit);
    for (int i = 0; i < NLAYERS && k > 0 && (size_t)k < n; ++i)
        k += snprintf(buf + k, n - k, "%s%s", conv_cfg_name(t.cfg[i]), i + 1 < NLAYERS ? "," : "\n");
}

static bool same_key(const TuneEntry &a, const TuneEntry &b, bool with_batch) {
    return a.dt == b.dt && a.c1 == b.c1 && a.c2 == b.c2 && a.c3 == b.c3 && a.L == b.L && a.f == b.f &&
           a.H == b.H && a.W == b.W && (!with_batch || a.B == b.B);
}

// caller holds g_tune_mu
static void load_cache_locked() {
    if (g_tune_loaded) return;
    g_tune_loaded = true;
    FILE *f = fopen(cache_path().c_str(), "r");
    if (!f) return;
    char line[512];
    bool corrupt = false;
    while (fgets(line, sizeof line, f)) {
        TuneEntry t;
        if (parse_entry(line, t))
            g_tune.push_back(t);
        else if (line[0] != '\n')
            corrupt = true;
    }
    fclose(f);
    if (corrupt)
        fprintf(stderr, "sv: ignoring malformed lines in autotune cache %s\n", cache_path().c_str());
}

static TuneEntry make_key(const NetShape &ns, int B, int H, int W) {
    TuneEntry k{};
    k.dt = ns.dtype; k.c1 = ns.c1; k.c2 = ns.c2; k.c3 = ns.c3; k.L = ns.L; k.f = ns.f;
    k.B = B; k.H = H; k.W = W;
    return k;
}

bool tuned_lookup(const NetShape &ns, int B, int H, int W, int *cfg, int *dsplit) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    load_cache_locked();
    const TuneEntry key = make_key(ns, B, H, W);
    const TuneEntry *best = nullptr;
    double bd = 1e30;
    for (const TuneEntry &t : g_tune) {
        if (!same_key(t, key, false)) continue;
        const double d = fabs(log((double)t.B / (double)B));
        if (d < bd) { bd = d; best = &t; }
    }
    if (!best) return false;
    for (int i = 0; i < NLAYERS; ++i) cfg[i] = best->cfg[i];
    if (dsplit) *dsplit = best->dsplit;
    return true;
}

static void cache_store(const TuneEntry &e) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    load_cache_locked();
    for (auto it = g_tune.begin(); it != g_tune.end();)
        it = same_key(*it, e, true) ? g_tune.erase(it) : it + 1;
    g_tune.push_back(e);
    const std::string path = cache_path();
    const size_t slash = path.rfind('/');
    if (slash != std::string::npos) (void)mkdir(path.substr(0, slash).c_str(), 0755);
    const std::string tmp = path + ".tmp";
    FILE *f = fopen(tmp.c_str(), "w");
    if (!f) return;
    char buf[512];
    for (const TuneEntry &t : g_tune) {
        format_entry(t, buf, sizeof buf);
        fputs(buf, f);
    }
    fclose(f);
    rename(tmp.c_str(), path.c_str());
}

// ---------------------------------------------------------------------------
// Plan helpers
// ---------------------------------------------------------------------------
static int conv_tiles(int cfg, int Ho, int Wo, int Cout) {
    int TH, TN;
    conv_cfg_tile(cfg, TH, TN);
    return cdiv(Wo, 16) * cdiv(Ho, TH) * cdiv(Cout, TN);
}

// The conv layers' stage ids, output level, input level and output channels.
struct LayerRun { int li, stage, in_level, out_level; };
static const LayerRun kRuns[9] = {
    {L_E1, BS_E1, 0, 1}, {L_E2, BS_E2, 1, 2}, {L_E3, BS_E3, 2, 3}, {L_HEAD, BS_HEAD, 3, 3},
    {L_G3, BS_G3, 3, 3}, {L_G2, BS_G2, 2, 2}, {L_G1, BS_G1, 1, 1}, {L_G0, BS_G0, 0, 0},
    {L_F, BS_FPROJ, 0, 0},
};

static int run_cout(const NetShape &ns, int li) { return li == L_F ? 9 : ns.ly[li].cout; }

// Tiles of every stage for one pair.
static void pair_tiles(const sv_batch_plan *pl, const PairGeo &g, int *tiles) {
    tiles[BS_CENSUS] = 2 * cdiv(g.w[0], CEN_TILE_W) * cdiv(g.h[0], pl->cen_th);
    tiles[BS_COST_WTA] = g.h[0] * cdiv(g.w[0], cost_wta_tile_width(pl->dsplit));
    for (const LayerRun &r : kRuns)
        tiles[r.stage] = conv_tiles(pl->cfg[r.li], g.h[r.out_level], g.w[r.out_level],
                                    run_cout(pl->ns, r.li));
    tiles[BS_E1] = enc1_tiles(g.h[1], g.w[1]);  // E1 runs as a direct stencil
    // the final layer: the gather's tiles when G0 projects, else k_final's
    const int final_tile_h = net_projects(pl->ns, false) ? pl->fin_th : FIN_TILE_H;
    tiles[BS_FINAL] = cdiv(g.W, FIN_TILE_W) * cdiv(g.H, final_tile_h);
}

static void fill_geo(const NetShape &ns, int H, int W, PairGeo &g) {
    const Levels lv = net_levels(ns, H, W);
    g.H = H; g.W = W;
    for (int k = 0; k < 4; ++k) { g.h[k] = lv.h[k]; g.w[k] = lv.w[k]; }
}

static ConvSrc tsrc(const void *p, int kind, int C, int pitch, int level, int sdt) {
    ConvSrc s{};
    s.ptr = p; s.kind = kind; s.C = C; s.pitch = pitch; s.level = level; s.sdt = sdt;
    return s;
}

// Enqueues the 12 stage launches of a plan on `st`.
static sv_status enqueue_stages(sv_batch_plan *pl, const void *packed, hipStream_t st) {
    const NetShape &ns = pl->ns;
    const int c1 = ns.c1, c2 = ns.c2, c3 = ns.c3, L = ns.L;
    sv_status r = launch_reduce_census_tab(pl->tab_dev, pl->grid[BS_CENSUS], ns.f, pl->cen_th,
                                           pl->win_w, pl->win_h, pl->low, pl->cl, pl->cr, st);
    if (r != SV_OK) return r;
    r = launch_cost_wta_tab(pl->tab_dev, pl->grid[BS_COST_WTA], pl->cl, pl->cr, pl->nbits, pl->disp,
                            pl->dsplit, st);
    if (r != SV_OK) return r;
    ConvSrc x0{};
    x0.ptr = pl->disp; x0.img = pl->low; x0.kind = SRC_X0; x0.C = 2; x0.level = 0;
    x0.scale0 = (float)ns.f / 256.0f;
    const ConvSrc none{};
    struct In { ConvSrc s0, s1; void *out; int pitch, f32, act; };
    const In ins[8] = {
        {x0, none, pl->E1, c1, 0, 1},
        {tsrc(pl->E1, SRC_TENSOR, c1, c1, 1, 0), none, pl->E2, c2, 0, 1},
        {tsrc(pl->E2, SRC_TENSOR, c2, c2, 2, 0), none, pl->E3, c3, 0, 1},
        {tsrc(pl->E3, SRC_TENSOR, c3, c3, 3, 0), none, pl->ML, 2 * L, 1, 0},
        {tsrc(pl->ML, SRC_TENSOR, L, 2 * L, 3, SDT_F32), none, pl->G3, c3, 0, 1},
        {tsrc(pl->G3, SRC_RESIZE, c3, c3, 3, 0), tsrc(pl->E2, SRC_TENSOR, c2, c2, 2, 0), pl->G2, c2, 0, 1},
        {tsrc(pl->G2, SRC_RESIZE, c2, c2, 2, 0), tsrc(pl->E1, SRC_TENSOR, c1, c1, 1, 0), pl->G1, c1, 0, 1},
        {tsrc(pl->G1, SRC_RESIZE, c1, c1, 1, 0), x0, pl->G0, c1, 0, 1},
    };
    r = launch_enc1_tab(ns.dtype, pl->tab_dev, pl->grid[BS_E1], pl->disp, pl->low, x0.scale0, c1,
                        (const char *)packed + ns.w_off[L_E1], ns.n_pad[L_E1], ns.cin_pad[L_E1],
                        (const float *)((const char *)packed + ns.b_off[L_E1]), pl->E1, st);
    if (r != SV_OK) return r;
    // the final layer's projection runs inside the final gather
    for (int k = 1; k < 8; ++k) {
        const LayerRun &run = kRuns[k];
        const int li = run.li;
        ConvParams p{};
        p.src[0] = ins[k].s0; p.src[1] = ins[k].s1;
        p.Cin = ins[k].s0.C + (ins[k].s1.kind ? ins[k].s1.C : 0);
        p.Cout = run_cout(ns, li);
        p.cin_pad = ns.cin_pad[li]; p.n_pad = ns.n_pad[li];
        p.wpk = (const char *)packed + ns.w_off[li];
        p.bias = li == L_F ? nullptr : (const float *)((const char *)packed + ns.b_off[li]);
        p.out = ins[k].out; p.out_pitch = ins[k].pitch; p.out_f32 = ins[k].f32; p.act = ins[k].act;
        p.tab = pl->tab_dev; p.stage = run.stage; p.in_level = run.in_level; p.out_level = run.out_level;
        if (li == L_G0 && net_projects(ns, false)) {
            // G0's epilogue writes the final layer's tap projections (FP32
            // planes of cap[0] pixels) into G0's buffer
            p.proj_w = (const float *)((const char *)packed + ns.w_off[L_F]);
            p.proj_pitch = ns.cin_pad[L_F];
            p.proj_out = (float *)pl->G0;
            p.proj_plane = (long long)pl->cap[0];
            p.proj_disp = pl->disp;
            p.proj_img = pl->low;
            p.proj_scale0 = x0.scale0;
        }
        const int ks = li == L_F ? 1 : ns.ly[li].k, stride = li == L_F ? 1 : ns.ly[li].stride;
        r = launch_conv_tab(li == L_F ? SV_F32 : ns.dtype, ks, stride, pl->cfg[li], p,
                            pl->grid[run.stage], st);
        if (r != SV_OK) return r;
    }
    if (net_projects(ns, false))
        return launch_final_gather_tab(pl->tab_dev, pl->grid[BS_FINAL], (const float *)pl->G0,
                                       (long long)pl->cap[0], pl->disp, ns.f, pl->fin_th,
                                       (const float *)((const char *)packed + ns.b_off[L_F]), st);
    return launch_final_tab(pl->tab_dev, pl->grid[BS_FINAL], ns.dtype, pl->G0, c1, pl->disp, pl->low,
                            (const float *)((const char *)packed + ns.w_off[L_F]), ns.cin_pad[L_F],
                            ns.f, (const float *)((const char *)packed + ns.b_off[L_F]), st);
}

static void destroy_graph(sv_batch_plan *pl) {
    if (pl->exec) (void)hipGraphExecDestroy(pl->exec);
    if (pl->graph) (void)hipGraphDestroy(pl->graph);
    pl->exec = nullptr;
    pl->graph = nullptr;
    pl->graph_w = nullptr;
}

static sv_status capture(sv_batch_plan *pl, const void *packed) {
    destroy_graph(pl);
    SV_HIP(hipStreamBeginCapture(pl->cap_stream, hipStreamCaptureModeThreadLocal));
    sv_status r = enqueue_stages(pl, packed, pl->cap_stream);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(pl->cap_stream, &g);
    if (r != SV_OK) {
        if (g) (void)hipGraphDestroy(g);
        return r;
    }
    if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
    pl->graph = g;
    SV_HIP(hipGraphInstantiate(&pl->exec, g, nullptr, nullptr, 0));
    pl->graph_w = packed;
    return SV_OK;
}

static bool graph_disabled() {
    const char *e = getenv("SV_DISABLE_GRAPH");
    return e && e[0] == '1';
}

}  // namespace sv

extern "C" {

sv_status sv_batch_plan_create(const sv_vae_desc *desc, int max_n, int max_H, int max_W,
                               int max_D, int win_w, int win_h, sv_batch_plan **plan_out) {
    if (!plan_out) return SV_ERR_NULL;
    *plan_out = nullptr;
    NetShape ns;
    sv_status r = net_shape(desc, ns);
    if (r != SV_OK) return r;
    if (ns.dtype == SV_I8) return SV_ERR_UNSUPPORTED;  // INT8: sv_vae_forward only
    if (max_n < 1 || max_n > SV_MAXN || max_H < 1 || max_W < 1 || max_H > 16384 || max_W > 16384)
        return SV_ERR_SHAPE;
    if (max_D < 1 || max_D > 256) return SV_ERR_RANGE;
    if (win_w < 1 || win_h < 1 || win_w % 2 == 0 || win_h % 2 == 0 || win_w > 17 || win_h > 17 ||
        win_w * win_h - 1 > 64 || win_w * win_h - 1 < 1)
        return SV_ERR_RANGE;

    sv_batch_plan *pl = new sv_batch_plan();
    memset((void *)pl, 0, sizeof(*pl));
    pl->ns = ns;
    pl->desc = *desc;
    pl->max_n = max_n; pl->max_H = max_H; pl->max_W = max_W; pl->max_D = max_D;
    pl->win_w = win_w; pl->win_h = win_h; pl->nbits = win_w * win_h - 1;
    // tile shapes: the autotune cache, else the single-call defaults
    const Levels mx = net_levels(ns, max_H, max_W);
    pl->dsplit = cost_wta_split_for(max_n, mx.h[0], mx.w[0], max_D);
    pl->cen_th = census_tile_height(max_n, mx.h[0], mx.w[0]);
    pl->fin_th = gather_tile_h(ns.f, (long long)max_n * max_H * max_W);
    for (int i = 0; i < NLAYERS; ++i) {
        const int lvl = i == L_E1 ? 1 : (i == L_E2 ? 2 : (i <= L_G3 ? 3 : (i == L_G2 ? 2 : (i == L_G1 ? 1 : 0))));
        pl->cfg[i] = net_default_cfg(ns, i, mx.h[lvl] * mx.w[lvl]);
    }
    int ds;
    int cfg[NLAYERS];
    if (tuned_lookup(ns, max_n, max_H, max_W, cfg, &ds)) {
        pl->dsplit = cost_wta_split_override() > 0 ? cost_wta_split_override() : ds;
        for (int i = 0; i < NLAYERS; ++i) {
            const int ov = net_get_cfg_override(ns.dtype, i);
            pl->cfg[i] = ov >= 0 ? ov : cfg[i];
        }
    }
    for (int i = 0; i < L_F; ++i)
        pl->cfg[i] = conv_resolve_cfg(ns.dtype, ns.ly[i].k, ns.ly[i].stride, conv_persistent_cfg(pl->cfg[i]));
    if (net_projects(ns, false)) pl->cfg[L_G0] = net_g0_proj_cfg(ns, pl->cfg[L_G0]);
    // capacities and persistent grid sizes from the largest pair
    for (int k = 0; k < 4; ++k) pl->cap[k] = (size_t)max_n * mx.h[k] * mx.w[k];
    PairGeo gmax{};
    fill_geo(ns, max_H, max_W, gmax);
    gmax.D = max_D;
    int tiles[BS_NSTAGES];
    pair_tiles(pl, gmax, tiles);
    for (int s = 0; s < BS_NSTAGES; ++s) {
        const long long t = (long long)tiles[s] * max_n;
        pl->grid[s] = (int)(t < kStageGridMax ? t : kStageGridMax);
        if (pl->grid[s] < 1) pl->grid[s] = 1;
    }
    // one device allocation for every buffer
    const int es = ns.es;
    size_t off = 0;
    auto take = [&](size_t bytes) { size_t o = off; off = align256(off + bytes); return o; };
    const size_t o_tab = take(sizeof(PairTable));
    const size_t o_cl = take(pl->cap[0] * 8), o_cr = take(pl->cap[0] * 8);
    const size_t o_low = take(pl->cap[0]), o_disp = take(pl->cap[0]);
    const size_t o_E1 = take(pl->cap[1] * ns.c1 * es), o_E2 = take(pl->cap[2] * ns.c2 * es);
    const size_t o_E3 = take(pl->cap[3] * ns.c3 * es), o_ML = take(pl->cap[3] * 2 * ns.L * 4);
    const size_t o_G3 = take(pl->cap[3] * ns.c3 * es), o_G2 = take(pl->cap[2] * ns.c2 * es);
    const size_t o_G1 = take(pl->cap[1] * ns.c1 * es);
    const size_t o_G0 = take(pl->cap[0] * std::max<size_t>((size_t)ns.c1 * es, 9 * sizeof(float)));
    hipError_t e = hipMalloc(&pl->dev, off);
    if (e != hipSuccess) {
        delete pl;
        return hip_fail(e, "hipMalloc(batch plan)");
    }
    char *d = (char *)pl->dev;
    pl->tab_dev = (PairTable *)(d + o_tab);
    pl->cl = (uint64_t *)(d + o_cl); pl->cr = (uint64_t *)(d + o_cr);
    pl->low = (uint8_t *)(d + o_low); pl->disp = (uint8_t *)(d + o_disp);
    pl->E1 = d + o_E1; pl->E2 = d + o_E2; pl->E3 = d + o_E3; pl->ML = (float *)(d + o_ML);
    pl->G3 = d + o_G3; pl->G2 = d + o_G2; pl->G1 = d + o_G1; pl->G0 = d + o_G0;
    e = hipStreamCreateWithFlags(&pl->cap_stream, hipStreamNonBlocking);
    for (int k = 0; k < SV_TAB_RING && e == hipSuccess; ++k) {
        e = hipHostMalloc((void **)&pl->tab_host[k], sizeof(PairTable), hipHostMallocDefault);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&pl->tab_done[k], hipEventDisableTiming);
    }
    if (e != hipSuccess) {
        sv_batch_plan_destroy(pl);
        return hip_fail(e, "batch plan resources");
    }
    *plan_out = pl;
    return SV_OK;
}

sv_status sv_batch_plan_destroy(sv_batch_plan *pl) {
    if (!pl) return SV_OK;
    for (int k = 0; k < SV_TAB_RING; ++k)
        if (pl->tab_pending[k]) (void)hipEventSynchronize(pl->tab_done[k]);
    destroy_graph(pl);
    for (int k = 0; k < SV_TAB_RING; ++k) {
        if (pl->tab_done[k]) (void)hipEventDestroy(pl->tab_done[k]);
        if (pl->tab_host[k]) (void)hipHostFree(pl->tab_host[k]);
    }
    if (pl->cap_stream) (void)hipStreamDestroy(pl->cap_stream);
    if (pl->dev) (void)hipFree(pl->dev);
    delete pl;
    return SV_OK;
}

sv_status sv_stereo_batch(sv_batch_plan *pl, const sv_pair *pairs, int n, const void *packed_w,
                          void *stream) {
    if (!pl || !pairs || !packed_w) return SV_ERR_NULL;
    if (n < 1 || n > pl->max_n) return SV_ERR_SHAPE;
    if ((uintptr_t)packed_w % 256) return SV_ERR_RANGE;
    for (int i = 0; i < n; ++i) {
        const sv_pair &p = pairs[i];
        if (!p.left || !p.right || !p.out) return SV_ERR_NULL;
        if (p.H < 1 || p.W < 1 || p.H > pl->max_H || p.W > pl->max_W) return SV_ERR_SHAPE;
        if (p.D < 1 || p.D > pl->max_D) return SV_ERR_RANGE;
    }
    hipStream_t st = (hipStream_t)stream;
    // the next pinned copy in turn; it may still be read by the upload of the
    // call SV_TAB_RING calls ago, the only case in which the host waits
    const int slot = (int)(pl->calls % SV_TAB_RING);
    if (pl->tab_pending[slot]) {
        SV_HIP(hipEventSynchronize(pl->tab_done[slot]));
        pl->tab_pending[slot] = false;
    }
    PairTable *t = pl->tab_host[slot];
    t->n = n;
    long long off[4] = {0, 0, 0, 0};
    for (int s = 0; s < BS_NSTAGES; ++s) t->cum[s][0] = 0;
    for (int i = 0; i < n; ++i) {
        PairGeo &g = t->pair[i];
        memset(&g, 0, sizeof g);
        fill_geo(pl->ns, pairs[i].H, pairs[i].W, g);
        g.D = pairs[i].D;
        for (int k = 0; k < 4; ++k) {
            g.off[k] = off[k];
            off[k] += (long long)g.h[k] * g.w[k];
        }
        g.left = pairs[i].left; g.right = pairs[i].right; g.out = pairs[i].out;
        g.disp_out = pairs[i].disp_low;
        int tiles[BS_NSTAGES];
        pair_tiles(pl, g, tiles);
        for (int s = 0; s < BS_NSTAGES; ++s) t->cum[s][i + 1] = t->cum[s][i] + tiles[s];
    }
    const size_t bytes = offsetof(PairTable, pair) + sizeof(PairGeo) * (size_t)n;
    // the device table is single: stream order puts this upload after the
    // previous call's kernels on the same stream
    SV_HIP(hipMemcpyAsync(pl->tab_dev, t, bytes, hipMemcpyHostToDevice, st));
    SV_HIP(hipEventRecord(pl->tab_done[slot], st));
    pl->tab_pending[slot] = true;
    ++pl->calls;
    if (graph_disabled()) return enqueue_stages(pl, packed_w, st);
    if (!pl->exec || pl->graph_w != packed_w) {
        sv_status r = capture(pl, packed_w);
        if (r != SV_OK) {
            destroy_graph(pl);
            return enqueue_stages(pl, packed_w, st);  // the same launches, eager
        }
    }
    SV_HIP(hipGraphLaunch(pl->exec, st));
    return SV_OK;
}

// ---------------------------------------------------------------------------
// Autotuner: times every tile shape of every stage on a uniform batch of the
// given shape and keeps the fastest (all shapes give bitwise-equal results).
// ---------------------------------------------------------------------------
__global__ void k_zero_f32(float *p, size_t n) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        p[i] = 0.f;
}

__global__ void k_fill_pattern(uint8_t *p, size_t n, uint32_t seed) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        uint32_t x = (uint32_t)i * 2654435761u ^ seed;
        x ^= x >> 15; x *= 2246822519u; x ^= x >> 13;
        p[i] = (uint8_t)(x >> 24);
    }
}

sv_status sv_autotune(const sv_vae_desc *desc, int B, int H, int W, int D, int win_w, int win_h) {
    NetShape ns;
    sv_status r = net_shape(desc, ns);
    if (r != SV_OK) return r;
    if (B < 1 || H < 1 || W < 1 || H > 16384 || W > 16384) return SV_ERR_SHAPE;
    if (D < 1 || D > 256) return SV_ERR_RANGE;
    const size_t ws = sv_vae_workspace_bytes(desc, B, H, W);
    const int h = cdiv(H, ns.f), w = cdiv(W, ns.f);
    const size_t nimg = (size_t)B * H * W, nlow = (size_t)B * h * w;
    // one scratch allocation: images, census, low, disp, out, packed weights, params, workspace
    size_t off = 0;
    auto take = [&](size_t bytes) { size_t o = off; off = align256(off + bytes); return o; };
    const size_t o_l = take(nimg), o_r = take(nimg), o_cl = take(nlow * 8), o_cr = take(nlow * 8);
    const size_t o_low = take(nlow), o_disp = take(nlow), o_out = take(nimg * 4);
    const size_t o_pk = take(ns.packed_bytes), o_par = take((size_t)ns.nparams * 4), o_ws = take(ws);
    void *mem = nullptr;
    SV_HIP(hipMalloc(&mem, off));
    char *d = (char *)mem;
    hipStream_t st = nullptr;
    hipLaunchKernelGGL(k_fill_pattern, dim3(1024), dim3(256), 0, st, (uint8_t *)(d + o_l), nimg, 1u);
    hipLaunchKernelGGL(k_fill_pattern, dim3(1024), dim3(256), 0, st, (uint8_t *)(d + o_r), nimg, 2u);
    hipLaunchKernelGGL(k_zero_f32, dim3(256), dim3(256), 0, st, (float *)(d + o_par), (size_t)ns.nparams);
    r = net_pack(ns, (const float *)(d + o_par), d + o_pk, st);
    const int reps = 8;
    int best_ds = 4;
    // the configurations under test travel with each forward call (cur), so
    // tuning changes no process-wide setting and other threads' calls are
    // unaffected
    int best_cfg[NLAYERS], cur[NLAYERS];
    for (int i = 0; i < NLAYERS; ++i) best_cfg[i] = cur[i] = net_heuristic_cfg(ns, i);
    if (r == SV_OK) {
        // census once, then every lane split of the cost + WTA kernel
        r = launch_reduce_census((uint8_t *)(d + o_l), (uint8_t *)(d + o_r), B, H, W, W, ns.f, win_w,
                                 win_h, (uint8_t *)(d + o_low), nullptr, (uint64_t *)(d + o_cl),
                                 (uint64_t *)(d + o_cr), st);
        float best = 1e30f;
        const int splits[4] = {1, 2, 4, 8};
        for (int k = 0; k < 4 && r == SV_OK; ++k) {
            hipEvent_t a, b;
            (void)hipEventCreate(&a);
            (void)hipEventCreate(&b);
            (void)hipEventRecord(a, st);
            for (int i = 0; i < reps && r == SV_OK; ++i)
                r = launch_cost_wta((uint64_t *)(d + o_cl), (uint64_t *)(d + o_cr), B, h, w, D,
                                    win_w * win_h - 1, (uint8_t *)(d + o_disp), splits[k], st);
            (void)hipEventRecord(b, st);
            (void)hipEventSynchronize(b);
            float t = 0.f;
            (void)hipEventElapsedTime(&t, a, b);
            (void)hipEventDestroy(a);
            (void)hipEventDestroy(b);
            if (t < best) { best = t; best_ds = splits[k]; }
        }
        const char *ve = getenv("SV_AUTOTUNE_VERBOSE");
        const bool verbose = ve && ve[0] == '1';
        // Stage 1, screening: each layer alone, every configuration, timed over
        // back-to-back launches of that one layer (on buffers a full forward
        // pass has filled); the fastest few per layer go on to stage 2.
        // Stage 2, in context: a whole forward pass captured in a graph and
        // replayed back to back, one layer's candidate varied at a time with
        // the others at their current best (layer by layer, twice over), so
        // effects a lone layer does not show (inputs fresh from the previous
        // layer, the extra launch of a split reduction) count.
        constexpr int NKEEP = 5;
        int keep[NLAYERS][NKEEP], nkeep[NLAYERS] = {};
        auto fwd_on = [&](hipStream_t s_, int only) {
            return net_forward(ns, d + o_pk, (uint8_t *)(d + o_disp), (uint8_t *)(d + o_low), B, H, W,
                               nullptr, (float *)(d + o_out), nullptr, nullptr, d + o_ws, s_, only, cur);
        };
        auto fwd = [&](int only) { return fwd_on(st, only); };
        // mean time per replay of a graph holding one whole forward pass, best
        // of two rounds (ms); the graph keeps launch overhead out of the timing
        hipStream_t cs = nullptr;
        if (r == SV_OK && hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) != hipSuccess)
            r = hip_fail(hipGetLastError(), "hipStreamCreateWithFlags");
        auto graph_timed = [&](int reps_) {
            float t = 1e30f;
            hipGraph_t g = nullptr;
            hipGraphExec_t ge = nullptr;
            if (r != SV_OK) return t;
            hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
            if (e != hipSuccess) { r = hip_fail(e, "hipStreamBeginCapture"); return t; }
            const sv_status rf = fwd_on(cs, -1);
            e = hipStreamEndCapture(cs, &g);
            if (rf != SV_OK) r = rf;
            else if (e != hipSuccess) r = hip_fail(e, "hipStreamEndCapture");
            if (r == SV_OK && (e = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0)) != hipSuccess)
                r = hip_fail(e, "hipGraphInstantiate");
            for (int round = 0; round < 2 && r == SV_OK; ++round) {
                for (int k = 0; k < 2; ++k) (void)hipGraphLaunch(ge, cs);
                hipEvent_t ea, eb;
                (void)hipEventCreate(&ea);
                (void)hipEventCreate(&eb);
                (void)hipEventRecord(ea, cs);
                for (int k = 0; k < reps_; ++k) (void)hipGraphLaunch(ge, cs);
                (void)hipEventRecord(eb, cs);
                if ((e = hipEventSynchronize(eb)) != hipSuccess) r = hip_fail(e, "autotune graph replay");
                float ms_ = 0.f;
                (void)hipEventElapsedTime(&ms_, ea, eb);
                (void)hipEventDestroy(ea);
                (void)hipEventDestroy(eb);
                t = std::min(t, ms_ / reps_);
            }
            if (ge) (void)hipGraphExecDestroy(ge);
            if (g) (void)hipGraphDestroy(g);
            return t;
        };
        // mean time per call of `reps` calls of f, best of two rounds (ms)
        auto timed = [&](int reps_, int only) {
            float t = 1e30f;
            for (int round = 0; round < 2 && r == SV_OK; ++round) {
                for (int k = 0; k < 2 && r == SV_OK; ++k) r = fwd(only);  // warm
                hipEvent_t ea, eb;
                (void)hipEventCreate(&ea);
                (void)hipEventCreate(&eb);
                (void)hipEventRecord(ea, st);
                for (int k = 0; k < reps_ && r == SV_OK; ++k) r = fwd(only);
                (void)hipEventRecord(eb, st);
                (void)hipEventSynchronize(eb);
                float ms_ = 0.f;
                (void)hipEventElapsedTime(&ms_, ea, eb);
                (void)hipEventDestroy(ea);
                (void)hipEventDestroy(eb);
                t = std::min(t, ms_ / reps_);
            }
            return t;
        };
        r = fwd(-1);
        const int nrep = B >= 16 ? 6 : 24;
        for (int i = 0; i < L_F && r == SV_OK; ++i) {
            if (i == L_E1) continue;  // a direct stencil, no tile configuration
            float kt[NKEEP];
            for (int c = 0; c < conv_num_cfgs() && r == SV_OK; ++c) {
                // a tile shape that does not fit this layer would run as the fallback,
                // a split that falls back to one pass repeats an unsplit candidate
                if (conv_resolve_cfg(ns.dtype, ns.ly[i].k, ns.ly[i].stride, c) != c) continue;
                if (net_layer_split(ns, i, c, B, H, W) != c / conv_num_tiles() + 1) continue;
                // G0 carrying the final layer's projection runs unsplit on tiles that
                // hold all of its channels: other candidates repeat one of those
                if (i == L_G0 && net_projects(ns, false) && net_g0_proj_cfg(ns, c) != c) continue;
                cur[i] = c;
                const float t = timed(nrep, i);
                if (r != SV_OK) break;
                if (verbose) fprintf(stderr, "sv_autotune dt%d B%d %dx%d layer %d cfg %-14s alone %8.2f us\n",
                                     ns.dtype, B, H, W, i, conv_cfg_name(c), t * 1e3f);
                // insert into the sorted short list
                int pos = nkeep[i];
                while (pos > 0 && kt[pos - 1] > t) {
                    if (pos < NKEEP) { kt[pos] = kt[pos - 1]; keep[i][pos] = keep[i][pos - 1]; }
                    --pos;
                }
                if (pos < NKEEP) {
                    kt[pos] = t;
                    keep[i][pos] = c;
                    if (nkeep[i] < NKEEP) ++nkeep[i];
                }
            }
            if (nkeep[i] > 0) best_cfg[i] = keep[i][0];
            cur[i] = best_cfg[i];
        }
        (void)hipStreamSynchronize(st);  // stage 1's launches are done before the replays
        const int nrep2 = B >= 16 ? 6 : 50;
        for (int pass = 0; pass < 2 && r == SV_OK; ++pass) {
            for (int i = 0; i < L_F && r == SV_OK; ++i) {
                if (nkeep[i] < 2) continue;
                float best_t = 1e30f;
                int best_c = best_cfg[i];
                for (int k = 0; k < nkeep[i] && r == SV_OK; ++k) {
                    cur[i] = keep[i][k];
                    const float t = graph_timed(nrep2);
                    if (verbose) fprintf(stderr, "sv_autotune dt%d B%d %dx%d layer %d cfg %-14s whole pass %8.2f us\n",
                                         ns.dtype, B, H, W, i, conv_cfg_name(keep[i][k]), t * 1e3f);
                    if (t < best_t) { best_t = t; best_c = keep[i][k]; }
                }
                best_cfg[i] = best_c;
                cur[i] = best_c;
            }
        }
        if (cs) (void)hipStreamDestroy(cs);
    }
    (void)hipStreamSynchronize(st);
    (void)hipFree(mem);
    if (r != SV_OK) return r;
    cost_wta_split_tuned(B, h, w, D, best_ds);
    TuneEntry e = make_key(ns, B, H, W);
    e.dsplit = best_ds;
    for (int i = 0; i < NLAYERS; ++i) e.cfg[i] = best_cfg[i];
    cache_store(e);
    return SV_OK;
}

sv_status sv_layer_cfgs(const sv_vae_desc *desc, int B, int H, int W, int *cfg_out) {
    NetShape ns;
    sv_status r = net_shape(desc, ns);
    if (r != SV_OK) return r;
    if (!cfg_out) return SV_ERR_NULL;
    if (B < 1 || H < 1 || W < 1) return SV_ERR_SHAPE;
    net_layer_cfgs(ns, B, H, W, cfg_out);
    return SV_OK;
}

const char *sv_conv_cfg_name(int cfg) { return conv_cfg_name(cfg); }

sv_status sv_tile_config(int stage, char *buf, int buflen) {
    if (!buf || buflen < 1) return SV_ERR_NULL;
    if (stage == 0) {
        snprintf(buf, buflen, "census tile %dx4 (one frame) or %dx16 (from 512 tall tiles)", CEN_TILE_W,
                 CEN_TILE_W);
    } else if (stage == 1) {
        const int ov = cost_wta_split_override();
        if (ov > 0)
            snprintf(buf, buflen, "cost_wta dsplit=%d (set)", ov);
        else
            snprintf(buf, buflen, "cost_wta dsplit per shape (autotuned, else 4)");
    } else if (stage >= 2 && stage < 2 + NLAYERS) {
        const int o32 = net_get_cfg_override(SV_F32, stage - 2), o16 = net_get_cfg_override(SV_BF16, stage - 2);
        snprintf(buf, buflen, "layer %d override f32=%s bf16=%s", stage - 2,
                 o32 >= 0 ? conv_cfg_name(o32) : "none", o16 >= 0 ? conv_cfg_name(o16) : "none");
    } else {
        buf[0] = 0;
        return SV_ERR_RANGE;
    }
    return SV_OK;
}

}  // extern "C"
