// igks_host.cpp - host side of libigks: mesh ingest and preprocessing
// (Sec. 2.4 mesh data -> faces, geometry, ghost-cell offsets, sweep
// wavefronts) for one or many instances, the workspace layout, the
// iteration driver with HIP-graph chunks, the launch-schedule autotuner and
// the C ABI declared in include/igks.h.
#include "../../include/igks.h"
#include "igks_dev.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <numeric>
#include <string>
#include <unordered_map>
#include <vector>

using namespace igks;

namespace {

// A cell is non-convex where its counter-clockwise boundary turns clockwise
// by more than asin(MAX_REFLEX_SIN), about 5.7 degrees.
constexpr double MAX_REFLEX_SIN = 0.1;

// One instance, in its upload order.
struct InstMesh {
    bool ok = false;
    int nn = 0, nc = 0, nlev = 0;
    std::vector<double> xy;
    std::vector<int> cptr, cn;                 // counter-clockwise vertex lists
    std::vector<double> area, xc, yc;
    struct UF { int l, r, tag, a, b; };        // faces; owner l = the lower upload index
    std::vector<UF> uf;
    std::vector<int> cf_ptr, cf_list;          // cell -> faces (in the order of uf), CSR
    std::vector<int> level;                    // sweep wavefront of each cell
    std::vector<int> sblk;                     // sweep block of each cell (empty: one block)
    std::vector<int> wall_uf;                  // WALL faces in the input order of the boundary edges
    bool have_flow = false;
    double alpha = 0;
    InstParam ip{};
};

// All instances concatenated in the internal order.
struct Global {
    int N = 0, F = 0, nlev = 0, nwall = 0, max_inst_cells = 0;
    int NB = 0;                      // entry / vertex blocks: N + one overflow block per polygon
    std::vector<int> lev_off;        // wavefront offsets (internal cells)
    // sweep blocks of all instances (an instance without blocks is one):
    // block gb's cells of its k-th wavefront are the internal cells
    // [bl_lo[bl_off[gb] + k], bl_hi[bl_off[gb] + k])
    std::vector<int> bl_off, bl_lo, bl_hi;
    std::vector<int> coff;           // first global upload id of each instance
    std::vector<int> g2i;            // global upload id -> internal cell
    std::vector<int> cinst, finst, icell, ioff, ipos, cperm;
    std::vector<double> xc, yc, area, lsinv, vtx;
    std::vector<int> cf_face, cf_nbr, cf_flag;   // MAXV entries per block
    std::vector<double> cf_dx, cf_dy;
    std::vector<double> enx, eny, es;    // per entry: normal out of the entry's cell, face length
    std::vector<int> fl, fr, ftag;
    std::vector<double> fnx, fny, flen, frl, frr, fdl, fdr, frn, fxm;
    std::vector<int> wall_faces, woff;   // internal face ids per instance (input order); offsets
    std::vector<double> wseg;            // wall segments (ax, ay, bx, by)
};

struct Buf {
    size_t off, bytes;
};

// timed kernel classes: prep, flux, gather, norms, forward sweep, backward sweep with update
constexpr int NKT = 6;

struct WsMap {
    Buf ip, is, slot, Wa, Wb, grad, lamc, vort, nu, M, lsum, sadiag, r2, dW, dW1, dinv, xc, yc, area, lsinv, dwall, vtx, phi;
    Buf cinst, finst, icell, ioff, g2i, cf_face, cf_nbr, cf_flag, cf_dx, cf_dy;
    Buf fl, fr, fbc, fnx, fny, flen, frl, frr, fidl, fidr, firn, ipart, hist, ipos, cperm;
    Buf frec, flam, fsak, enx, eny, es;
    Buf wall_faces, wall_out, woff, wseg, lev_off, bl_off, bl_lo, bl_hi, stage, backup;
    size_t total;
};

}  // namespace

struct igks_ctx {
    igks_options opt{};
    hipStream_t stream = nullptr;
    bool own_stream = false;
    std::string err;
    std::vector<InstMesh> inst;
    Global g;
    bool combined = false;
    // workspace
    char *ws = nullptr;
    size_t ws_bytes = 0;
    bool bound = false;
    int static_dev = -1;               // device whose static workspace is bound, -1: a caller's buffer
    unsigned long long static_gen = 0; // binding generation of that static workspace
    WsMap w{};
    Params<double> P64{};
    Params<float> P32{};
    int hist_cap = 0;
    // launch schedule
    int block[NCLASS] = {256, 256, 256, 256};
    int sweep_mode = 1;       // LU-SGS sweeps: 1 a launch per wavefront, 2 one workgroup, 3 a wave per sweep block
    bool flux_pair = false;   // face flux on two lanes per face
    // host copies of the device scalars and the history of the last iterate call
    std::vector<InstScalars> hs;
    std::vector<std::vector<double>> hist;
    // graph of one chunk
    hipGraphExec_t gexec = nullptr;
    int gexec_k = 0;                   // iterations captured in gexec
    // profiling
    bool profiling = false;
    double ktimes[NKT] = {0, 0, 0, 0, 0, 0};
};

// The library's own workspace for callers that cannot allocate device
// memory (igks_bind_static_workspace): one array per GPU, which each GPU the
// library runs on holds until the process ends.  In host code `scratch` only
// names the array; its device address comes from hipGetSymbolAddress, once
// per device, with that device current.
constexpr size_t STATIC_WS_BYTES = size_t(64) << 20;
static __device__ __align__(256) char scratch[STATIC_WS_BYTES];

namespace {

constexpr int MAX_DEVICES = 64;
struct StaticWs {
    void *ptr = nullptr;          // device address of `scratch` on this device
    unsigned long long gen = 0;   // bumped by every binding: a context holds the array while its gen is current
};
std::mutex static_mu;
StaticWs static_ws[MAX_DEVICES];

int fail(igks_ctx *c, int code, const std::string &msg)
{
    if (c) c->err = msg;
    return code;
}

#define HIPCHK(ctx, call)                                                                           \
    do {                                                                                            \
        hipError_t e_ = (call);                                                                     \
        if (e_ != hipSuccess) return fail(ctx, IGKS_EHIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

void destroy_graph(igks_ctx *c)
{
    if (c->gexec) {
        (void)hipGraphExecDestroy(c->gexec);
        c->gexec = nullptr;
    }
    c->gexec_k = 0;
}

// Iterations per captured graph: the requested chunk, cut so that a graph
// holds at most MAX_GRAPH_NODES launches (one launch per wavefront and sweep
// direction makes an iteration of a many-wavefront batch thousands of
// launches long); 0 = no graphs.
constexpr int MAX_GRAPH_NODES = 8192;
bool two_block_passes(const igks_ctx *c);
int launches_per_iteration(const igks_ctx *c, int sweep_mode)
{
    const int nlev = std::max(1, c->g.nlev);
    // per-wavefront sweeps: forward steps of wavefronts 1 .. nlev-2, the last
    // wavefront's two steps, backward steps of nlev-2 .. 0; the other
    // schedules: forward, backward, update
    int sweeps = c->opt.scheme == 1 ? 1 : (sweep_mode >= 2 ? 3 : std::max(1, 2 * nlev - 2));
    if (c->opt.scheme != 1 && sweep_mode == 3 && two_block_passes(c)) sweeps += 2;   // the first pass
    return 5 + sweeps;   // prep, flux, gather, reduce, commit + the update / sweep launches
}
int graph_chunk_for(const igks_ctx *c, int sweep_mode)
{
    if (c->opt.chunk <= 0) return 0;
    return std::max(1, std::min(c->opt.chunk, MAX_GRAPH_NODES / launches_per_iteration(c, sweep_mode)));
}
int graph_chunk(const igks_ctx *c) { return graph_chunk_for(c, c->sweep_mode); }

// The schedule chosen at binding time from the sizes: one workgroup for the
// sweeps when wavefronts are many and narrow (one workgroup of 512 threads
// takes a wavefront per round of 512 cells and a launch per wavefront costs
// a few microseconds, so the workgroup wins up to about two rounds); one
// lane per face (its kernel holds two waves per SIMD and executes the
// fewest instructions per face) except on small meshes, where two lanes
// per face give the SIMDs twice as many waves to switch between.
//
// With sweep blocks the cells of different blocks never wait for each other,
// so one wave sweeps each block on its own (no launch per wavefront, no
// barrier across blocks).
bool any_sweep_blocks(const igks_ctx *c)
{
    for (const auto &m : c->inst)
        if (!m.sblk.empty()) return true;
    return false;
}
// two block passes (option block_passes = 2 and some instance has blocks)
bool two_block_passes(const igks_ctx *c) { return c->opt.block_passes == 2 && any_sweep_blocks(c); }
int auto_sweep_mode(const igks_ctx *c)
{
    if (c->opt.sweep > 0) return c->opt.sweep;
    if (any_sweep_blocks(c)) return 3;
    const double width = (double)c->g.N / std::max(1, c->g.nlev);
    return (c->g.nlev > 16 && width < 1024.0) ? 2 : 1;
}
bool auto_flux_pair(const igks_ctx *c) { return c->opt.flux_lanes == 2 || (c->opt.flux_lanes == 0 && c->g.F < 32768); }

// ------------------------------------------------------------------ ingest

// neighbours the sweeps couple: interior, and in the same sweep block
bool same_block(const InstMesh &m, int a, int b) { return m.sblk.empty() || m.sblk[a] == m.sblk[b]; }

// sweep wavefronts: level(i) = 1 + max level of the coupled neighbours with a
// smaller index (0 without any)
void compute_levels(InstMesh &m)
{
    const int N = m.nc;
    m.level.assign(N, 0);
    m.nlev = 0;
    for (int i = 0; i < N; i++) {
        int lv = 0;
        for (int e = m.cf_ptr[i]; e < m.cf_ptr[i + 1]; e++) {
            const auto &f = m.uf[m.cf_list[e]];
            int o = f.l == i ? f.r : f.l;
            if (o >= 0 && o < i && same_block(m, i, o)) lv = std::max(lv, m.level[o] + 1);
        }
        m.level[i] = lv;
        m.nlev = std::max(m.nlev, lv + 1);
    }
}

int build_instance(igks_ctx *ctx, int n_nodes, const double *xy, int n_cells, const int32_t *cell_ptr,
                   const int32_t *cell_nodes, int n_bfaces, const int32_t *bface_nodes, const int32_t *bface_tag,
                   InstMesh &m)
{
    if (n_nodes <= 0 || n_cells <= 0 || n_bfaces < 0 || !xy || !cell_ptr || !cell_nodes ||
        (n_bfaces > 0 && (!bface_nodes || !bface_tag)))
        return fail(ctx, IGKS_EINVAL, "empty mesh or null pointer");
    if (cell_ptr[0] != 0) return fail(ctx, IGKS_EMESH, "cell_ptr[0] must be 0");
    m = InstMesh();
    m.nn = n_nodes;
    m.nc = n_cells;
    const int N = n_cells;
    m.xy.assign(xy, xy + 2 * (size_t)n_nodes);
    m.cptr.assign(cell_ptr, cell_ptr + N + 1);
    for (int i = 0; i < N; i++) {
        int k = m.cptr[i + 1] - m.cptr[i];
        if (k < 3 || k > MAXP)
            return fail(ctx, IGKS_EMESH, "cell " + std::to_string(i) + " has " + std::to_string(k) +
                                             " nodes (3 to " + std::to_string(MAXP) + " supported)");
    }
    m.cn.resize(m.cptr[N]);
    for (int p = 0; p < m.cptr[N]; p++) {
        int v = cell_nodes[p];
        if (v < 0 || v >= n_nodes) return fail(ctx, IGKS_EMESH, "node index out of range");
        m.cn[p] = v;
    }
    // counter-clockwise orientation, area and centroid (relative to the
    // first vertex to limit cancellation)
    m.area.resize(N); m.xc.resize(N); m.yc.resize(N);
    for (int i = 0; i < N; i++) {
        int p0 = m.cptr[i], k = m.cptr[i + 1] - p0;
        double x0 = xy[2 * m.cn[p0]], y0 = xy[2 * m.cn[p0] + 1];
        double a2 = 0, sx = 0, sy = 0;
        for (int j = 1; j + 1 < k; j++) {
            double ax = xy[2 * m.cn[p0 + j]] - x0, ay = xy[2 * m.cn[p0 + j] + 1] - y0;
            double bx = xy[2 * m.cn[p0 + j + 1]] - x0, by = xy[2 * m.cn[p0 + j + 1] + 1] - y0;
            double t = ax * by - ay * bx;
            a2 += t;
            sx += t * (ax + bx);
            sy += t * (ay + by);
        }
        if (a2 < 0) {
            std::reverse(m.cn.begin() + p0, m.cn.begin() + p0 + k);
            a2 = -a2; sx = -sx; sy = -sy;
        }
        if (!(a2 > 0)) return fail(ctx, IGKS_EMESH, "degenerate cell " + std::to_string(i));
        m.area[i] = 0.5 * a2;
        m.xc[i] = x0 + sx / (3.0 * a2);
        m.yc[i] = y0 + sy / (3.0 * a2);
        // convex: no vertex turns clockwise by more than asin(MAX_REFLEX_SIN)
        // (hanging nodes on curved edges turn back slightly), and the
        // centroid lies strictly inside every face's half plane (the
        // centroid-face distances d_l, d_r divide in the face flux)
        for (int j = 0; j < k; j++) {
            const double *pa = &xy[2 * m.cn[p0 + (j + k - 1) % k]], *pb = &xy[2 * m.cn[p0 + j]],
                         *pc = &xy[2 * m.cn[p0 + (j + 1) % k]];
            const double ux = pb[0] - pa[0], uy = pb[1] - pa[1], vx = pc[0] - pb[0], vy = pc[1] - pb[1];
            const double sn = (ux * vy - uy * vx) / (std::hypot(ux, uy) * std::hypot(vx, vy));
            if (!(sn >= -MAX_REFLEX_SIN)) return fail(ctx, IGKS_EMESH, "non-convex cell " + std::to_string(i));
            const double cr = (pb[0] - m.xc[i]) * (pc[1] - m.yc[i]) - (pb[1] - m.yc[i]) * (pc[0] - m.xc[i]);
            if (!(cr > 0)) return fail(ctx, IGKS_EMESH, "cell " + std::to_string(i) + ": centroid outside a face");
        }
    }
    // edges -> faces
    struct E { long long key; int cell, loc; };
    std::vector<E> ev(m.cptr[N]);
    for (int i = 0; i < N; i++) {
        int p0 = m.cptr[i], k = m.cptr[i + 1] - p0;
        for (int j = 0; j < k; j++) {
            long long a = m.cn[p0 + j], b = m.cn[p0 + (j + 1) % k];
            ev[p0 + j] = {std::min(a, b) * (long long)(n_nodes + 1) + std::max(a, b), i, j};
        }
    }
    std::sort(ev.begin(), ev.end(), [](const E &a, const E &b) {
        return a.key != b.key ? a.key < b.key : (a.cell != b.cell ? a.cell < b.cell : a.loc < b.loc);
    });
    std::unordered_map<long long, int> bmap;
    bmap.reserve(n_bfaces * 2 + 1);
    for (int b = 0; b < n_bfaces; b++) {
        long long a = bface_nodes[2 * b], d = bface_nodes[2 * b + 1];
        if (a < 0 || a >= n_nodes || d < 0 || d >= n_nodes) return fail(ctx, IGKS_EMESH, "boundary node out of range");
        int t = bface_tag[b];
        if (t < 1 || t > 6) return fail(ctx, IGKS_EMESH, "bad boundary tag");
        if (!bmap.emplace(std::min(a, d) * (long long)(n_nodes + 1) + std::max(a, d), b).second)
            return fail(ctx, IGKS_EMESH, "duplicate boundary edge");
    }
    std::vector<char> bused(n_bfaces, 0);
    std::vector<int> wslot(n_bfaces, -1);
    for (size_t i = 0; i < ev.size();) {
        size_t j = i + 1;
        while (j < ev.size() && ev[j].key == ev[i].key) j++;
        if (j - i > 2) return fail(ctx, IGKS_EMESH, "edge shared by more than two cells");
        int ow = ev[i].cell, lo = ev[i].loc;
        int p0 = m.cptr[ow], k = m.cptr[ow + 1] - p0;
        InstMesh::UF f{ow, -1, 0, m.cn[p0 + lo], m.cn[p0 + (lo + 1) % k]};
        if (j - i == 2) {
            f.r = ev[i + 1].cell;
        } else {
            auto it = bmap.find(ev[i].key);
            if (it == bmap.end()) return fail(ctx, IGKS_EMESH, "boundary edge without a tag");
            f.tag = bface_tag[it->second];
            bused[it->second] = 1;
            if (f.tag == BC_WALL) wslot[it->second] = (int)m.uf.size();
        }
        m.uf.push_back(f);
        i = j;
    }
    for (int b = 0; b < n_bfaces; b++)
        if (!bused[b]) return fail(ctx, IGKS_EMESH, "tagged edge " + std::to_string(b) + " is not on the mesh boundary");
    for (int b = 0; b < n_bfaces; b++)
        if (wslot[b] >= 0) m.wall_uf.push_back(wslot[b]);
    // cell -> faces
    m.cf_ptr.assign(N + 1, 0);
    for (auto &f : m.uf) {
        m.cf_ptr[f.l + 1]++;
        if (f.r >= 0) m.cf_ptr[f.r + 1]++;
    }
    for (int i = 0; i < N; i++) m.cf_ptr[i + 1] += m.cf_ptr[i];
    m.cf_list.resize(m.cf_ptr[N]);
    {
        std::vector<int> fill(N, 0);
        for (int q = 0; q < (int)m.uf.size(); q++) {
            m.cf_list[m.cf_ptr[m.uf[q].l] + fill[m.uf[q].l]++] = q;
            if (m.uf[q].r >= 0) m.cf_list[m.cf_ptr[m.uf[q].r] + fill[m.uf[q].r]++] = q;
        }
    }
    compute_levels(m);
    m.ok = true;
    return IGKS_OK;
}

// Concatenate the instances in the internal order: cells by (wavefront,
// instance, upload index); interior faces by internal owner, then boundary
// faces by internal owner.
// Processing order of the cell kernels (Global::cperm): per instance, its
// cells ranked along a Morton curve of their centroids and cut into tiles
// of TILE_CELLS; each tile's cells by wavefront, then internal index.  In a
// colour order every neighbour of a cell lies in another wavefront; the
// internal order keeps the wavefronts apart, while this order puts a tile's
// wavefronts one after another, so a cell and its neighbours are read by
// the same XCD (the launch gives each XCD a contiguous range of it) close
// together in time.
#ifndef IGKS_TILE_CELLS
#define IGKS_TILE_CELLS 4096
#endif
constexpr int TILE_CELLS = IGKS_TILE_CELLS;
void cell_tiles(Global &G, int ni)
{
    const int N = G.N;
    std::vector<uint32_t> key(N);
    std::vector<int> lev(N);
    for (int l = 0; l < G.nlev; l++)
        for (int c = G.lev_off[l]; c < G.lev_off[l + 1]; c++) lev[c] = l;
    G.cperm.clear();
    G.cperm.reserve(N);
    for (int i = 0; i < ni; i++) {
        const int *cells = G.icell.data() + G.ioff[i];
        const int n = G.ioff[i + 1] - G.ioff[i];
        double x0 = INFINITY, x1 = -INFINITY, y0 = INFINITY, y1 = -INFINITY;
        for (int k = 0; k < n; k++) {
            const int c = cells[k];
            x0 = std::min(x0, G.xc[c]); x1 = std::max(x1, G.xc[c]);
            y0 = std::min(y0, G.yc[c]); y1 = std::max(y1, G.yc[c]);
        }
        const double sx = 65535.0 / std::max(x1 - x0, 1e-300), sy = 65535.0 / std::max(y1 - y0, 1e-300);
        auto spread = [](uint32_t v) {   // the 16 bits of v to the even bit positions
            v &= 0xffffu;
            v = (v | (v << 8)) & 0x00ff00ffu;
            v = (v | (v << 4)) & 0x0f0f0f0fu;
            v = (v | (v << 2)) & 0x33333333u;
            return (v | (v << 1)) & 0x55555555u;
        };
        std::vector<int> r(cells, cells + n);
        for (int c : r)
            key[c] = spread((uint32_t)((G.xc[c] - x0) * sx)) | (spread((uint32_t)((G.yc[c] - y0) * sy)) << 1);
        std::stable_sort(r.begin(), r.end(), [&](int a, int b) { return key[a] < key[b]; });
        for (int t0 = 0; t0 < n; t0 += TILE_CELLS) {
            const int t1 = std::min(n, t0 + TILE_CELLS);
            std::sort(r.begin() + t0, r.begin() + t1,
                      [&](int a, int b) { return lev[a] != lev[b] ? lev[a] < lev[b] : a < b; });
        }
        G.cperm.insert(G.cperm.end(), r.begin(), r.end());
    }
}

int combine(igks_ctx *ctx)
{
    Global &G = ctx->g;
    G = Global();
    const int ni = (int)ctx->inst.size();
    G.coff.assign(ni + 1, 0);
    for (int i = 0; i < ni; i++) {
        G.coff[i + 1] = G.coff[i] + ctx->inst[i].nc;
        G.nlev = std::max(G.nlev, ctx->inst[i].nlev);
        G.max_inst_cells = std::max(G.max_inst_cells, ctx->inst[i].nc);
    }
    const int N = G.coff[ni];
    G.N = N;
    std::vector<int> gi(N), gu(N), glev(N), gblk(N);
    int ngb = 0;   // sweep blocks over all instances
    for (int i = 0; i < ni; i++) {
        const InstMesh &m = ctx->inst[i];
        int nb = 1;
        for (int u = 0; u < m.nc; u++) {
            int gid = G.coff[i] + u;
            gi[gid] = i; gu[gid] = u; glev[gid] = m.level[u];
            gblk[gid] = ngb + (m.sblk.empty() ? 0 : m.sblk[u]);
            if (!m.sblk.empty()) nb = std::max(nb, m.sblk[u] + 1);
        }
        ngb += nb;
    }
    std::vector<int> order(N);   // internal cell -> global upload id: by wavefront, instance, sweep block, upload index
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(),
                     [&](int a, int b) { return glev[a] != glev[b] ? glev[a] < glev[b] : gblk[a] < gblk[b]; });
    G.g2i.resize(N);
    for (int c = 0; c < N; c++) G.g2i[order[c]] = c;
    G.lev_off.assign(G.nlev + 1, 0);
    for (int c = 0; c < N; c++) G.lev_off[glev[order[c]] + 1]++;
    for (int l = 0; l < G.nlev; l++) G.lev_off[l + 1] += G.lev_off[l];
    {
        // per sweep block, its wavefronts in order: each a contiguous range of
        // internal cells (the internal order is by wavefront, then block)
        std::vector<std::vector<std::pair<int, int>>> rng(ngb);
        for (int c = 0; c < N; c++) {
            auto &r = rng[gblk[order[c]]];
            const int lv = glev[order[c]];
            if ((int)r.size() == lv) r.push_back({c, c + 1});
            else r.back().second = c + 1;   // cells of one block and wavefront are adjacent
        }
        G.bl_off.assign(ngb + 1, 0);
        G.bl_lo.clear(); G.bl_hi.clear();
        for (int b = 0; b < ngb; b++) {
            for (auto &p : rng[b]) { G.bl_lo.push_back(p.first); G.bl_hi.push_back(p.second); }
            G.bl_off[b + 1] = (int)G.bl_lo.size();
        }
    }
    G.cinst.resize(N);
    for (int c = 0; c < N; c++) G.cinst[c] = gi[order[c]];
    G.ioff.assign(ni + 1, 0);
    for (int c = 0; c < N; c++) G.ioff[G.cinst[c] + 1]++;
    for (int i = 0; i < ni; i++) G.ioff[i + 1] += G.ioff[i];
    G.icell.resize(N);
    G.ipos.resize(N);
    {
        std::vector<int> fill(ni, 0);
        for (int c = 0; c < N; c++) {
            int k = G.ioff[G.cinst[c]] + fill[G.cinst[c]]++;
            G.icell[k] = c;
            G.ipos[c] = k;
        }
    }
    // the cell kernels' processing order (needs the centroids in internal order)
    G.xc.resize(N); G.yc.resize(N);
    for (int c = 0; c < N; c++) {
        const InstMesh &m = ctx->inst[gi[order[c]]];
        G.xc[c] = m.xc[gu[order[c]]]; G.yc[c] = m.yc[gu[order[c]]];
    }
    cell_tiles(G, ni);
    std::vector<int> trank(N);   // position of each cell in that order
    for (int k = 0; k < N; k++) trank[G.cperm[k]] = k;
    // faces: interior faces, then boundary faces, each sorted by their owner's
    // position in the cell kernels' order (the faces of a spatial tile together)
    struct FRef { int inst, q; };
    std::vector<FRef> all;
    for (int i = 0; i < ni; i++)
        for (int q = 0; q < (int)ctx->inst[i].uf.size(); q++) all.push_back({i, q});
    auto boundary = [&](const FRef &r) { return ctx->inst[r.inst].uf[r.q].r < 0; };
    auto owner = [&](const FRef &r) { return G.g2i[G.coff[r.inst] + ctx->inst[r.inst].uf[r.q].l]; };
    std::stable_sort(all.begin(), all.end(), [&](const FRef &a, const FRef &b) {
        bool ba = boundary(a), bb = boundary(b);
        if (ba != bb) return bb;
        return trank[owner(a)] < trank[owner(b)];
    });
    const int F = (int)all.size();
    G.F = F;
    std::vector<std::vector<int>> fpos(ni);
    for (int i = 0; i < ni; i++) fpos[i].assign(ctx->inst[i].uf.size(), -1);
    for (int q = 0; q < F; q++) fpos[all[q].inst][all[q].q] = q;
    G.fl.resize(F); G.fr.resize(F); G.ftag.resize(F); G.finst.resize(F);
    G.fnx.resize(F); G.fny.resize(F); G.flen.resize(F); G.frl.resize(2 * (size_t)F); G.frr.resize(2 * (size_t)F);
    G.fdl.resize(F); G.fdr.resize(F); G.frn.resize(F); G.fxm.resize(F);
    for (int q = 0; q < F; q++) {
        const InstMesh &m = ctx->inst[all[q].inst];
        const auto &u = m.uf[all[q].q];
        const double *xy = m.xy.data();
        double ax = xy[2 * u.a], ay = xy[2 * u.a + 1], bx = xy[2 * u.b], by = xy[2 * u.b + 1];
        double dx = bx - ax, dy = by - ay, L = std::sqrt(dx * dx + dy * dy);
        double nx = dy / L, ny = -dx / L;   // outward normal of the owner's counter-clockwise edge
        double xm = 0.5 * (ax + bx), ym = 0.5 * (ay + by);
        int off = G.coff[all[q].inst];
        G.finst[q] = all[q].inst;
        G.fl[q] = G.g2i[off + u.l];
        G.fr[q] = u.r >= 0 ? G.g2i[off + u.r] : -1;
        G.ftag[q] = u.tag;
        G.fnx[q] = nx; G.fny[q] = ny; G.flen[q] = L; G.fxm[q] = xm;
        double rlx = xm - m.xc[u.l], rly = ym - m.yc[u.l];
        G.frl[2 * (size_t)q] = rlx; G.frl[2 * (size_t)q + 1] = rly;
        double dl = rlx * nx + rly * ny;
        G.fdl[q] = dl;
        if (u.r >= 0) {
            double rrx = xm - m.xc[u.r], rry = ym - m.yc[u.r];
            G.frr[2 * (size_t)q] = rrx; G.frr[2 * (size_t)q + 1] = rry;
            G.fdr[q] = -(rrx * nx + rry * ny);
            G.frn[q] = std::fabs((m.xc[u.r] - m.xc[u.l]) * nx + (m.yc[u.r] - m.yc[u.l]) * ny);
        } else {
            G.frr[2 * (size_t)q] = G.frr[2 * (size_t)q + 1] = 0.0;
            G.fdr[q] = dl;
            G.frn[q] = 2.0 * dl;
        }
    }
    // wall faces and segments, per instance
    G.woff.assign(ni + 1, 0);
    for (int i = 0; i < ni; i++) {
        const InstMesh &m = ctx->inst[i];
        for (int q : m.wall_uf) {
            const auto &u = m.uf[q];
            G.wall_faces.push_back(fpos[i][q]);
            G.wseg.push_back(m.xy[2 * u.a]); G.wseg.push_back(m.xy[2 * u.a + 1]);
            G.wseg.push_back(m.xy[2 * u.b]); G.wseg.push_back(m.xy[2 * u.b + 1]);
        }
        G.woff[i + 1] = (int)G.wall_faces.size();
    }
    G.nwall = (int)G.wall_faces.size();
    // cells in internal order; a polygon with more than MAXV faces gets an
    // overflow block (blocks N, N + 1, ... in internal cell order)
    G.xc.resize(N); G.yc.resize(N); G.area.resize(N); G.lsinv.resize(3 * (size_t)N);
    std::vector<int> ovf(N, -1);
    int NB = N;
    for (int c = 0; c < N; c++) {
        const InstMesh &m = ctx->inst[gi[order[c]]];
        const int u = gu[order[c]];
        if (m.cf_ptr[u + 1] - m.cf_ptr[u] > MAXV || m.cptr[u + 1] - m.cptr[u] > MAXV) ovf[c] = NB++;
    }
    if (NB - N >= (1 << (31 - CF_NEXT_SHIFT)))
        return fail(ctx, IGKS_EMESH, "too many cells with more than " + std::to_string(MAXV) + " faces");
    G.NB = NB;
    G.vtx.resize(2 * MAXV * (size_t)NB);
    // entries: MAXV per block, in the order of the cell's faces; unused
    // entries point at the cell's first face with no flags
    const size_t ne = (size_t)MAXV * NB;
    G.cf_face.assign(ne, 0); G.cf_nbr.assign(ne, -1); G.cf_flag.assign(ne, 0);
    G.cf_dx.assign(ne, 0.0); G.cf_dy.assign(ne, 0.0);
    G.enx.assign(ne, 0.0); G.eny.assign(ne, 0.0); G.es.assign(ne, 0.0);
    for (int c = 0; c < N; c++) {
        const int i = gi[order[c]], u = gu[order[c]], off = G.coff[i];
        const InstMesh &m = ctx->inst[i];
        G.xc[c] = m.xc[u]; G.yc[c] = m.yc[u]; G.area[c] = m.area[u];
        double a11 = 0, a12 = 0, a22 = 0;
        const int nfc = m.cf_ptr[u + 1] - m.cf_ptr[u];
        auto slot = [&](int k) {   // entry index of the cell's k-th face
            return k < MAXV ? (size_t)MAXV * c + k : (size_t)MAXV * ovf[c] + (k - MAXV);
        };
        for (int kk = 0; kk < nfc; kk++) {
            const int k = m.cf_ptr[u] + kk;
            const size_t e = slot(kk);
            const int q = m.cf_list[k];
            const auto &f = m.uf[q];
            const int qi = fpos[i][q];
            const bool own = f.l == u;
            const int other = own ? f.r : f.l;
            double dx, dy;
            if (other >= 0) {
                dx = m.xc[other] - m.xc[u];
                dy = m.yc[other] - m.yc[u];
            } else {   // ghost centroid: the cell centroid reflected in the face line
                dx = 2.0 * G.fdl[qi] * G.fnx[qi];
                dy = 2.0 * G.fdl[qi] * G.fny[qi];
            }
            G.cf_face[e] = qi;
            G.enx[e] = own ? G.fnx[qi] : -G.fnx[qi];
            G.eny[e] = own ? G.fny[qi] : -G.fny[qi];
            G.es[e] = G.flen[qi];
            G.cf_nbr[e] = other >= 0 ? G.g2i[off + other] : -1;
            const bool coupled = other >= 0 && same_block(m, u, other);
            G.cf_flag[e] = CF_VALID | (own ? CF_OWNER : 0) | ((coupled && other < u) ? CF_LOWER : 0) |
                           ((other >= 0 && !coupled) ? CF_OTHER : 0);
            G.cf_dx[e] = dx;
            G.cf_dy[e] = dy;
            a11 += dx * dx; a12 += dx * dy; a22 += dy * dy;
        }
        const int nslots = ovf[c] >= 0 ? 2 * MAXV : MAXV;
        for (int kk = nfc; kk < nslots; kk++) G.cf_face[slot(kk)] = G.cf_face[(size_t)MAXV * c];
        if (ovf[c] >= 0) G.cf_flag[(size_t)MAXV * c + MAXV - 1] |= (ovf[c] - N + 1) << CF_NEXT_SHIFT;
        double det = a11 * a22 - a12 * a12;
        if (!(det > 0))
            return fail(ctx, IGKS_EMESH, "instance " + std::to_string(i) + ": singular least-squares stencil at cell " +
                                             std::to_string(u));
        G.lsinv[c] = a22 / det;
        G.lsinv[(size_t)N + c] = -a12 / det;
        G.lsinv[2 * (size_t)N + c] = a11 / det;
        int p0 = m.cptr[u], k = m.cptr[u + 1] - p0;
        for (int v = 0; v < (ovf[c] >= 0 ? 2 * MAXV : MAXV); v++) {
            int node = m.cn[p0 + (v < k ? v : 0)];
            const size_t b = v < MAXV ? (size_t)c : (size_t)ovf[c], sv = v % MAXV;
            G.vtx[(2 * sv) * (size_t)NB + b] = m.xy[2 * node] - m.xc[u];
            G.vtx[(2 * sv + 1) * (size_t)NB + b] = m.xy[2 * node + 1] - m.yc[u];
        }
    }
    ctx->combined = true;
    return IGKS_OK;
}

// ---------------------------------------------------------------- workspace

struct Layout {
    size_t total = 0;
    Buf add(size_t bytes)
    {
        Buf b{total, bytes};
        total += (bytes + 255) / 256 * 256;
        return b;
    }
};

// residual-norm partial sums per instance (slices of NORM_SLICE squares)
int norm_rb(const Global &G) { return std::max(1, (G.max_inst_cells + NORM_SLICE - 1) / NORM_SLICE); }

WsMap layout(const Global &G, int ninst, const igks_options &o, int hist_cap)
{
    Layout L;
    WsMap w;
    const size_t N = G.N, F = G.F, E = (size_t)MAXV * G.NB, D = sizeof(double),
                 I = sizeof(int), NI = ninst, NW = std::max(1, G.nwall);
    w.ip = L.add(NI * sizeof(InstParam));
    w.is = L.add(NI * sizeof(InstScalars));
    w.slot = L.add(NI * NSL * NSLOT * SLOT_STRIDE * sizeof(unsigned long long));
    w.Wa = L.add(5 * N * D); w.Wb = L.add(5 * N * D);
    w.grad = L.add(8 * N * D); w.lamc = L.add(N * D); w.vort = L.add(N * D); w.nu = L.add(N * D);
    w.phi = L.add(4 * N * D);
    w.M = L.add(5 * N * D); w.lsum = L.add(N * D); w.sadiag = L.add(N * D); w.r2 = L.add(2 * N * D);
    w.dW = L.add(5 * N * (o.precision == IGKS_MIXED ? sizeof(float) : D));
    // the first pass's increments (two block passes)
    w.dW1 = L.add(o.block_passes == 2 ? 5 * N * (o.precision == IGKS_MIXED ? sizeof(float) : D) : 0);
    // the inverted 4x4 LU-SGS diagonal blocks (Roe-matrix operator)
    w.dinv = L.add(o.lusgs_op >= 1 && o.scheme == 0 ? 16 * N * (o.precision == IGKS_MIXED ? sizeof(float) : D) : 0);
    w.xc = L.add(N * D); w.yc = L.add(N * D); w.area = L.add(N * D); w.lsinv = L.add(3 * N * D);
    w.dwall = L.add(N * D); w.vtx = L.add(2 * MAXV * (size_t)G.NB * D);
    w.cinst = L.add(N * I); w.finst = L.add(F * I); w.icell = L.add(N * I); w.ioff = L.add((NI + 1) * I);
    w.g2i = L.add(N * I);
    w.cf_face = L.add(E * I); w.cf_nbr = L.add(E * I); w.cf_flag = L.add(E * I);
    w.cf_dx = L.add(E * D); w.cf_dy = L.add(E * D);
    w.fl = L.add(F * I); w.fr = L.add(F * I); w.fbc = L.add(F * I);
    w.fnx = L.add(F * D); w.fny = L.add(F * D); w.flen = L.add(F * D); w.frl = L.add(2 * F * D);
    w.frr = L.add(2 * F * D); w.fidl = L.add(F * D); w.fidr = L.add(F * D); w.firn = L.add(F * D);
    w.frec = L.add(FR_STRIDE * F * D); w.flam = L.add(F * D); w.fsak = L.add(F * D);
    w.enx = L.add(E * D); w.eny = L.add(E * D); w.es = L.add(E * D);
    w.ipart = L.add(2 * NI * (size_t)norm_rb(G) * D);
    w.ipos = L.add(N * I);
    w.cperm = L.add(N * I);
    w.hist = L.add((size_t)HIST_W * NI * hist_cap * D);
    w.wall_faces = L.add(NW * I);
    w.wall_out = L.add(4 * NW * D);
    w.woff = L.add((NI + 1) * I);
    w.wseg = L.add(4 * NW * D);
    w.lev_off = L.add((size_t)(G.nlev + 1) * I);
    w.bl_off = L.add(G.bl_off.size() * I);
    w.bl_lo = L.add(std::max<size_t>(1, G.bl_lo.size()) * I);
    w.bl_hi = L.add(std::max<size_t>(1, G.bl_hi.size()) * I);
    w.stage = L.add(5 * (size_t)std::max(1, G.max_inst_cells) * D);
    w.backup = L.add(10 * N * D + NI * sizeof(InstScalars));
    w.total = L.total;
    return w;
}

int hist_cap_of(const igks_options &o) { return std::max(1, o.chunk > 0 ? o.chunk : 64); }

template <typename T>
void fill_params(igks_ctx *c, Params<T> &P)
{
    const WsMap &w = c->w;
    char *b = c->ws;
    auto D = [&](const Buf &x) { return (double *)(b + x.off); };
    auto In = [&](const Buf &x) { return (int *)(b + x.off); };
    P = Params<T>{};
    P.nc = c->g.N; P.nf = c->g.F; P.ninst = (int)c->inst.size();
    P.limiter = c->opt.limiter; P.visc_sr = c->opt.visc_sr; P.mu_law = c->opt.mu_law;
    P.cfl_mode = c->opt.scheme == 1 ? 1 : c->opt.cfl_mode;   // the explicit scheme keeps its CFL
    P.cfl_init = c->opt.cfl_init; P.cfl_min = c->opt.cfl_min; P.cfl_max = c->opt.cfl_max; P.cfl_flux = c->opt.cfl_flux;
    P.limiter_freeze = c->opt.limiter_freeze; P.phi = D(w.phi); P.tau_jump = c->opt.tau_jump;
    P.cinst = In(w.cinst); P.finst = In(w.finst);
    P.ip = (const InstParam *)(b + w.ip.off);
    P.is = (InstScalars *)(b + w.is.off);
    P.slot = (unsigned long long *)(b + w.slot.off);
    P.Wa = D(w.Wa); P.Wb = D(w.Wb); P.grad = D(w.grad); P.lamc = D(w.lamc); P.vort = D(w.vort); P.nu = D(w.nu);
    P.M = D(w.M); P.lsum = D(w.lsum); P.sadiag = D(w.sadiag); P.r2 = D(w.r2); P.dW = (T *)(b + w.dW.off);
    P.dWx = nullptr;
    P.dinv = c->opt.lusgs_op >= 1 && c->opt.scheme == 0 ? (T *)(b + w.dinv.off) : nullptr;
    P.roe_kin = c->opt.lusgs_op == 2;
    P.xc = D(w.xc); P.yc = D(w.yc); P.area = D(w.area); P.lsinv = D(w.lsinv); P.dwall = D(w.dwall); P.vtx = D(w.vtx);
    P.nb = c->g.NB;
    P.cf_face = In(w.cf_face); P.cf_nbr = In(w.cf_nbr); P.cf_flag = In(w.cf_flag);
    P.cf_dx = D(w.cf_dx); P.cf_dy = D(w.cf_dy);
    P.fl = In(w.fl); P.fr = In(w.fr); P.fbc = In(w.fbc);
    P.fnx = D(w.fnx); P.fny = D(w.fny); P.flen = D(w.flen); P.frl = D(w.frl); P.frr = D(w.frr);
    P.fidl = D(w.fidl); P.fidr = D(w.fidr); P.firn = D(w.firn);
    P.frec = D(w.frec); P.flam = D(w.flam); P.fsak = D(w.fsak);
    P.enx = D(w.enx); P.eny = D(w.eny); P.es = D(w.es);
    P.icell = In(w.icell); P.ioff = In(w.ioff); P.ipos = In(w.ipos); P.cperm = In(w.cperm); P.ipart = D(w.ipart); P.rb = norm_rb(c->g);
    P.hist = D(w.hist); P.hist_cap = c->hist_cap;
}

Launch launch_of(igks_ctx *c)
{
    Launch L;
    L.s = c->stream;
    for (int k = 0; k < NCLASS; k++) L.block[k] = c->block[k];
    L.flux_pair = c->flux_pair;
    return L;
}

// queue one nonlinear iteration of every instance
template <typename T>
void queue_iteration(igks_ctx *c, const Params<T> &P, hipEvent_t *ev, int it)
{
    Launch L = launch_of(c);
    const int *lev = (const int *)(c->ws + c->w.lev_off.off);
    const Global &G = c->g;
    const int lev1 = G.nlev > 1 ? G.lev_off[1] : 0;   // cells of the first wavefront
    auto mark = [&](int k) { if (ev) (void)hipEventRecord(ev[k], c->stream); };
    mark(0);
    launch_prep(L, P);
    mark(1);
    launch_flux(L, P);
    mark(2);
    launch_gather(L, P);
    mark(3);
    launch_reduce(L, P, it);
    mark(4);
    if (c->opt.scheme == 1) {
        // explicit scheme: one update kernel in place of the sweeps
        launch_explicit(L, P);
        mark(5);
        launch_commit(L, P, it);
        mark(6);
        return;
    }
    // Roe-matrix operator: the inverted diagonal blocks, which need the CFL
    // number the reduction has just set (timed with the forward sweep)
    if (P.dinv) launch_roe_diag(L, P);
    const int *blo = (const int *)(c->ws + c->w.bl_off.off), *bll = (const int *)(c->ws + c->w.bl_lo.off),
              *blh = (const int *)(c->ws + c->w.bl_hi.off);
    const int ngb = (int)G.bl_off.size() - 1;
    if (c->sweep_mode == 3 && two_block_passes(c)) {
        // a first block pass into the second increment array, then the
        // second pass with its cross-block terms (the forward class holds
        // the first pass and the second forward sweep)
        Params<T> P1 = P;
        P1.dW = (T *)(c->ws + c->w.dW1.off);
        P1.dWx = nullptr;
        launch_sweep_blk(L, P1, blo, bll, blh, ngb, true);
        launch_sweep_blk(L, P1, blo, bll, blh, ngb, false, false);
        Params<T> P2 = P;
        P2.dWx = P1.dW;
        launch_sweep_blk(L, P2, blo, bll, blh, ngb, true);
    } else if (c->sweep_mode == 3) launch_sweep_blk(L, P, blo, bll, blh, ngb, true);
    else if (c->sweep_mode == 2) launch_sweep_wg(L, P, lev, G.nlev, true);
    else
        // forward over the wavefronts after the first (whose forward
        // increments D^-1 M are formed where they are read); the last one
        // also takes its backward step (only ghosts lie above it)
        for (int l = G.nlev > 1 ? 1 : 0; l < G.nlev; l++)
            launch_sweep(L, P, G.lev_off[l], G.lev_off[l + 1], l + 1 < G.nlev ? 0 : 2, lev1);
    mark(5);
    // backward sweep with the update
    if (c->sweep_mode == 3) launch_sweep_blk(L, P, blo, bll, blh, ngb, false);
    else if (c->sweep_mode == 2) launch_sweep_wg(L, P, lev, G.nlev, false);
    else
        for (int l = G.nlev - 2; l >= 0; l--) launch_sweep(L, P, G.lev_off[l], G.lev_off[l + 1], 1, lev1);
    mark(6);   // the backward sweeps' class ends here; the commit belongs to no class
    launch_commit(L, P, it);
}

template <typename T>
void queue_residual(igks_ctx *c, const Params<T> &P)
{
    Launch L = launch_of(c);
    launch_prep(L, P);
    launch_flux(L, P);
    launch_gather(L, P);
}

int sync_scalars(igks_ctx *c)
{
    const size_t ni = c->inst.size();
    c->hs.resize(ni);
    HIPCHK(c, hipMemcpyAsync(c->hs.data(), c->P64.is, sizeof(InstScalars) * ni, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return IGKS_OK;
}

// k iterations of every instance, then the scalars and the history entries
template <typename T>
int run_chunk(igks_ctx *c, const Params<T> &P, int k)
{
    if (c->profiling) {
        hipEvent_t ev[NKT + 1];
        for (auto &e : ev) HIPCHK(c, hipEventCreate(&e));
        for (int i = 0; i < k; i++) {
            queue_iteration(c, P, ev, i);
            HIPCHK(c, hipEventSynchronize(ev[NKT]));
            for (int j = 0; j < NKT; j++) {
                float ms = 0;
                (void)hipEventElapsedTime(&ms, ev[j], ev[j + 1]);
                c->ktimes[j] += ms;
            }
        }
        for (auto &e : ev) (void)hipEventDestroy(e);
    } else if (k > 0 && k == graph_chunk(c)) {
        if (c->gexec && c->gexec_k != k) destroy_graph(c);
        if (!c->gexec) {
            hipGraph_t g;
            HIPCHK(c, hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
            for (int i = 0; i < k; i++) queue_iteration(c, P, nullptr, i);
            HIPCHK(c, hipStreamEndCapture(c->stream, &g));
            hipError_t e = hipGraphInstantiate(&c->gexec, g, nullptr, nullptr, 0);
            (void)hipGraphDestroy(g);
            if (e != hipSuccess) {
                c->gexec = nullptr;
                return fail(c, IGKS_EHIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
            }
            c->gexec_k = k;
        }
        HIPCHK(c, hipGraphLaunch(c->gexec, c->stream));
    } else {
        for (int i = 0; i < k; i++) queue_iteration(c, P, nullptr, i);
    }
    HIPCHK(c, hipGetLastError());
    const size_t ni = c->inst.size();
    std::vector<int> n0(ni), h0(ni);
    for (size_t i = 0; i < ni; i++) { n0[i] = c->hs[i].ncommit; h0[i] = c->hs[i].halt; }
    int rc = sync_scalars(c);
    if (rc) return rc;
    const int nh = std::min(k, c->hist_cap);
    if (nh > 0) {
        std::vector<double> h((size_t)HIST_W * ni * nh);
        HIPCHK(c, hipMemcpyAsync(h.data(), P.hist, sizeof(double) * h.size(), hipMemcpyDeviceToHost, c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
        c->hist.resize(ni);
        for (size_t i = 0; i < ni; i++) {
            // entries of the iterations this instance ran: the committed ones
            // and the rejected one that froze it
            int ran = c->hs[i].ncommit - n0[i] + ((c->hs[i].halt && !h0[i]) ? 1 : 0);
            for (int e = 0; e < std::min(nh, ran); e++) {
                const double *src = &h[(size_t)HIST_W * ((size_t)e * ni + i)];
                c->hist[i].insert(c->hist[i].end(), src, src + HIST_W);
            }
        }
    }
    return IGKS_OK;
}

int check_inst(const igks_ctx *c, int inst)
{
    if (!c) return IGKS_EINVAL;
    if (inst < 0 || inst >= (int)c->inst.size())
        return fail(const_cast<igks_ctx *>(c), IGKS_EINVAL, "instance index out of range");
    return IGKS_OK;
}

int check_ready(igks_ctx *c, bool need_flow)
{
    if (!c) return IGKS_EINVAL;
    for (size_t i = 0; i < c->inst.size(); i++)
        if (!c->inst[i].ok) return fail(c, IGKS_EINVAL, "no mesh uploaded for instance " + std::to_string(i));
    if (!c->bound) return fail(c, IGKS_EINVAL, "no workspace bound");
    if (c->static_dev >= 0) {
        std::lock_guard<std::mutex> lk(static_mu);
        if (static_ws[c->static_dev].gen != c->static_gen) {
            c->bound = false;
            return fail(c, IGKS_EINVAL, "the static workspace was bound to another context since; bind a workspace again");
        }
    }
    if (need_flow)
        for (size_t i = 0; i < c->inst.size(); i++)
            if (!c->inst[i].have_flow)
                return fail(c, IGKS_EINVAL, "set the free stream of instance " + std::to_string(i) + " first");
    return IGKS_OK;
}

// the context is bound and instance inst has its free stream
int check_inst_ready(igks_ctx *c, int inst)
{
    int rc = check_inst(c, inst);
    if (rc) return rc;
    rc = check_ready(c, false);
    if (rc) return rc;
    if (!c->inst[inst].have_flow)
        return fail(c, IGKS_EINVAL, "set the free stream of instance " + std::to_string(inst) + " first");
    return IGKS_OK;
}

int ensure_combined(igks_ctx *c)
{
    for (size_t i = 0; i < c->inst.size(); i++)
        if (!c->inst[i].ok) return fail(c, IGKS_EINVAL, "no mesh uploaded for instance " + std::to_string(i));
    if (!c->combined) {
        int rc = combine(c);
        if (rc) return rc;
        c->hist_cap = hist_cap_of(c->opt);
    }
    return IGKS_OK;
}

// internal ids of instance i's cells in its upload order (device)
const int *inst_cells(igks_ctx *c, int i) { return (const int *)(c->ws + c->w.g2i.off) + c->g.coff[i]; }

double *cur_buffer(igks_ctx *c, int i) { return (c->hs[i].ncommit & 1) ? c->P64.Wb : c->P64.Wa; }

double *stage_buffer(igks_ctx *c) { return (double *)(c->ws + c->w.stage.off); }

// FARFIELD faces: free stream where V_inf . n < 0, else Riemann outflow
int upload_bc(igks_ctx *c)
{
    std::vector<int> fbc(c->g.ftag);
    for (int q = 0; q < c->g.F; q++)
        if (fbc[q] == BC_FARFIELD) {
            const InstParam &ip = c->inst[c->g.finst[q]].ip;
            fbc[q] = (ip.Winf[1] * c->g.fnx[q] + ip.Winf[2] * c->g.fny[q] < 0.0) ? BC_FREESTREAM : BC_OUTFLOW;
        }
    HIPCHK(c, hipMemcpyAsync(c->ws + c->w.fbc.off, fbc.data(), sizeof(int) * c->g.F, hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return IGKS_OK;
}

// fresh scalars of one instance: iteration counter 0 or a checkpoint's
InstScalars fresh_scalars(const igks_scalars *sc)
{
    InstScalars s;
    std::memset(&s, 0, sizeof s);
    if (sc) {
        s.ncommit = sc->iteration;
        s.cfl = sc->cfl;
        s.res_inf_prev = sc->res_inf_prev;
        s.res0 = sc->res0;
    }
    return s;
}

template <typename T>
int iterate_impl(igks_ctx *c, const Params<T> &P, int n, int *n_done)
{
    const size_t ni = c->inst.size();
    c->hist.assign(ni, std::vector<double>());
    for (double &t : c->ktimes) t = 0.0;
    std::vector<int> was_halted(ni);
    for (size_t i = 0; i < ni; i++) was_halted[i] = c->hs[i].halt;
    const int start0 = c->hs[0].ncommit;
    int executed = 0;
    while (executed < n) {
        const int gc = graph_chunk(c);
        int k = gc > 0 ? std::min(gc, n - executed) : n - executed;
        if (c->profiling) k = std::min(k, 64);
        int rc = run_chunk(c, P, k);
        if (rc) return rc;
        executed += k;
        if (n_done) *n_done = c->hs[0].ncommit - start0;
        bool all = true;
        for (size_t i = 0; i < ni; i++) all = all && c->hs[i].halt;
        if (all) break;
    }
    if (c->profiling && executed > 0)
        for (double &t : c->ktimes) t /= executed;
    std::string frozen;
    bool all = true;
    for (size_t i = 0; i < ni; i++) {
        all = all && c->hs[i].halt;
        if (c->hs[i].halt && !was_halted[i]) frozen += (frozen.empty() ? "" : ", ") + std::to_string(i);
    }
    if (!frozen.empty())
        return fail(c, IGKS_ENONPHYS, "non-physical update (rho <= 0, p <= 0 or non-finite) rejected; instance(s) " +
                                          frozen + " frozen at their last committed state");
    if (all && n > 0) return fail(c, IGKS_ENONPHYS, "every instance is frozen; set a state or a free stream");
    return IGKS_OK;
}

template <typename T>
int tune_run(igks_ctx *c, const Params<T> &P, int iters)
{
    c->profiling = true;
    for (double &x : c->ktimes) x = 0.0;
    int rc = run_chunk(c, P, iters);
    c->profiling = false;
    return rc;
}

}  // namespace

// ====================================================================== C ABI

// `reps` launches of one residual-phase kernel class back to back between
// two events, after the launches that produce its inputs; the classes timed
// here read the state and write only derived arrays and idempotent min/max
// slots, which are cleared afterwards, so the iteration is unaffected
template <typename T>
static int time_class(igks_ctx *c, const Params<T> &P, int klass, int reps, double *ms)
{
    Launch L = launch_of(c);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    HIPCHK(c, hipEventCreate(&e0));
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return fail(c, IGKS_EHIP, "hipEventCreate failed");
    }
    launch_reset(L, P, 1, -1);
    if (klass >= 1) launch_prep(L, P);
    if (klass >= 2) launch_flux(L, P);
    (void)hipEventRecord(e0, c->stream);
    for (int r = 0; r < reps; r++) {
        if (klass == 0) launch_prep(L, P);
        else if (klass == 1) launch_flux(L, P);
        else launch_gather(L, P);
    }
    (void)hipEventRecord(e1, c->stream);
    launch_reset(L, P, 1, -1);
    hipError_t err = hipGetLastError();
    if (err == hipSuccess) err = hipEventSynchronize(e1);
    float t = 0.0f;
    if (err == hipSuccess) err = hipEventElapsedTime(&t, e0, e1);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (err != hipSuccess) return fail(c, IGKS_EHIP, std::string("kernel timing: ") + hipGetErrorString(err));
    *ms = (double)t / reps;
    return IGKS_OK;
}

extern "C" {

void igks_default_options(igks_options *o)
{
    if (!o) return;
    o->precision = IGKS_FP64;
    o->limiter = 0;
    o->cfl_init = 1000.0;
    o->cfl_min = 1.0;
    o->cfl_max = 1e6;
    o->cfl_mode = 0;
    o->cfl_flux = 1.0;
    o->visc_sr = 1;
    o->mu_law = 0;
    o->chunk = 20;
    o->block = 256;
    o->sweep = 0;
    o->flux_lanes = 0;
    o->scheme = 0;
    o->wall_temp = 0.0;
    o->limiter_freeze = 0.0;
    o->tau_jump = 0;
    o->block_passes = 1;
    o->lusgs_op = 0;
}

int igks_batch_create(igks_ctx **out, const igks_options *opt, void *hip_stream, int32_t n_inst)
{
    if (!out) return IGKS_EINVAL;
    *out = nullptr;
    if (n_inst < 1) return IGKS_EINVAL;
    igks_ctx *c = new (std::nothrow) igks_ctx();
    if (!c) return IGKS_ENOMEM;
    if (opt) c->opt = *opt; else igks_default_options(&c->opt);
    if (c->opt.precision != IGKS_FP64 && c->opt.precision != IGKS_MIXED) { delete c; return IGKS_EINVAL; }
    if (c->opt.block <= 0) c->opt.block = 256;
    if (c->opt.block % 64 != 0 || c->opt.block > 256) { delete c; return IGKS_EINVAL; }
    if (c->opt.sweep < 0 || c->opt.sweep > 3 || c->opt.chunk < 0) { delete c; return IGKS_EINVAL; }
    if (c->opt.flux_lanes < 0 || c->opt.flux_lanes > 2) { delete c; return IGKS_EINVAL; }
    if (c->opt.scheme < 0 || c->opt.scheme > 1) { delete c; return IGKS_EINVAL; }
    if (!(c->opt.wall_temp >= 0.0) || !std::isfinite(c->opt.wall_temp)) { delete c; return IGKS_EINVAL; }
    if (!(c->opt.limiter_freeze >= 0.0) || !(c->opt.limiter_freeze < 1.0)) { delete c; return IGKS_EINVAL; }
    if (c->opt.tau_jump < 0 || c->opt.tau_jump > 1) { delete c; return IGKS_EINVAL; }
    if (c->opt.block_passes == 0) c->opt.block_passes = 1;
    if (c->opt.block_passes < 1 || c->opt.block_passes > 2) { delete c; return IGKS_EINVAL; }
    if (c->opt.block_passes == 2 && c->opt.sweep != 0 && c->opt.sweep != 3) { delete c; return IGKS_EINVAL; }
    if (c->opt.lusgs_op < 0 || c->opt.lusgs_op > 2) { delete c; return IGKS_EINVAL; }
    for (int k = 0; k < NCLASS; k++) c->block[k] = c->opt.block;
    if (hip_stream) {
        c->stream = (hipStream_t)hip_stream;
    } else {
        if (hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking) != hipSuccess) { delete c; return IGKS_EHIP; }
        c->own_stream = true;
    }
    c->inst.resize(n_inst);
    c->hs.resize(n_inst);
    c->hist.resize(n_inst);
    *out = c;
    return IGKS_OK;
}

int igks_create(igks_ctx **out, const igks_options *opt, void *hip_stream)
{
    return igks_batch_create(out, opt, hip_stream, 1);
}

void igks_destroy(igks_ctx *c)
{
    if (!c) return;
    destroy_graph(c);
    if (c->own_stream && c->stream) (void)hipStreamDestroy(c->stream);
    delete c;
}

const char *igks_last_error(const igks_ctx *c) { return c ? c->err.c_str() : "null context"; }

int igks_batch_mesh_upload(igks_ctx *c, int32_t inst, int32_t n_nodes, const double *xy, int32_t n_cells,
                           const int32_t *cell_ptr, const int32_t *cell_nodes, int32_t n_bfaces,
                           const int32_t *bface_nodes, const int32_t *bface_tag)
{
    int rc = check_inst(c, inst);
    if (rc) return rc;
    destroy_graph(c);
    c->bound = false;
    c->combined = false;
    for (auto &m : c->inst) m.have_flow = false;
    InstMesh m;
    rc = build_instance(c, n_nodes, xy, n_cells, cell_ptr, cell_nodes, n_bfaces, bface_nodes, bface_tag, m);
    c->inst[inst] = rc ? InstMesh() : std::move(m);
    return rc;
}

int igks_mesh_upload(igks_ctx *c, int32_t n_nodes, const double *xy, int32_t n_cells, const int32_t *cell_ptr,
                     const int32_t *cell_nodes, int32_t n_bfaces, const int32_t *bface_nodes,
                     const int32_t *bface_tag)
{
    return igks_batch_mesh_upload(c, 0, n_nodes, xy, n_cells, cell_ptr, cell_nodes, n_bfaces, bface_nodes, bface_tag);
}

int igks_set_sweep_blocks(igks_ctx *c, int32_t inst, const int32_t *block_of_cell)
{
    int rc = check_inst(c, inst);
    if (rc) return rc;
    InstMesh &m = c->inst[inst];
    if (!m.ok) return fail(c, IGKS_EINVAL, "no mesh uploaded for instance " + std::to_string(inst));
    if (block_of_cell)
        for (int i = 0; i < m.nc; i++)
            if (block_of_cell[i] < 0) return fail(c, IGKS_EINVAL, "negative sweep block at cell " + std::to_string(i));
    destroy_graph(c);
    c->bound = false;
    c->combined = false;
    for (auto &x : c->inst) x.have_flow = false;
    if (block_of_cell) m.sblk.assign(block_of_cell, block_of_cell + m.nc);
    else m.sblk.clear();
    compute_levels(m);
    return IGKS_OK;
}

int igks_mesh_info(const igks_ctx *cc, int32_t *nc, int32_t *nf, int32_t *nw, int32_t *nl)
{
    igks_ctx *c = const_cast<igks_ctx *>(cc);   // combining the instances is cached
    if (!c) return IGKS_EINVAL;
    int rc = ensure_combined(c);
    if (rc) return rc;
    if (nc) *nc = c->g.N;
    if (nf) *nf = c->g.F;
    if (nw) *nw = c->g.nwall;
    if (nl) *nl = c->g.nlev;
    return IGKS_OK;
}

int igks_wavefront_sizes(const igks_ctx *cc, int32_t *sizes, int32_t cap)
{
    igks_ctx *c = const_cast<igks_ctx *>(cc);
    if (!c || !sizes || cap < 1) return IGKS_EINVAL;
    int rc = ensure_combined(c);
    if (rc) return rc;
    const int n = std::min<int>(cap, c->g.nlev);
    for (int l = 0; l < n; l++) sizes[l] = c->g.lev_off[l + 1] - c->g.lev_off[l];
    return IGKS_OK;
}

int igks_batch_mesh_info(const igks_ctx *c, int32_t inst, int32_t *nc, int32_t *nf, int32_t *nw)
{
    int rc = check_inst(c, inst);
    if (rc) return rc;
    const InstMesh &m = c->inst[inst];
    if (!m.ok) return fail(const_cast<igks_ctx *>(c), IGKS_EINVAL, "no mesh uploaded for this instance");
    if (nc) *nc = m.nc;
    if (nf) *nf = (int)m.uf.size();
    if (nw) *nw = (int)m.wall_uf.size();
    return IGKS_OK;
}

int igks_workspace_size(const igks_ctx *cc, size_t *bytes)
{
    igks_ctx *c = const_cast<igks_ctx *>(cc);
    if (!c || !bytes) return IGKS_EINVAL;
    int rc = ensure_combined(c);
    if (rc) return rc;
    *bytes = layout(c->g, (int)c->inst.size(), c->opt, c->hist_cap).total;
    return IGKS_OK;
}

int igks_bind_workspace(igks_ctx *c, void *dptr, size_t bytes)
{
    if (!c) return IGKS_EINVAL;
    int rc = ensure_combined(c);
    if (rc) return rc;
    WsMap w = layout(c->g, (int)c->inst.size(), c->opt, c->hist_cap);
    if (!dptr || bytes < w.total) return fail(c, IGKS_ENOMEM, "workspace smaller than igks_workspace_size");
    if (((uintptr_t)dptr) % 256 != 0) return fail(c, IGKS_EINVAL, "workspace must be 256-byte aligned");
    destroy_graph(c);
    c->bound = false;
    c->static_dev = -1;
    c->ws = (char *)dptr;
    c->ws_bytes = bytes;
    c->w = w;
    fill_params(c, c->P64);
    fill_params(c, c->P32);
    const Global &G = c->g;
    char *b = c->ws;
    auto up = [&](const Buf &x, const void *src, size_t n) -> int {
        if (n == 0) return IGKS_OK;
        HIPCHK(c, hipMemcpyAsync(b + x.off, src, n, hipMemcpyHostToDevice, c->stream));
        return IGKS_OK;
    };
    const size_t D = sizeof(double), I = sizeof(int), N = G.N, F = G.F, E = (size_t)MAXV * G.NB;
    rc = 0;
    rc |= up(w.xc, G.xc.data(), N * D); rc |= up(w.yc, G.yc.data(), N * D); rc |= up(w.area, G.area.data(), N * D);
    rc |= up(w.lsinv, G.lsinv.data(), 3 * N * D); rc |= up(w.vtx, G.vtx.data(), G.vtx.size() * D);
    rc |= up(w.cinst, G.cinst.data(), N * I); rc |= up(w.finst, G.finst.data(), F * I);
    rc |= up(w.icell, G.icell.data(), N * I); rc |= up(w.ioff, G.ioff.data(), G.ioff.size() * I);
    rc |= up(w.ipos, G.ipos.data(), N * I);
    rc |= up(w.cperm, G.cperm.data(), N * I);
    rc |= up(w.g2i, G.g2i.data(), N * I);
    rc |= up(w.cf_face, G.cf_face.data(), E * I);
    rc |= up(w.cf_nbr, G.cf_nbr.data(), E * I); rc |= up(w.cf_flag, G.cf_flag.data(), E * I);
    rc |= up(w.cf_dx, G.cf_dx.data(), E * D); rc |= up(w.cf_dy, G.cf_dy.data(), E * D);
    rc |= up(w.enx, G.enx.data(), E * D); rc |= up(w.eny, G.eny.data(), E * D); rc |= up(w.es, G.es.data(), E * D);
    rc |= up(w.fl, G.fl.data(), F * I); rc |= up(w.fr, G.fr.data(), F * I); rc |= up(w.fbc, G.ftag.data(), F * I);
    rc |= up(w.fnx, G.fnx.data(), F * D); rc |= up(w.fny, G.fny.data(), F * D); rc |= up(w.flen, G.flen.data(), F * D);
    rc |= up(w.frl, G.frl.data(), 2 * F * D); rc |= up(w.frr, G.frr.data(), 2 * F * D);
    {
        // the kernels multiply by the inverse distances
        std::vector<double> idl(F), idr(F), irn(F);
        for (int q = 0; q < F; q++) { idl[q] = 1.0 / G.fdl[q]; idr[q] = 1.0 / G.fdr[q]; irn[q] = 1.0 / G.frn[q]; }
        rc |= up(w.fidl, idl.data(), F * D); rc |= up(w.fidr, idr.data(), F * D); rc |= up(w.firn, irn.data(), F * D);
    }
    rc |= up(w.wall_faces, G.wall_faces.data(), G.wall_faces.size() * I);
    rc |= up(w.woff, G.woff.data(), G.woff.size() * I);
    rc |= up(w.wseg, G.wseg.data(), G.wseg.size() * D);
    rc |= up(w.lev_off, G.lev_off.data(), G.lev_off.size() * I);
    rc |= up(w.bl_off, G.bl_off.data(), G.bl_off.size() * I);
    rc |= up(w.bl_lo, G.bl_lo.data(), G.bl_lo.size() * I);
    rc |= up(w.bl_hi, G.bl_hi.data(), G.bl_hi.size() * I);
    if (rc) return rc;
    c->sweep_mode = auto_sweep_mode(c);
    c->flux_pair = auto_flux_pair(c);
    // instance parameters and scalars start zeroed (no free stream yet)
    std::vector<InstParam> ip0(c->inst.size());
    std::memset(ip0.data(), 0, sizeof(InstParam) * ip0.size());
    for (auto &m : c->inst) std::memset(&m.ip, 0, sizeof m.ip);
    rc = up(w.ip, ip0.data(), sizeof(InstParam) * ip0.size());
    if (rc) return rc;
    Launch L = launch_of(c);
    launch_wall_distance(L, G.N, c->P64.xc, c->P64.yc, c->P64.cinst, (const int *)(b + w.woff.off),
                         (const double *)(b + w.wseg.off), (double *)(b + w.dwall.off));
    launch_reset(L, c->P64, 15, -1);
    HIPCHK(c, hipGetLastError());
    HIPCHK(c, hipStreamSynchronize(c->stream));
    c->bound = true;
    for (auto &m : c->inst) m.have_flow = false;
    for (auto &h : c->hist) h.clear();
    return sync_scalars(c);
}

int igks_bind_static_workspace(igks_ctx *c)
{
    if (!c) return IGKS_EINVAL;
    int rc = ensure_combined(c);
    if (rc) return rc;
    const size_t need = layout(c->g, (int)c->inst.size(), c->opt, c->hist_cap).total;
    if (need > STATIC_WS_BYTES)
        return fail(c, IGKS_ENOMEM, "the mesh needs a workspace of " + std::to_string(need) +
                                        " bytes; the static workspace holds " + std::to_string(STATIC_WS_BYTES));
    int dev = -1;
    HIPCHK(c, hipGetDevice(&dev));
    if (dev < 0 || dev >= MAX_DEVICES) return fail(c, IGKS_EINVAL, "device index out of range");
    void *ptr = nullptr;
    unsigned long long gen = 0;
    {
        std::lock_guard<std::mutex> lk(static_mu);
        if (!static_ws[dev].ptr) {
            void *p = nullptr;
            hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
            if (e != hipSuccess || !p)
                return fail(c, IGKS_EHIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
            static_ws[dev].ptr = p;
        }
        ptr = static_ws[dev].ptr;
        gen = ++static_ws[dev].gen;
    }
    rc = igks_bind_workspace(c, ptr, STATIC_WS_BYTES);
    if (rc) return rc;
    c->static_dev = dev;
    c->static_gen = gen;
    return IGKS_OK;
}

int igks_batch_set_freestream(igks_ctx *c, int32_t inst, double mach, double alpha_deg, double reynolds,
                              double nut_ratio)
{
    int rc = check_inst(c, inst);
    if (rc) return rc;
    rc = check_ready(c, false);
    if (rc) return rc;
    if (!(mach > 0) || !(reynolds > 0) || !std::isfinite(alpha_deg))
        return fail(c, IGKS_EINVAL, "mach and reynolds must be positive");
    InstMesh &m = c->inst[inst];
    m.alpha = alpha_deg;
    // non-dimensionalisation: rho_inf = 1, |V_inf| = 1, reference length 1
    InstParam &ip = m.ip;
    std::memset(&ip, 0, sizeof ip);
    const double pinf = 1.0 / (GAMMA * mach * mach);
    ip.p_inf = pinf;
    ip.tw = c->opt.wall_temp * pinf;   // RT = p / rho with rho_inf = 1
    ip.lam_inf = 1.0 / (2.0 * pinf);
    ip.mu_inf = 1.0 / reynolds;
    ip.sa = nut_ratio >= 0.0;
    const double a = alpha_deg * M_PI / 180.0;
    ip.Winf[0] = 1.0; ip.Winf[1] = std::cos(a); ip.Winf[2] = std::sin(a);
    ip.Winf[3] = pinf / (GAMMA - 1.0) + 0.5;
    ip.Winf[4] = ip.sa ? nut_ratio * ip.mu_inf : 0.0;
    HIPCHK(c, hipMemcpyAsync(c->ws + c->w.ip.off + inst * sizeof(InstParam), &ip, sizeof(InstParam),
                             hipMemcpyHostToDevice, c->stream));
    rc = upload_bc(c);
    if (rc) return rc;
    InstScalars s = fresh_scalars(nullptr);   // iteration 0 -> state buffer A
    HIPCHK(c, hipMemcpyAsync(c->P64.is + inst, &s, sizeof s, hipMemcpyHostToDevice, c->stream));
    Launch L = launch_of(c);
    launch_reset(L, c->P64, 1, inst);
    launch_fill_instance(L, m.nc, inst_cells(c, inst), c->g.N, ip.Winf, c->P64.Wa);
    HIPCHK(c, hipGetLastError());
    m.have_flow = true;
    c->hist[inst].clear();
    return sync_scalars(c);
}

int igks_set_freestream(igks_ctx *c, double mach, double alpha_deg, double reynolds, double nut_ratio)
{
    return igks_batch_set_freestream(c, 0, mach, alpha_deg, reynolds, nut_ratio);
}

int igks_iterate(igks_ctx *c, int32_t n, int32_t *n_done)
{
    if (n_done) *n_done = 0;
    int rc = check_ready(c, true);
    if (rc) return rc;
    if (n < 0) return fail(c, IGKS_EINVAL, "negative iteration count");
    return (c->opt.precision == IGKS_MIXED) ? iterate_impl(c, c->P32, n, n_done) : iterate_impl(c, c->P64, n, n_done);
}

int igks_batch_status(igks_ctx *c, int32_t inst, int32_t *halted)
{
    int rc = check_inst(c, inst);
    if (rc) return rc;
    if (halted) *halted = c->hs[inst].halt;
    return IGKS_OK;
}

int igks_batch_get_residual(igks_ctx *c, int32_t inst, igks_residual *out)
{
    int rc = check_inst_ready(c, inst);
    if (rc) return rc;
    if (!out) return IGKS_EINVAL;
    const InstScalars &s = c->hs[inst];
    out->iteration = s.ncommit;
    out->res_l2 = s.res_l2;
    out->res_drop = s.res0 > 0 ? s.res_l2 / s.res0 : 0.0;
    out->res_inf = s.res_inf;
    out->eq40 = s.e40;
    out->cfl = s.cfl;
    out->dt_flux = s.dt;
    out->sa_l2 = s.sa_l2;
    return IGKS_OK;
}

int igks_get_residual(igks_ctx *c, igks_residual *out) { return igks_batch_get_residual(c, 0, out); }

int igks_batch_get_history(igks_ctx *c, int32_t inst, double *out, int32_t max, int32_t *n_out)
{
    int rc = check_inst(c, inst);
    if (rc) return rc;
    int n = (int)(c->hist[inst].size() / HIST_W);
    n = std::max(0, std::min(n, (int)max));
    if (out && n > 0) std::memcpy(out, c->hist[inst].data(), sizeof(double) * HIST_W * n);
    if (n_out) *n_out = n;
    return IGKS_OK;
}

int igks_get_history(igks_ctx *c, double *out, int32_t max, int32_t *n_out)
{
    return igks_batch_get_history(c, 0, out, max, n_out);
}

int igks_batch_get_state(igks_ctx *c, int32_t inst, double *W)
{
    int rc = check_inst_ready(c, inst);
    if (rc) return rc;
    if (!W) return IGKS_EINVAL;
    const int n = c->inst[inst].nc;
    Launch L = launch_of(c);
    launch_copy_instance(L, n, inst_cells(c, inst), c->g.N, cur_buffer(c, inst), stage_buffer(c), false);
    HIPCHK(c, hipGetLastError());
    HIPCHK(c, hipMemcpyAsync(W, stage_buffer(c), sizeof(double) * 5 * n, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return IGKS_OK;
}

int igks_get_state(igks_ctx *c, double *W) { return igks_batch_get_state(c, 0, W); }

int igks_batch_set_state(igks_ctx *c, int32_t inst, const double *W, const igks_scalars *sc)
{
    int rc = check_inst_ready(c, inst);
    if (rc) return rc;
    if (!W) return IGKS_EINVAL;
    const int n = c->inst[inst].nc;
    for (int i = 0; i < n; i++) {
        double r = W[i], mx = W[n + i], my = W[2 * n + i], E = W[3 * n + i], t = W[4 * n + i];
        double p = E - 0.5 * (mx * mx + my * my) / r;
        if (!(r > 0) || !(p > 0) || !std::isfinite(t) || !std::isfinite(p))
            return fail(c, IGKS_ENONPHYS, "non-physical state at cell " + std::to_string(i));
    }
    if (sc && sc->iteration < 0) return fail(c, IGKS_EINVAL, "negative iteration count in the scalars");
    InstScalars s = fresh_scalars(sc);
    HIPCHK(c, hipMemcpyAsync(c->P64.is + inst, &s, sizeof s, hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(stage_buffer(c), W, sizeof(double) * 5 * n, hipMemcpyHostToDevice, c->stream));
    Launch L = launch_of(c);
    launch_reset(L, c->P64, 1, inst);
    launch_copy_instance(L, n, inst_cells(c, inst), c->g.N, stage_buffer(c), (s.ncommit & 1) ? c->P64.Wb : c->P64.Wa,
                         true);
    HIPCHK(c, hipGetLastError());
    c->hist[inst].clear();
    return sync_scalars(c);
}

int igks_set_state(igks_ctx *c, const double *W, const igks_scalars *sc) { return igks_batch_set_state(c, 0, W, sc); }

int igks_batch_get_scalars(igks_ctx *c, int32_t inst, igks_scalars *out)
{
    int rc = check_inst_ready(c, inst);
    if (rc) return rc;
    if (!out) return IGKS_EINVAL;
    out->iteration = c->hs[inst].ncommit;
    out->cfl = c->hs[inst].cfl;
    out->res_inf_prev = c->hs[inst].res_inf_prev;
    out->res0 = c->hs[inst].res0;
    return IGKS_OK;
}

int igks_get_scalars(igks_ctx *c, igks_scalars *out) { return igks_batch_get_scalars(c, 0, out); }

// residual evaluation of every live instance without advancing the iteration
static int eval_residual(igks_ctx *c, int inst)
{
    // the kernels run over every instance, so every instance needs its flow
    int rc = check_inst(c, inst);
    if (rc) return rc;
    rc = check_ready(c, true);
    if (rc) return rc;
    if (c->hs[inst].halt) return fail(c, IGKS_ENONPHYS, "instance is frozen after a rejected update");
    Launch L = launch_of(c);
    launch_reset(L, c->P64, 1, -1);
    queue_residual(c, c->P64);
    launch_reset(L, c->P64, 1, -1);
    HIPCHK(c, hipGetLastError());
    return IGKS_OK;
}

int igks_batch_compute_residual(igks_ctx *c, int32_t inst, double *M)
{
    int rc = eval_residual(c, inst);
    if (rc) return rc;
    const int n = c->inst[inst].nc;
    Launch L = launch_of(c);
    launch_copy_instance(L, n, inst_cells(c, inst), c->g.N, c->P64.M, stage_buffer(c), false);
    HIPCHK(c, hipGetLastError());
    if (M) HIPCHK(c, hipMemcpyAsync(M, stage_buffer(c), sizeof(double) * 5 * n, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return IGKS_OK;
}

int igks_compute_residual(igks_ctx *c, double *M) { return igks_batch_compute_residual(c, 0, M); }

int igks_batch_get_wall_loads(igks_ctx *c, int32_t inst, double *cl, double *cd, double *cf, double *cp, double *xw)
{
    int rc = eval_residual(c, inst);
    if (rc) return rc;
    const int w0 = c->g.woff[inst], nw = c->g.woff[inst + 1] - w0;
    double *wout = (double *)(c->ws + c->w.wall_out.off);
    Launch L = launch_of(c);
    launch_gather_faces(L, nw, (const int *)(c->ws + c->w.wall_faces.off) + w0, c->P64.frec, c->g.F, wout);
    HIPCHK(c, hipGetLastError());
    std::vector<double> fw(4 * (size_t)std::max(nw, 1));
    if (nw > 0) HIPCHK(c, hipMemcpyAsync(fw.data(), wout, sizeof(double) * 4 * nw, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    const InstMesh &m = c->inst[inst];
    const double a = m.alpha * M_PI / 180.0, ca = std::cos(a), sa = std::sin(a), q = 0.5;
    double Fx = 0, Fy = 0;
    for (int k = 0; k < nw; k++) {
        const int f = c->g.wall_faces[w0 + k];
        const double fx = fw[4 * k + 1], fy = fw[4 * k + 2], S = c->g.flen[f];
        Fx += fx;
        Fy += fy;
        double nx = c->g.fnx[f], ny = c->g.fny[f], tx = -ny, ty = nx;
        if (tx * ca + ty * sa < 0) { tx = -tx; ty = -ty; }
        if (cp) cp[k] = ((fx * nx + fy * ny) / S - m.ip.p_inf) / q;
        if (cf) cf[k] = ((fx * tx + fy * ty) / S) / q;
        if (xw) xw[k] = c->g.fxm[f];
    }
    if (cd) *cd = (Fx * ca + Fy * sa) / q;
    if (cl) *cl = (-Fx * sa + Fy * ca) / q;
    return IGKS_OK;
}

int igks_get_wall_loads(igks_ctx *c, double *cl, double *cd, double *cf, double *cp, double *xw)
{
    return igks_batch_get_wall_loads(c, 0, cl, cd, cf, cp, xw);
}

int igks_set_profiling(igks_ctx *c, int on)
{
    if (!c) return IGKS_EINVAL;
    c->profiling = on != 0;
    return IGKS_OK;
}

int igks_time_kernel(igks_ctx *c, int32_t klass, int32_t reps, double *ms)
{
    if (!c || !ms || klass < 0 || klass > 2 || reps < 1 || reps > 10000) return IGKS_EINVAL;
    int rc = check_ready(c, true);
    if (rc) return rc;
    for (size_t i = 0; i < c->inst.size(); i++)
        if (c->hs[i].halt) return fail(c, IGKS_ENONPHYS, "instance " + std::to_string(i) + " is frozen");
    return (c->opt.precision == IGKS_MIXED) ? time_class(c, c->P32, klass, reps, ms)
                                            : time_class(c, c->P64, klass, reps, ms);
}

int igks_get_kernel_times(igks_ctx *c, double *ms6)
{
    if (!c || !ms6) return IGKS_EINVAL;
    for (int k = 0; k < NKT; k++) ms6[k] = c->ktimes[k];
    return IGKS_OK;
}

int igks_get_schedule(const igks_ctx *c, int32_t *s6)
{
    if (!c || !s6) return IGKS_EINVAL;
    for (int k = 0; k < NCLASS; k++) s6[k] = c->block[k];
    s6[NCLASS] = c->sweep_mode;
    s6[NCLASS + 1] = c->flux_pair ? 2 : 1;
    return IGKS_OK;
}

int igks_set_schedule(igks_ctx *c, const int32_t *s6)
{
    int rc = check_ready(c, false);
    if (rc) return rc;
    if (!s6) return fail(c, IGKS_EINVAL, "null schedule");
    for (int k = 0; k < NCLASS; k++)
        if (s6[k] != 64 && s6[k] != 128 && s6[k] != 256)
            return fail(c, IGKS_EINVAL, "block sizes must be 64, 128 or 256");
    if (s6[NCLASS] < 1 || s6[NCLASS] > 3 || (s6[NCLASS + 1] != 1 && s6[NCLASS + 1] != 2))
        return fail(c, IGKS_EINVAL, "the sweep schedule must be 1, 2 or 3 and the lanes per face 1 or 2");
    if (two_block_passes(c) && s6[NCLASS] != 3)
        return fail(c, IGKS_EINVAL, "two block passes run on the wave-per-block sweep schedule (3)");
    destroy_graph(c);
    for (int k = 0; k < NCLASS; k++) c->block[k] = s6[k];
    c->sweep_mode = s6[NCLASS];
    c->flux_pair = s6[NCLASS + 1] == 2;
    return IGKS_OK;
}

int igks_graph_chunk(const igks_ctx *cc, int32_t *iters, int32_t *launches)
{
    igks_ctx *c = const_cast<igks_ctx *>(cc);
    if (!c) return IGKS_EINVAL;
    int rc = ensure_combined(c);
    if (rc) return rc;
    const int mode = c->bound ? c->sweep_mode : auto_sweep_mode(c);
    if (iters) *iters = graph_chunk_for(c, mode);
    if (launches) *launches = launches_per_iteration(c, mode);
    return IGKS_OK;
}

int igks_autotune(igks_ctx *c, int32_t iters, int32_t *s6)
{
    int rc = check_ready(c, true);
    if (rc) return rc;
    if (iters < 1 || iters > 1000) return fail(c, IGKS_EINVAL, "iters must be in 1..1000");
    for (size_t i = 0; i < c->inst.size(); i++)
        if (c->hs[i].halt) return fail(c, IGKS_ENONPHYS, "instance " + std::to_string(i) + " is frozen");
    destroy_graph(c);
    const bool prof = c->profiling;
    // the candidates run real iterations: keep both state buffers and the scalars
    const size_t N = c->g.N, ni = c->inst.size(), SB = 5 * N * sizeof(double);
    char *bk = c->ws + c->w.backup.off;
    HIPCHK(c, hipMemcpyAsync(bk, c->P64.Wa, SB, hipMemcpyDeviceToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(bk + SB, c->P64.Wb, SB, hipMemcpyDeviceToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(bk + 2 * SB, c->P64.is, ni * sizeof(InstScalars), hipMemcpyDeviceToDevice, c->stream));
    std::vector<std::vector<double>> hist_keep = c->hist;
    // kernel class -> event interval: prep 0, flux 1, gather 2, sweep 4 + 5
    const int ev_of[NCLASS] = {0, 1, 2, 4};
    const int cand[3] = {64, 128, 256};
    int best[NCLASS];
    double best_t[NCLASS];
    for (int k = 0; k < NCLASS; k++) { best[k] = c->block[k]; best_t[k] = 1e300; }
    bool best_pair = c->flux_pair;
    const int mode_auto = c->sweep_mode;
    const bool pair_auto = c->flux_pair;
    for (int pair = 0; pair < 2 && !rc; pair++)
        for (int b : cand) {
            for (int k = 0; k < NCLASS; k++) c->block[k] = b;
            c->sweep_mode = 1;
            c->flux_pair = pair != 0;
            rc = (c->opt.precision == IGKS_MIXED) ? tune_run(c, c->P32, iters) : tune_run(c, c->P64, iters);
            if (rc) break;
            for (int k = 0; k < NCLASS; k++) {
                double tk = c->ktimes[ev_of[k]] + (k == 3 ? c->ktimes[5] : 0.0);
                if (tk < best_t[k]) {
                    best_t[k] = tk;
                    best[k] = b;
                    if (k == 1) best_pair = pair != 0;
                }
            }
        }
    for (int k = 0; k < NCLASS; k++) c->block[k] = best[k];
    c->flux_pair = rc ? pair_auto : best_pair;
    // sweeps: one launch per wavefront (timed above), one workgroup (a
    // candidate only while wavefronts are narrow), a wave per sweep block
    // (with sweep blocks)
    int best_mode = two_block_passes(c) ? 3 : 1;   // two passes run on the wave-per-block schedule only
    double best_sweep = best_t[3];
    for (int mode = 2; mode <= 3 && !rc && !two_block_passes(c); mode++) {
        if (mode == 2 && !((double)c->g.N / std::max(1, c->g.nlev) < 16384.0)) continue;
        if (mode == 3 && !any_sweep_blocks(c)) continue;
        c->sweep_mode = mode;
        rc = (c->opt.precision == IGKS_MIXED) ? tune_run(c, c->P32, iters) : tune_run(c, c->P64, iters);
        if (!rc && c->ktimes[4] + c->ktimes[5] < best_sweep) {
            best_sweep = c->ktimes[4] + c->ktimes[5];
            best_mode = mode;
        }
    }
    c->sweep_mode = rc ? mode_auto : best_mode;
    c->profiling = prof;
    HIPCHK(c, hipMemcpyAsync(c->P64.Wa, bk, SB, hipMemcpyDeviceToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(c->P64.Wb, bk + SB, SB, hipMemcpyDeviceToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(c->P64.is, bk + 2 * SB, ni * sizeof(InstScalars), hipMemcpyDeviceToDevice, c->stream));
    launch_reset(launch_of(c), c->P64, 1, -1);
    c->hist = hist_keep;
    for (double &x : c->ktimes) x = 0.0;
    int rc2 = sync_scalars(c);
    if (rc) return rc;
    if (rc2) return rc2;
    if (s6) igks_get_schedule(c, s6);
    return IGKS_OK;
}

}  // extern "C"
