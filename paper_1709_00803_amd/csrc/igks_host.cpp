// igks_host.cpp - host side of libigks: mesh ingest and preprocessing
// (Sec. 2.4 mesh data -> faces, geometry, ghost-cell offsets, sweep
// wavefronts), workspace layout, the iteration driver with HIP-graph
// chunks, and the C ABI declared in include/igks.h.
#include "../../include/igks.h"
#include "igks_dev.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>
#include <string>
#include <unordered_map>
#include <vector>

using namespace igks;

namespace {

struct HostMesh {
    int nn = 0, nc = 0, nf = 0, nwall = 0, nlev = 0;
    std::vector<int> perm;     // internal cell -> upload index
    std::vector<int> iperm;    // upload index -> internal cell
    std::vector<int> lev_off;  // wavefront offsets in internal order
    // cells (internal order)
    std::vector<double> xc, yc, area, lsinv, vtx;
    std::vector<int> cf_ptr, cf_face, cf_nbr, cf_flag;
    std::vector<double> cf_dx, cf_dy;
    // faces (internal order)
    std::vector<int> fl, fr, ftag;
    std::vector<double> fnx, fny, flen, frl, frr, fdl, fdr, frn, fxm, fym;
    std::vector<int> wall_faces;   // internal face ids in input order of the WALL edges
    std::vector<double> wseg;      // wall segments (ax, ay, bx, by)
};

struct Buf {
    size_t off, bytes;
};

}  // namespace

struct igks_ctx {
    igks_options opt{};
    hipStream_t stream = nullptr;
    bool own_stream = false;
    std::string err;
    HostMesh m;
    bool have_mesh = false;
    // workspace
    char *ws = nullptr;
    size_t ws_bytes = 0;
    bool bound = false;
    // device views
    Params<double> P64{};
    Params<float> P32{};
    int *d_wall_faces = nullptr;
    int *d_lev_off = nullptr;
    bool sweep_wg = false;
    double *d_wall_out = nullptr;
    double *d_wseg = nullptr;
    int max_blocks = 0;
    int hist_cap = 0;
    // flow
    bool have_flow = false;
    double mach = 0, alpha = 0, re = 0, nut_ratio = -1;
    // host copies of the device scalars and history
    DevScalars hs{};
    std::vector<double> hist;
    // graphs
    hipGraphExec_t gexec = nullptr;
    int gexec_n = 0;
    // profiling
    bool profiling = false;
    double ktimes[7] = {0, 0, 0, 0, 0, 0, 0};
};

namespace {

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

template <typename T>
std::vector<T> permute_cells(const std::vector<T> &src, int ncomp, const std::vector<int> &perm)
{
    size_t n = perm.size();
    std::vector<T> out(src.size());
    for (int k = 0; k < ncomp; k++)
        for (size_t i = 0; i < n; i++) out[k * n + i] = src[k * n + perm[i]];
    return out;
}

void destroy_graph(igks_ctx *c)
{
    if (c->gexec) {
        (void)hipGraphExecDestroy(c->gexec);
        c->gexec = nullptr;
        c->gexec_n = 0;
    }
}

// ------------------------------------------------------------------ ingest

int build_mesh(igks_ctx *ctx, int n_nodes, const double *xy, int n_cells, const int32_t *cell_ptr,
               const int32_t *cell_nodes, int n_bfaces, const int32_t *bface_nodes, const int32_t *bface_tag,
               HostMesh &m)
{
    if (n_nodes <= 0 || n_cells <= 0 || n_bfaces < 0 || !xy || !cell_ptr || !cell_nodes)
        return fail(ctx, IGKS_EINVAL, "empty mesh or null pointer");
    if (cell_ptr[0] != 0) return fail(ctx, IGKS_EMESH, "cell_ptr[0] must be 0");
    m = HostMesh();
    m.nn = n_nodes;
    m.nc = n_cells;
    const int N = n_cells;
    // cells: counter-clockwise vertex lists, area, centroid (relative to the
    // first vertex to limit cancellation)
    std::vector<int> cptr(cell_ptr, cell_ptr + N + 1), cn(cell_ptr[N]);
    for (int i = 0; i < N; i++) {
        int k = cptr[i + 1] - cptr[i];
        if (k < 3 || k > MAXV) return fail(ctx, IGKS_EMESH, "cell " + std::to_string(i) + " has " + std::to_string(k) + " nodes (3 or 4 supported)");
    }
    for (int p = 0; p < cell_ptr[N]; p++) {
        int v = cell_nodes[p];
        if (v < 0 || v >= n_nodes) return fail(ctx, IGKS_EMESH, "node index out of range");
        cn[p] = v;
    }
    std::vector<double> area(N), xc(N), yc(N);
    for (int i = 0; i < N; i++) {
        int p0 = cptr[i], k = cptr[i + 1] - p0;
        double x0 = xy[2 * cn[p0]], y0 = xy[2 * cn[p0] + 1];
        double a2 = 0, sx = 0, sy = 0;
        for (int j = 1; j + 1 < k; j++) {
            double ax = xy[2 * cn[p0 + j]] - x0, ay = xy[2 * cn[p0 + j] + 1] - y0;
            double bx = xy[2 * cn[p0 + j + 1]] - x0, by = xy[2 * cn[p0 + j + 1] + 1] - y0;
            double t = ax * by - ay * bx;
            a2 += t;
            sx += t * (ax + bx);
            sy += t * (ay + by);
        }
        if (a2 < 0) {
            std::reverse(cn.begin() + p0, cn.begin() + p0 + k);
            a2 = -a2; sx = -sx; sy = -sy;
        }
        if (!(a2 > 0)) return fail(ctx, IGKS_EMESH, "degenerate cell " + std::to_string(i));
        area[i] = 0.5 * a2;
        xc[i] = x0 + sx / (3.0 * a2);
        yc[i] = y0 + sy / (3.0 * a2);
    }
    // edges -> faces; owner = the lower upload index
    struct E { long long key; int cell, loc; };
    std::vector<E> ev(cell_ptr[N]);
    for (int i = 0; i < N; i++) {
        int p0 = cptr[i], k = cptr[i + 1] - p0;
        for (int j = 0; j < k; j++) {
            long long a = cn[p0 + j], b = cn[p0 + (j + 1) % k];
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
        if (t < 1 || t > 5) return fail(ctx, IGKS_EMESH, "bad boundary tag");
        if (!bmap.emplace(std::min(a, d) * (long long)(n_nodes + 1) + std::max(a, d), b).second)
            return fail(ctx, IGKS_EMESH, "duplicate boundary edge");
    }
    struct UF { int l, r, tag, bidx, a, b; };   // upload-order faces
    std::vector<UF> uf;
    uf.reserve(ev.size());
    std::vector<char> bused(n_bfaces, 0);
    for (size_t i = 0; i < ev.size();) {
        size_t j = i + 1;
        while (j < ev.size() && ev[j].key == ev[i].key) j++;
        if (j - i > 2) return fail(ctx, IGKS_EMESH, "edge shared by more than two cells");
        int ow = ev[i].cell, lo = ev[i].loc;
        int p0 = cptr[ow], k = cptr[ow + 1] - p0;
        UF f{ow, -1, 0, -1, cn[p0 + lo], cn[p0 + (lo + 1) % k]};
        if (j - i == 2) {
            f.r = ev[i + 1].cell;
        } else {
            auto it = bmap.find(ev[i].key);
            if (it == bmap.end()) return fail(ctx, IGKS_EMESH, "boundary edge without a tag");
            f.bidx = it->second;
            f.tag = bface_tag[it->second];
            bused[it->second] = 1;
        }
        uf.push_back(f);
        i = j;
    }
    for (int b = 0; b < n_bfaces; b++)
        if (!bused[b]) return fail(ctx, IGKS_EMESH, "tagged edge " + std::to_string(b) + " is not on the mesh boundary");
    // cell -> faces in upload order
    std::vector<std::vector<int>> cfaces(N);
    for (size_t q = 0; q < uf.size(); q++) {
        cfaces[uf[q].l].push_back((int)q);
        if (uf[q].r >= 0) cfaces[uf[q].r].push_back((int)q);
    }
    // sweep wavefronts: level(i) = 1 + max level of neighbours with a smaller index
    std::vector<int> level(N, 0);
    int nlev = 0;
    for (int i = 0; i < N; i++) {
        int lv = 0;
        for (int q : cfaces[i]) {
            int o = uf[q].l == i ? uf[q].r : uf[q].l;
            if (o >= 0 && o < i) lv = std::max(lv, level[o] + 1);
        }
        level[i] = lv;
        nlev = std::max(nlev, lv + 1);
    }
    m.nlev = nlev;
    m.perm.resize(N);
    std::iota(m.perm.begin(), m.perm.end(), 0);
    std::stable_sort(m.perm.begin(), m.perm.end(), [&](int a, int b) { return level[a] < level[b]; });
    m.iperm.resize(N);
    for (int i = 0; i < N; i++) m.iperm[m.perm[i]] = i;
    m.lev_off.assign(nlev + 1, 0);
    for (int i = 0; i < N; i++) m.lev_off[level[i] + 1]++;
    for (int l = 0; l < nlev; l++) m.lev_off[l + 1] += m.lev_off[l];
    // faces in internal order: interior faces by owner, then boundary faces by owner
    std::vector<int> forder(uf.size());
    std::iota(forder.begin(), forder.end(), 0);
    std::stable_sort(forder.begin(), forder.end(), [&](int a, int b) {
        bool ba = uf[a].r < 0, bb = uf[b].r < 0;
        if (ba != bb) return bb;   // interior first
        return m.iperm[uf[a].l] < m.iperm[uf[b].l];
    });
    const int F = (int)uf.size();
    m.nf = F;
    std::vector<int> fpos(F);
    for (int q = 0; q < F; q++) fpos[forder[q]] = q;
    m.fl.resize(F); m.fr.resize(F); m.ftag.resize(F);
    m.fnx.resize(F); m.fny.resize(F); m.flen.resize(F); m.frl.resize(2 * F); m.frr.resize(2 * F);
    m.fdl.resize(F); m.fdr.resize(F); m.frn.resize(F); m.fxm.resize(F); m.fym.resize(F);
    for (int q = 0; q < F; q++) {
        const UF &u = uf[forder[q]];
        double ax = xy[2 * u.a], ay = xy[2 * u.a + 1], bx = xy[2 * u.b], by = xy[2 * u.b + 1];
        double dx = bx - ax, dy = by - ay, L = std::sqrt(dx * dx + dy * dy);
        double nx = dy / L, ny = -dx / L;   // outward normal of the owner's CCW edge
        double xm = 0.5 * (ax + bx), ym = 0.5 * (ay + by);
        m.fl[q] = m.iperm[u.l];
        m.fr[q] = u.r >= 0 ? m.iperm[u.r] : -1;
        m.ftag[q] = u.tag;
        m.fnx[q] = nx; m.fny[q] = ny; m.flen[q] = L; m.fxm[q] = xm; m.fym[q] = ym;
        double rlx = xm - xc[u.l], rly = ym - yc[u.l];
        m.frl[2 * q] = rlx; m.frl[2 * q + 1] = rly;
        double dl = rlx * nx + rly * ny;
        m.fdl[q] = dl;
        if (u.r >= 0) {
            double rrx = xm - xc[u.r], rry = ym - yc[u.r];
            m.frr[2 * q] = rrx; m.frr[2 * q + 1] = rry;
            m.fdr[q] = -(rrx * nx + rry * ny);
            m.frn[q] = std::fabs((xc[u.r] - xc[u.l]) * nx + (yc[u.r] - yc[u.l]) * ny);
        } else {
            m.frr[2 * q] = m.frr[2 * q + 1] = 0.0;
            m.fdr[q] = dl;
            m.frn[q] = 2.0 * dl;
        }
    }
    // wall faces in input order
    {
        std::vector<int> slot(n_bfaces, -1);
        for (int q = 0; q < F; q++) {
            const UF &u = uf[forder[q]];
            if (u.tag == BC_WALL) slot[u.bidx] = q;
        }
        for (int b = 0; b < n_bfaces; b++)
            if (slot[b] >= 0) {
                int q = slot[b];
                const UF &u = uf[forder[q]];
                m.wall_faces.push_back(q);
                m.wseg.push_back(xy[2 * u.a]); m.wseg.push_back(xy[2 * u.a + 1]);
                m.wseg.push_back(xy[2 * u.b]); m.wseg.push_back(xy[2 * u.b + 1]);
            }
        m.nwall = (int)m.wall_faces.size();
    }
    // cells in internal order
    m.xc.resize(N); m.yc.resize(N); m.area.resize(N); m.lsinv.resize(3 * N); m.vtx.resize(2 * MAXV * N);
    m.cf_ptr.assign(N + 1, 0);
    for (int c = 0; c < N; c++) m.cf_ptr[c + 1] = m.cf_ptr[c] + (int)cfaces[m.perm[c]].size();
    int ne = m.cf_ptr[N];
    m.cf_face.resize(ne); m.cf_nbr.resize(ne); m.cf_flag.resize(ne); m.cf_dx.resize(ne); m.cf_dy.resize(ne);
    for (int c = 0; c < N; c++) {
        int u = m.perm[c];
        m.xc[c] = xc[u]; m.yc[c] = yc[u]; m.area[c] = area[u];
        double a11 = 0, a12 = 0, a22 = 0;
        int e = m.cf_ptr[c];
        for (int q : cfaces[u]) {
            const UF &f = uf[q];
            int qi = fpos[q];
            bool owner = f.l == u;
            int other = owner ? f.r : f.l;
            double dx, dy;
            if (other >= 0) {
                dx = xc[other] - xc[u];
                dy = yc[other] - yc[u];
            } else {   // ghost centroid: the cell centroid reflected in the face line
                double dn = m.fdl[qi];
                dx = 2.0 * dn * m.fnx[qi];
                dy = 2.0 * dn * m.fny[qi];
            }
            m.cf_face[e] = qi;
            m.cf_nbr[e] = other >= 0 ? m.iperm[other] : -1;
            m.cf_flag[e] = (owner ? CF_OWNER : 0) | ((other >= 0 && other < u) ? CF_LOWER : 0);
            m.cf_dx[e] = dx;
            m.cf_dy[e] = dy;
            a11 += dx * dx; a12 += dx * dy; a22 += dy * dy;
            e++;
        }
        double det = a11 * a22 - a12 * a12;
        if (!(det > 0)) return fail(ctx, IGKS_EMESH, "singular least-squares stencil at cell " + std::to_string(u));
        m.lsinv[c] = a22 / det;
        m.lsinv[N + c] = -a12 / det;
        m.lsinv[2 * N + c] = a11 / det;
        int p0 = cptr[u], k = cptr[u + 1] - p0;
        for (int v = 0; v < MAXV; v++) {
            int node = cn[p0 + (v < k ? v : 0)];
            m.vtx[(2 * v) * N + c] = xy[2 * node] - xc[u];
            m.vtx[(2 * v + 1) * N + c] = xy[2 * node + 1] - yc[u];
        }
    }
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

struct WsMap {
    Buf sc, Wa, Wb, grad, lamc, vort, nu, M, lsum, sadiag, dW, xc, yc, area, lsinv, dwall, vtx;
    Buf cf_ptr, cf_face, cf_nbr, cf_flag, cf_dx, cf_dy;
    Buf fl, fr, fbc, fnx, fny, flen, frl, frr, fdl, fdr, frn, flux, lam, saf, sag, part, hist;
    Buf wall_faces, wall_out, wseg, lev_off;
    size_t total;
};

WsMap layout(const HostMesh &m, const igks_options &o, int max_blocks, int hist_cap)
{
    Layout L;
    WsMap w;
    const size_t N = m.nc, F = m.nf, E = m.cf_ptr.empty() ? 0 : (size_t)m.cf_ptr.back(), D = sizeof(double),
                 I = sizeof(int);
    w.sc = L.add(sizeof(DevScalars));
    w.Wa = L.add(5 * N * D); w.Wb = L.add(5 * N * D);
    w.grad = L.add(8 * N * D); w.lamc = L.add(N * D); w.vort = L.add(N * D); w.nu = L.add(N * D);
    w.M = L.add(5 * N * D); w.lsum = L.add(N * D); w.sadiag = L.add(N * D);
    w.dW = L.add(5 * N * (o.precision == IGKS_MIXED ? sizeof(float) : D));
    w.xc = L.add(N * D); w.yc = L.add(N * D); w.area = L.add(N * D); w.lsinv = L.add(3 * N * D);
    w.dwall = L.add(N * D); w.vtx = L.add(2 * MAXV * N * D);
    w.cf_ptr = L.add((N + 1) * I); w.cf_face = L.add(E * I); w.cf_nbr = L.add(E * I); w.cf_flag = L.add(E * I);
    w.cf_dx = L.add(E * D); w.cf_dy = L.add(E * D);
    w.fl = L.add(F * I); w.fr = L.add(F * I); w.fbc = L.add(F * I);
    w.fnx = L.add(F * D); w.fny = L.add(F * D); w.flen = L.add(F * D); w.frl = L.add(2 * F * D);
    w.frr = L.add(2 * F * D); w.fdl = L.add(F * D); w.fdr = L.add(F * D); w.frn = L.add(F * D);
    w.flux = L.add(4 * F * D); w.lam = L.add(F * D); w.saf = L.add(F * D); w.sag = L.add(F * D);
    w.part = L.add(2 * (size_t)max_blocks * D);
    w.hist = L.add((size_t)HIST_W * hist_cap * D);
    w.wall_faces = L.add((size_t)std::max(1, m.nwall) * I);
    w.wall_out = L.add((size_t)4 * std::max(1, m.nwall) * D);
    w.wseg = L.add((size_t)4 * std::max(1, m.nwall) * D);
    w.lev_off = L.add((size_t)(m.nlev + 1) * I);
    w.total = L.total;
    return w;
}

int hist_cap_of(const igks_options &o) { return std::max(1, o.chunk > 0 ? o.chunk : 64); }

template <typename T>
void fill_params(igks_ctx *c, Params<T> &P, const WsMap &w)
{
    char *b = c->ws;
    auto D = [&](const Buf &x) { return (double *)(b + x.off); };
    auto In = [&](const Buf &x) { return (int *)(b + x.off); };
    P = Params<T>{};
    P.nc = c->m.nc; P.nf = c->m.nf;
    P.limiter = c->opt.limiter; P.visc_sr = c->opt.visc_sr; P.mu_law = c->opt.mu_law; P.cfl_mode = c->opt.cfl_mode;
    P.cfl_init = c->opt.cfl_init; P.cfl_min = c->opt.cfl_min; P.cfl_max = c->opt.cfl_max; P.cfl_flux = c->opt.cfl_flux;
    P.Wa = D(w.Wa); P.Wb = D(w.Wb); P.grad = D(w.grad); P.lamc = D(w.lamc); P.vort = D(w.vort); P.nu = D(w.nu);
    P.M = D(w.M); P.lsum = D(w.lsum); P.sadiag = D(w.sadiag); P.dW = (T *)(b + w.dW.off);
    P.xc = D(w.xc); P.yc = D(w.yc); P.area = D(w.area); P.lsinv = D(w.lsinv); P.dwall = D(w.dwall); P.vtx = D(w.vtx);
    P.cf_ptr = In(w.cf_ptr); P.cf_face = In(w.cf_face); P.cf_nbr = In(w.cf_nbr); P.cf_flag = In(w.cf_flag);
    P.cf_dx = D(w.cf_dx); P.cf_dy = D(w.cf_dy);
    P.fl = In(w.fl); P.fr = In(w.fr); P.fbc = In(w.fbc);
    P.fnx = D(w.fnx); P.fny = D(w.fny); P.flen = D(w.flen); P.frl = D(w.frl); P.frr = D(w.frr);
    P.fdl = D(w.fdl); P.fdr = D(w.fdr); P.frn = D(w.frn);
    P.flux = D(w.flux); P.lam = D(w.lam); P.saf = D(w.saf); P.sag = D(w.sag);
    P.part = D(w.part); P.max_blocks = c->max_blocks;
    P.hist = D(w.hist); P.hist_cap = c->hist_cap;
    P.sc = (DevScalars *)(b + w.sc.off);
}

template <typename T>
void set_flow_params(igks_ctx *c, Params<T> &P)
{
    const double g = GAMMA;
    double pinf = 1.0 / (g * c->mach * c->mach);
    P.p_inf = pinf;
    P.lam_inf = 1.0 / (2.0 * pinf);
    P.mu_inf = 1.0 / c->re;
    P.sa = c->nut_ratio >= 0.0;
    double a = c->alpha * M_PI / 180.0;
    P.Winf[0] = 1.0; P.Winf[1] = std::cos(a); P.Winf[2] = std::sin(a);
    P.Winf[3] = pinf / (g - 1.0) + 0.5;
    P.Winf[4] = P.sa ? c->nut_ratio * P.mu_inf : 0.0;
}

Launch launch_of(igks_ctx *c) { return Launch{c->stream, c->opt.block > 0 ? c->opt.block : 256}; }

// queue one nonlinear iteration
template <typename T>
void queue_iteration(igks_ctx *c, const Params<T> &P, hipEvent_t *ev)
{
    Launch L = launch_of(c);
    auto mark = [&](int k) { if (ev) (void)hipEventRecord(ev[k], c->stream); };
    mark(0);
    launch_prep(L, P);
    mark(1);
    launch_flux(L, P);
    mark(2);
    launch_gather(L, P);
    mark(3);
    launch_reduce(L, P);
    mark(4);
    if (c->sweep_wg) launch_sweep_wg(L, P, c->d_lev_off, c->m.nlev, true);
    else
        for (int l = 0; l < c->m.nlev; l++) launch_sweep(L, P, c->m.lev_off[l], c->m.lev_off[l + 1], true);
    mark(5);
    if (c->sweep_wg) launch_sweep_wg(L, P, c->d_lev_off, c->m.nlev, false);
    else
        for (int l = c->m.nlev - 1; l >= 0; l--) launch_sweep(L, P, c->m.lev_off[l], c->m.lev_off[l + 1], false);
    mark(6);
    launch_update(L, P);
    mark(7);
    launch_commit(L, P);
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
    HIPCHK(c, hipMemcpyAsync(&c->hs, c->P64.sc, sizeof(DevScalars), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return IGKS_OK;
}

template <typename T>
int run_chunk(igks_ctx *c, const Params<T> &P, int k)
{
    Launch L = launch_of(c);
    launch_reset(L, P, 4);
    if (c->profiling) {
        hipEvent_t ev[8];
        for (auto &e : ev) HIPCHK(c, hipEventCreate(&e));
        for (int i = 0; i < k; i++) {
            queue_iteration(c, P, ev);
            HIPCHK(c, hipEventSynchronize(ev[7]));
            for (int j = 0; j < 7; j++) {
                float ms = 0;
                (void)hipEventElapsedTime(&ms, ev[j], ev[j + 1]);
                c->ktimes[j] += ms;
            }
        }
        for (auto &e : ev) (void)hipEventDestroy(e);
    } else if (c->opt.chunk > 0 && k == c->opt.chunk) {
        if (!c->gexec) {
            hipGraph_t g;
            HIPCHK(c, hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
            for (int i = 0; i < k; i++) queue_iteration(c, P, nullptr);
            HIPCHK(c, hipStreamEndCapture(c->stream, &g));
            hipError_t e = hipGraphInstantiate(&c->gexec, g, nullptr, nullptr, 0);
            (void)hipGraphDestroy(g);
            if (e != hipSuccess) return fail(c, IGKS_EHIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
            c->gexec_n = k;
        }
        HIPCHK(c, hipGraphLaunch(c->gexec, c->stream));
    } else {
        for (int i = 0; i < k; i++) queue_iteration(c, P, nullptr);
    }
    HIPCHK(c, hipGetLastError());
    int rc = sync_scalars(c);
    if (rc) return rc;
    int nh = std::min(c->hs.hist_n, c->hist_cap);
    if (nh > 0) {
        size_t old = c->hist.size();
        c->hist.resize(old + (size_t)HIST_W * nh);
        HIPCHK(c, hipMemcpy(c->hist.data() + old, P.hist, sizeof(double) * HIST_W * nh, hipMemcpyDeviceToHost));
    }
    return IGKS_OK;
}

int check_ready(igks_ctx *c, bool need_flow)
{
    if (!c) return IGKS_EINVAL;
    if (!c->have_mesh) return fail(c, IGKS_EINVAL, "no mesh uploaded");
    if (!c->bound) return fail(c, IGKS_EINVAL, "no workspace bound");
    if (need_flow && !c->have_flow) return fail(c, IGKS_EINVAL, "set_freestream first");
    return IGKS_OK;
}

double *cur_buffer(igks_ctx *c) { return (c->hs.ncommit & 1) ? c->P64.Wb : c->P64.Wa; }

}  // namespace

// ====================================================================== C ABI

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
}

int igks_create(igks_ctx **out, const igks_options *opt, void *hip_stream)
{
    if (!out) return IGKS_EINVAL;
    *out = nullptr;
    igks_ctx *c = new (std::nothrow) igks_ctx();
    if (!c) return IGKS_ENOMEM;
    if (opt) c->opt = *opt; else igks_default_options(&c->opt);
    if (c->opt.precision != IGKS_FP64 && c->opt.precision != IGKS_MIXED) { delete c; return IGKS_EINVAL; }
    if (c->opt.block <= 0) c->opt.block = 256;
    if (c->opt.block % 64 != 0 || c->opt.block > 1024) { delete c; return IGKS_EINVAL; }
    if (c->opt.sweep < 0 || c->opt.sweep > 2) { delete c; return IGKS_EINVAL; }
    if (hip_stream) {
        c->stream = (hipStream_t)hip_stream;
    } else {
        if (hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking) != hipSuccess) { delete c; return IGKS_EHIP; }
        c->own_stream = true;
    }
    *out = c;
    return IGKS_OK;
}

void igks_destroy(igks_ctx *c)
{
    if (!c) return;
    destroy_graph(c);
    if (c->own_stream && c->stream) (void)hipStreamDestroy(c->stream);
    delete c;
}

const char *igks_last_error(const igks_ctx *c) { return c ? c->err.c_str() : "null context"; }

int igks_mesh_upload(igks_ctx *c, int32_t n_nodes, const double *xy, int32_t n_cells, const int32_t *cell_ptr,
                     const int32_t *cell_nodes, int32_t n_bfaces, const int32_t *bface_nodes,
                     const int32_t *bface_tag)
{
    if (!c) return IGKS_EINVAL;
    destroy_graph(c);
    c->have_mesh = c->bound = c->have_flow = false;
    HostMesh m;
    int rc = build_mesh(c, n_nodes, xy, n_cells, cell_ptr, cell_nodes, n_bfaces, bface_nodes, bface_tag, m);
    if (rc) return rc;
    c->m = std::move(m);
    c->max_blocks = (c->m.nc + 255) / 256;
    c->hist_cap = hist_cap_of(c->opt);
    c->have_mesh = true;
    return IGKS_OK;
}

int igks_mesh_info(const igks_ctx *c, int32_t *nc, int32_t *nf, int32_t *nw, int32_t *nl)
{
    if (!c || !c->have_mesh) return IGKS_EINVAL;
    if (nc) *nc = c->m.nc;
    if (nf) *nf = c->m.nf;
    if (nw) *nw = c->m.nwall;
    if (nl) *nl = c->m.nlev;
    return IGKS_OK;
}

int igks_workspace_size(const igks_ctx *c, size_t *bytes)
{
    if (!c || !bytes || !c->have_mesh) return IGKS_EINVAL;
    *bytes = layout(c->m, c->opt, c->max_blocks, c->hist_cap).total;
    return IGKS_OK;
}

int igks_bind_workspace(igks_ctx *c, void *dptr, size_t bytes)
{
    if (!c) return IGKS_EINVAL;
    if (!c->have_mesh) return fail(c, IGKS_EINVAL, "no mesh uploaded");
    WsMap w = layout(c->m, c->opt, c->max_blocks, c->hist_cap);
    if (!dptr || bytes < w.total) return fail(c, IGKS_ENOMEM, "workspace smaller than igks_workspace_size");
    if (((uintptr_t)dptr) % 256 != 0) return fail(c, IGKS_EINVAL, "workspace must be 256-byte aligned");
    destroy_graph(c);
    c->ws = (char *)dptr;
    c->ws_bytes = bytes;
    fill_params(c, c->P64, w);
    fill_params(c, c->P32, w);
    const HostMesh &m = c->m;
    char *b = c->ws;
    auto up = [&](const Buf &x, const void *src, size_t n) -> int {
        if (n == 0) return IGKS_OK;
        HIPCHK(c, hipMemcpyAsync(b + x.off, src, n, hipMemcpyHostToDevice, c->stream));
        return IGKS_OK;
    };
    const size_t D = sizeof(double), I = sizeof(int), N = m.nc, F = m.nf, E = m.cf_ptr.back();
    int rc = 0;
    rc |= up(w.xc, m.xc.data(), N * D); rc |= up(w.yc, m.yc.data(), N * D); rc |= up(w.area, m.area.data(), N * D);
    rc |= up(w.lsinv, m.lsinv.data(), 3 * N * D); rc |= up(w.vtx, m.vtx.data(), 2 * MAXV * N * D);
    rc |= up(w.cf_ptr, m.cf_ptr.data(), (N + 1) * I); rc |= up(w.cf_face, m.cf_face.data(), E * I);
    rc |= up(w.cf_nbr, m.cf_nbr.data(), E * I); rc |= up(w.cf_flag, m.cf_flag.data(), E * I);
    rc |= up(w.cf_dx, m.cf_dx.data(), E * D); rc |= up(w.cf_dy, m.cf_dy.data(), E * D);
    rc |= up(w.fl, m.fl.data(), F * I); rc |= up(w.fr, m.fr.data(), F * I); rc |= up(w.fbc, m.ftag.data(), F * I);
    rc |= up(w.fnx, m.fnx.data(), F * D); rc |= up(w.fny, m.fny.data(), F * D); rc |= up(w.flen, m.flen.data(), F * D);
    rc |= up(w.frl, m.frl.data(), 2 * F * D); rc |= up(w.frr, m.frr.data(), 2 * F * D);
    rc |= up(w.fdl, m.fdl.data(), F * D); rc |= up(w.fdr, m.fdr.data(), F * D); rc |= up(w.frn, m.frn.data(), F * D);
    rc |= up(w.wall_faces, m.wall_faces.data(), m.wall_faces.size() * I);
    rc |= up(w.wseg, m.wseg.data(), m.wseg.size() * D);
    rc |= up(w.lev_off, m.lev_off.data(), m.lev_off.size() * I);
    if (rc) return rc;
    c->d_lev_off = (int *)(b + w.lev_off.off);
    {
        double width = (double)m.nc / std::max(1, m.nlev);
        c->sweep_wg = c->opt.sweep == 2 || (c->opt.sweep == 0 && m.nlev > 16 && width < 4096.0);
    }
    c->d_wall_faces = (int *)(b + w.wall_faces.off);
    c->d_wall_out = (double *)(b + w.wall_out.off);
    c->d_wseg = (double *)(b + w.wseg.off);
    Launch L = launch_of(c);
    launch_wall_distance(L, m.nc, c->P64.xc, c->P64.yc, m.nwall, c->d_wseg, (double *)c->P64.dwall);
    HIPCHK(c, hipGetLastError());
    HIPCHK(c, hipMemsetAsync(c->P64.sc, 0, sizeof(DevScalars), c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    c->bound = true;
    c->have_flow = false;
    return IGKS_OK;
}

int igks_set_freestream(igks_ctx *c, double mach, double alpha_deg, double reynolds, double nut_ratio)
{
    int rc = check_ready(c, false);
    if (rc) return rc;
    if (!(mach > 0) || !(reynolds > 0)) return fail(c, IGKS_EINVAL, "mach and reynolds must be positive");
    destroy_graph(c);
    c->mach = mach; c->alpha = alpha_deg; c->re = reynolds; c->nut_ratio = nut_ratio;
    set_flow_params(c, c->P64);
    set_flow_params(c, c->P32);
    // FARFIELD faces: free stream where V_inf . n < 0, else Riemann outflow
    std::vector<int> fbc(c->m.ftag);
    for (int q = 0; q < c->m.nf; q++)
        if (fbc[q] == BC_FARFIELD)
            fbc[q] = (c->P64.Winf[1] * c->m.fnx[q] + c->P64.Winf[2] * c->m.fny[q] < 0.0) ? BC_FREESTREAM : BC_OUTFLOW;
    HIPCHK(c, hipMemcpyAsync((void *)c->P64.fbc, fbc.data(), sizeof(int) * c->m.nf, hipMemcpyHostToDevice, c->stream));
    Launch L = launch_of(c);
    launch_set_state(L, c->m.nc, c->P64.Winf, c->P64.Wa);
    HIPCHK(c, hipMemsetAsync(c->P64.sc, 0, sizeof(DevScalars), c->stream));
    launch_reset(L, c->P64, 7);
    HIPCHK(c, hipGetLastError());
    c->have_flow = true;
    c->hist.clear();
    return sync_scalars(c);
}

int igks_iterate(igks_ctx *c, int32_t n, int32_t *n_done)
{
    if (n_done) *n_done = 0;
    int rc = check_ready(c, true);
    if (rc) return rc;
    if (n < 0) return fail(c, IGKS_EINVAL, "negative iteration count");
    c->hist.clear();
    for (double &t : c->ktimes) t = 0.0;
    int start = c->hs.ncommit, done = 0;
    Launch L = launch_of(c);
    // clear flags a previous rejected update may have left
    launch_reset(L, c->P64, 3);
    while (done < n) {
        int k = c->opt.chunk > 0 ? std::min(c->opt.chunk, n - done) : n - done;
        if (c->profiling) k = std::min(k, 64);
        rc = (c->opt.precision == IGKS_MIXED) ? run_chunk(c, c->P32, k) : run_chunk(c, c->P64, k);
        if (rc) return rc;
        done = c->hs.ncommit - start;
        if (n_done) *n_done = done;
        if (c->hs.halt) {
            launch_reset(L, c->P64, 3);
            return fail(c, IGKS_ENONPHYS, "non-physical state (rho <= 0, p <= 0 or non-finite); last good state kept");
        }
    }
    if (c->profiling && n > 0)
        for (double &t : c->ktimes) t /= n;
    return IGKS_OK;
}

int igks_get_residual(igks_ctx *c, igks_residual *out)
{
    int rc = check_ready(c, true);
    if (rc) return rc;
    if (!out) return IGKS_EINVAL;
    out->iteration = c->hs.ncommit;
    out->res_l2 = c->hs.res_l2;
    out->res_drop = c->hs.res0 > 0 ? c->hs.res_l2 / c->hs.res0 : 0.0;
    out->res_inf = c->hs.res_inf;
    out->eq40 = c->hs.e40;
    out->cfl = c->hs.cfl;
    out->dt_flux = c->hs.dt_flux;
    out->sa_l2 = c->hs.sa_l2;
    return IGKS_OK;
}

int igks_get_history(igks_ctx *c, double *out, int32_t max, int32_t *n_out)
{
    if (!c) return IGKS_EINVAL;
    int n = (int)(c->hist.size() / HIST_W);
    n = std::min(n, (int)max);
    if (out && n > 0) std::memcpy(out, c->hist.data(), sizeof(double) * HIST_W * n);
    if (n_out) *n_out = n;
    return IGKS_OK;
}

int igks_get_state(igks_ctx *c, double *W)
{
    int rc = check_ready(c, true);
    if (rc) return rc;
    if (!W) return IGKS_EINVAL;
    const int N = c->m.nc;
    std::vector<double> tmp(5 * (size_t)N);
    HIPCHK(c, hipMemcpyAsync(tmp.data(), cur_buffer(c), sizeof(double) * 5 * N, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    for (int k = 0; k < 5; k++)
        for (int i = 0; i < N; i++) W[(size_t)k * N + c->m.perm[i]] = tmp[(size_t)k * N + i];
    return IGKS_OK;
}

int igks_set_state(igks_ctx *c, const double *W, const igks_scalars *sc)
{
    int rc = check_ready(c, true);
    if (rc) return rc;
    if (!W) return IGKS_EINVAL;
    const int N = c->m.nc;
    for (int i = 0; i < N; i++) {
        double r = W[i], mx = W[N + i], my = W[2 * N + i], E = W[3 * N + i], t = W[4 * N + i];
        double p = E - 0.5 * (mx * mx + my * my) / r;
        if (!(r > 0) || !(p > 0) || !std::isfinite(t) || !std::isfinite(p))
            return fail(c, IGKS_ENONPHYS, "non-physical state at cell " + std::to_string(i));
    }
    std::vector<double> tmp(5 * (size_t)N);
    for (int k = 0; k < 5; k++)
        for (int i = 0; i < N; i++) tmp[(size_t)k * N + i] = W[(size_t)k * N + c->m.perm[i]];
    DevScalars s{};
    if (sc) {
        s.ncommit = sc->iteration;
        s.cfl = sc->cfl;
        s.res_inf_prev = sc->res_inf_prev;
        s.res0 = sc->res0;
    }
    for (int i = 0; i < NSLOT; i++) s.dtmin_bits[i] = 0x7ff0000000000000ull;
    double *dst = (s.ncommit & 1) ? c->P64.Wb : c->P64.Wa;
    HIPCHK(c, hipMemcpyAsync(dst, tmp.data(), sizeof(double) * 5 * N, hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(c->P64.sc, &s, sizeof(DevScalars), hipMemcpyHostToDevice, c->stream));
    c->hist.clear();
    return sync_scalars(c);
}

int igks_get_scalars(igks_ctx *c, igks_scalars *out)
{
    int rc = check_ready(c, true);
    if (rc) return rc;
    if (!out) return IGKS_EINVAL;
    out->iteration = c->hs.ncommit;
    out->cfl = c->hs.cfl;
    out->res_inf_prev = c->hs.res_inf_prev;
    out->res0 = c->hs.res0;
    return IGKS_OK;
}

int igks_compute_residual(igks_ctx *c, double *M)
{
    int rc = check_ready(c, true);
    if (rc) return rc;
    Launch L = launch_of(c);
    launch_reset(L, c->P64, 3);
    queue_residual(c, c->P64);
    launch_reset(L, c->P64, 1);
    HIPCHK(c, hipGetLastError());
    const int N = c->m.nc;
    std::vector<double> tmp(5 * (size_t)N);
    HIPCHK(c, hipMemcpyAsync(tmp.data(), c->P64.M, sizeof(double) * 5 * N, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    if (M)
        for (int k = 0; k < 5; k++)
            for (int i = 0; i < N; i++) M[(size_t)k * N + c->m.perm[i]] = tmp[(size_t)k * N + i];
    return IGKS_OK;
}

int igks_get_wall_loads(igks_ctx *c, double *cl, double *cd, double *cf, double *cp, double *xw)
{
    int rc = check_ready(c, true);
    if (rc) return rc;
    Launch L = launch_of(c);
    launch_reset(L, c->P64, 3);
    queue_residual(c, c->P64);
    launch_reset(L, c->P64, 1);
    const int nw = c->m.nwall;
    launch_gather_faces(L, nw, c->d_wall_faces, c->P64.flux, c->m.nf, c->d_wall_out);
    HIPCHK(c, hipGetLastError());
    std::vector<double> fw(4 * (size_t)std::max(nw, 1));
    if (nw > 0) HIPCHK(c, hipMemcpyAsync(fw.data(), c->d_wall_out, sizeof(double) * 4 * nw, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    double a = c->alpha * M_PI / 180.0, ca = std::cos(a), sa = std::sin(a), q = 0.5;
    double Fx = 0, Fy = 0;
    for (int w = 0; w < nw; w++) {
        int f = c->m.wall_faces[w];
        double fx = fw[4 * w + 1], fy = fw[4 * w + 2], S = c->m.flen[f];
        Fx += fx;
        Fy += fy;
        double nx = c->m.fnx[f], ny = c->m.fny[f], tx = -ny, ty = nx;
        if (tx * ca + ty * sa < 0) { tx = -tx; ty = -ty; }
        if (cp) cp[w] = ((fx * nx + fy * ny) / S - c->P64.p_inf) / q;
        if (cf) cf[w] = ((fx * tx + fy * ty) / S) / q;
        if (xw) xw[w] = c->m.fxm[f];
    }
    if (cd) *cd = (Fx * ca + Fy * sa) / q;
    if (cl) *cl = (-Fx * sa + Fy * ca) / q;
    return IGKS_OK;
}

int igks_set_profiling(igks_ctx *c, int on)
{
    if (!c) return IGKS_EINVAL;
    c->profiling = on != 0;
    return IGKS_OK;
}

int igks_get_kernel_times(igks_ctx *c, double *ms7)
{
    if (!c || !ms7) return IGKS_EINVAL;
    for (int k = 0; k < 7; k++) ms7[k] = c->ktimes[k];
    return IGKS_OK;
}

}  // extern "C"
