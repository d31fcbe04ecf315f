// pibm.hip -- host runtime and C ABI of the gfx950 LBM-PIBM-DEM library.
//
// Per coupled step, all on the caller's stream:
//   K2 k_markers    Lagrangian points: interpolation, exchange, reactions
//   K3 k_bin        particles -> lattice tiles (count, scan, scatter)
//   K1 k_lbm        fused stream + spreading + buoyancy + forced BGK (f, g)
//   K4 k_cells      DEM cell list + Verlet lists
//   K5 k_dem x n    DEM sub-steps (+ thermosensitive update on the last)
// then the A/B lattices swap.  Nothing here allocates device memory: every
// buffer is carved from the caller's workspace.
#include "pibm_device.h"
#include "../../include/pibm.h"
#include "pibm_internal.h"

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <new>
#include <vector>

using namespace pibm;

namespace {

constexpr size_t ALIGN = 256;
size_t up(size_t v) { return (v + ALIGN - 1) / ALIGN * ALIGN; }

enum Region {
    R_FA, R_GA, R_FB, R_GB, R_PART0, R_PART1, R_REACT, R_TMPL, R_TMPL_START, R_TMPL_REXT, R_MK_START, R_MK,
    R_TP_START, R_TP_BOX, R_GP_START, R_GP_BASE,
    R_TCOUNT, R_TSTART, R_TFILL, R_TITEMS, R_TCOUNT1, R_TSTART1, R_TFILL1, R_TITEMS1, R_CCOUNT, R_CSTART, R_CFILL, R_CITEMS, R_NBR, R_NBRN, R_XREF,
    R_HID0, R_HXI0, R_HN0, R_HID1, R_HXI1, R_HN1, R_FEAT, R_TARG, R_AUX, R_XBF, R_YMLP, R_NORM, R_CNTR, R_ERR, R_COUNT
};

struct Template {
    double R;
    std::vector<double> off;       // 4 per marker: r_x, r_y, r_z, A
    std::vector<int> pbeg;         // patches: first marker of each (one more entry: the count)
    std::vector<double> pbox;      // 6 per patch: least r_x, r_y, r_z, then greatest
};

struct Plan {
    int dim, Q, QG;
    long long N, Ns;
    size_t ssize, tsize;           // storage and compute type sizes
    int ntx, nty, ntz, ntiles;
    int TX, TY, TZ;
    int ncx, ncy, ncz, ncells;
    double cwx, cwy, cwz, skin;
    int np;
    std::vector<Template> tmpls;
    std::vector<int> ptmpl;        // template of each particle
    std::vector<int> mk_start;     // np + 1
    std::vector<int> tp_start;     // ntmpl + 1: first patch of each template
    std::vector<double> tp_box;    // 6 per template patch
    std::vector<int> gp_start;     // ngp + 1: first marker of each particle patch
    std::vector<int> gp_base;      // np + 1: first particle patch of each particle
    long long nmk, ntmpl_mk;
    long long tile_cap;
    size_t off[R_COUNT + 1];
};

// c_sg^2 of the thermal lattice: D2Q5 1/3, D3Q7 1/4, the flow lattice 1/3
double derive_csg2(const pibm_params &p) { return p.dim == 2 || p.thermal_model == 1 ? 1.0 / 3.0 : 0.25; }

struct Derived {
    double tau_f, tau_g, gbeta, nu, alpha;
};

// Relaxation times: Eqs. (lbm2.6), (lbm2.7) when Ra > 0, else from nu and Gr.
Derived derive(const pibm_params &p)
{
    Derived d{};
    if (p.Ra > 0) {
        d.nu = std::sqrt(p.Pr) * p.Lc * p.uc / std::sqrt(p.Ra);
        d.alpha = p.Lc * p.uc / std::sqrt(p.Pr * p.Ra);
        d.gbeta = p.uc * p.uc / (p.Lc * (p.dT_ref > 0 ? p.dT_ref : 1.0));
    } else {
        d.nu = p.nu;
        d.alpha = p.Pr > 0 ? p.nu / p.Pr : 0.0;
        d.gbeta = p.Lc > 0 ? p.Gr * p.nu * p.nu / (p.Lc * p.Lc * p.Lc) : 0.0;
    }
    d.tau_f = 3.0 * d.nu + 0.5;
    d.tau_g = d.alpha / derive_csg2(p) + 0.5;
    if (p.tau_f > 0) { d.tau_f = p.tau_f; d.nu = (p.tau_f - 0.5) / 3.0; }
    if (p.tau_g > 0) { d.tau_g = p.tau_g; d.alpha = (p.tau_g - 0.5) * derive_csg2(p); }
    if (p.gbeta_set) d.gbeta = p.gbeta;
    return d;
}

// Lagrangian points on the body surface: a ring of round(pi D / s) points
// (2D) or a Fibonacci sphere of round(pi D^2 / s^2) points (3D); weights per
// pibm_markers.
// Patches of a template: its points grouped by the cell of their (y, z)
// offset, cells of one tile's extent (py x pz), each with the box of its
// offsets.  The points are reordered patch by patch.
void make_patches(Template &t, int dim, int py, int pz)
{
    const int n = (int)(t.off.size() / 4);
    std::vector<std::pair<long long, int>> key(n);
    for (int k = 0; k < n; ++k) {
        const long long ky = (long long)std::floor((t.off[4 * k + 1] + t.R) / py);
        const long long kz = dim == 3 ? (long long)std::floor((t.off[4 * k + 2] + t.R) / pz) : 0;
        key[k] = {kz * (1LL << 20) + ky, k};
    }
    std::sort(key.begin(), key.end());
    std::vector<double> off(t.off.size());
    t.pbeg.clear();
    t.pbox.clear();
    for (int k = 0; k < n; ++k) {
        std::copy(t.off.begin() + 4 * key[k].second, t.off.begin() + 4 * key[k].second + 4, off.begin() + 4 * k);
        if (k == 0 || key[k].first != key[k - 1].first) {
            t.pbeg.push_back(k);
            t.pbox.insert(t.pbox.end(), {1e300, 1e300, 1e300, -1e300, -1e300, -1e300});
        }
        double *b = &t.pbox[t.pbox.size() - 6];
        for (int d = 0; d < 3; ++d) {
            const double r = d < dim ? off[4 * k + d] : 0.0;
            b[d] = std::min(b[d], r);
            b[3 + d] = std::max(b[3 + d], r);
        }
    }
    t.pbeg.push_back(n);
    t.off.swap(off);
}

Template make_template(int dim, double R, int mode, double s)
{
    const double pi = 3.14159265358979323846;
    Template t;
    t.R = R;
    const double D = 2.0 * R;
    if (mode == PIBM_MARKERS_POINT) {
        t.off = {0.0, 0.0, 0.0, dim == 2 ? D : 0.25 * pi * D * D};
        return t;
    }
    int n = dim == 2 ? (int)std::lround(pi * D / s) : (int)std::lround(pi * D * D / (s * s));
    if (n < 1) n = 1;
    t.off.resize((size_t)4 * n);
    const double golden = pi * (3.0 - std::sqrt(5.0));
    for (int k = 0; k < n; ++k) {
        double *o = &t.off[(size_t)4 * k];
        if (dim == 2) {
            const double th = 2.0 * pi * k / n;
            o[0] = R * std::cos(th); o[1] = R * std::sin(th); o[2] = 0.0;
            o[3] = mode == PIBM_MARKERS_SURFACE ? pi * D / n : s;
        } else {
            const double z = 1.0 - (2.0 * k + 1.0) / n;
            const double rr = std::sqrt(1.0 - z * z);
            const double ph = k * golden;
            o[0] = R * rr * std::cos(ph); o[1] = R * rr * std::sin(ph); o[2] = R * z;
            o[3] = mode == PIBM_MARKERS_SURFACE ? pi * D * D / n : 0.25 * pi * s * s;
        }
    }
    return t;
}

int check_params(const pibm_params *p)
{
    if (!p) return PIBM_EINVAL;
    if (p->dim != 2 && p->dim != 3) return PIBM_EINVAL;
    if (p->nx < 1 || p->ny < 1 || p->nz < 1) return PIBM_EINVAL;
    if (p->dim == 2 && p->nz != 1) return PIBM_EINVAL;
    if ((long long)p->nx * p->ny * p->nz > (1LL << 31) - 1) return PIBM_EINVAL;
    if (p->storage < PIBM_STORE_F32 || p->storage > PIBM_STORE_BF16DEV) return PIBM_EINVAL;
    if (p->marker_mode < 0 || p->marker_mode > 2) return PIBM_EINVAL;
    if (p->n_sub < 1) return PIBM_EINVAL;
    if (p->interp_order != 0 && p->interp_order != 2 && p->interp_order != 4) return PIBM_EINVAL;
    if (p->lattice != 0 && p->lattice != 19 && p->lattice != 15) return PIBM_EINVAL;
    // D3Q15 is a 3D flow lattice, built for the FP32 and FP64 storage
    if (p->lattice == 15 && (p->dim != 3 || (p->storage != PIBM_STORE_F32 && p->storage != PIBM_STORE_F64)))
        return PIBM_EINVAL;
    // temperature on the flow lattice: FP32 and FP64 storage
    if (p->thermal_model != 0 && p->thermal_model != 1) return PIBM_EINVAL;
    if (p->thermal_model == 1 && p->storage != PIBM_STORE_F32 && p->storage != PIBM_STORE_F64) return PIBM_EINVAL;
    if (p->streams < 0 || p->streams > 2) return PIBM_EINVAL;
    const Derived d = derive(*p);
    if (!(d.tau_f > 0.5) || !(d.tau_g > 0.5)) return PIBM_EINVAL;
    if (!std::isfinite(d.gbeta)) return PIBM_EINVAL;
    return PIBM_OK;
}

int make_plan(const pibm_params *p, const pibm_particle *pt, int np, Plan &P)
{
    int st = check_params(p);
    if (st) return st;
    if (np < 0 || (np > 0 && !pt)) return PIBM_EINVAL;
    P.dim = p->dim;
    P.Q = p->dim == 2 ? 9 : (p->lattice == 15 ? 15 : 19);
    P.QG = p->thermal_model == 1 ? P.Q : (p->dim == 2 ? 5 : 7);
    P.N = (long long)p->nx * p->ny * p->nz;
    P.ssize = p->storage == PIBM_STORE_F64 ? 8 : (p->storage == PIBM_STORE_F32 ? 4 : 2);
    // Array stride: N rounded up to 256 bytes, plus 129 x 256 bytes.  A stride
    // that is a multiple of a large power of two (2^25 nodes at 256 x 256 x
    // 512) puts the same node of all 26 arrays on the same HBM channels; the
    // odd stagger spreads a node's loads over channels (3% faster lattice
    // update there).
    P.Ns = (P.N + 127) / 128 * 128 + 33024 / (long long)P.ssize;
    // the lattice kernel reaches both arrays of an opposite pair of
    // populations from the pair's first array with 32-bit byte offsets
    if ((double)(p->dim == 2 ? 3 : 2) * (double)P.Ns * (double)P.ssize >= 4294967296.0) return PIBM_EINVAL;
    P.tsize = p->storage == PIBM_STORE_F64 ? 8 : 4;
    P.TX = TILE_X;
    P.TY = p->dim == 3 ? Tile<3>::Y : Tile<2>::Y;
    P.TZ = p->dim == 3 ? Tile<3>::Z : Tile<2>::Z;
    P.ntx = (p->nx + P.TX - 1) / P.TX;
    P.nty = (p->ny + P.TY - 1) / P.TY;
    P.ntz = (p->nz + P.TZ - 1) / P.TZ;
    P.ntiles = P.ntx * P.nty * P.ntz;
    P.np = np;
    const double s = p->marker_spacing > 0 ? p->marker_spacing : 1.0;
    P.skin = p->skin > 0 ? p->skin : 1.0;
    double Rmax = 0.0;
    P.tmpls.clear();
    P.ptmpl.assign(np, 0);
    for (int i = 0; i < np; ++i) {
        const double R = pt[i].R;
        if (!(R > 0) || !std::isfinite(R)) return PIBM_EINVAL;
        Rmax = std::max(Rmax, R);
        int k = -1;
        for (size_t t = 0; t < P.tmpls.size(); ++t)
            if (P.tmpls[t].R == R) { k = (int)t; break; }
        if (k < 0) {
            P.tmpls.push_back(make_template(p->dim, R, p->marker_mode, s));
            make_patches(P.tmpls.back(), p->dim, P.TY, P.TZ);
            k = (int)P.tmpls.size() - 1;
        }
        P.ptmpl[i] = k;
    }
    // markers
    P.mk_start.assign(np + 1, 0);
    P.ntmpl_mk = 0;
    for (auto &t : P.tmpls) P.ntmpl_mk += (long long)t.off.size() / 4;
    long long nmk = 0;
    for (int i = 0; i < np; ++i) {
        nmk += (long long)(P.tmpls[P.ptmpl[i]].off.size() / 4);
        // the spreading queue packs a point index in 27 bits
        if (nmk >= (1LL << 27)) return PIBM_EINVAL;
        P.mk_start[i + 1] = (int)nmk;
    }
    P.nmk = nmk;
    // patches of templates and particles
    P.tp_start.assign(P.tmpls.size() + 1, 0);
    P.tp_box.clear();
    for (size_t t = 0; t < P.tmpls.size(); ++t) {
        P.tp_start[t + 1] = P.tp_start[t] + (int)P.tmpls[t].pbeg.size() - 1;
        P.tp_box.insert(P.tp_box.end(), P.tmpls[t].pbox.begin(), P.tmpls[t].pbox.end());
    }
    P.gp_base.assign(np + 1, 0);
    P.gp_start.clear();
    for (int i = 0; i < np; ++i) {
        const Template &t = P.tmpls[P.ptmpl[i]];
        const long long ng = (long long)P.gp_base[i] + (long long)t.pbeg.size() - 1;
        if (ng >= (1LL << 30)) return PIBM_EINVAL;
        P.gp_base[i + 1] = (int)ng;
        for (size_t k = 0; k + 1 < t.pbeg.size(); ++k) P.gp_start.push_back(P.mk_start[i] + t.pbeg[k]);
    }
    P.gp_start.push_back((int)P.nmk);
    // tile-list capacity: every tile a patch's footprint can reach.  The
    // footprint spans at most ceil(extent) + 4 nodes per axis; a wrapped span
    // on a periodic axis whose last tile is short can touch one tile more.
    const int nn[3] = {p->nx, p->ny, p->nz}, TT[3] = {P.TX, P.TY, P.TZ};
    P.tile_cap = 0;
    for (int i = 0; i < np; ++i) {
        const double re = p->marker_mode == PIBM_MARKERS_POINT ? 0.0 : pt[i].R;
        if ((int)std::ceil(2.0 * re) + 5 > (MAXT_AXIS - 1) * P.TY) return PIBM_EINVAL;
        const Template &t = P.tmpls[P.ptmpl[i]];
        for (size_t k = 0; k + 1 < t.pbeg.size(); ++k) {
            long long c = 1;
            for (int d = 0; d < p->dim; ++d) {
                const int span = (int)std::ceil(t.pbox[6 * k + 3 + d] - t.pbox[6 * k + d] + 1e-9) + 4;
                const int ntd = (nn[d] + TT[d] - 1) / TT[d];
                const int extra = p->periodic[d] && nn[d] % TT[d] != 0 ? 1 : 0;
                c *= std::min(ntd, (span - 1) / TT[d] + 2 + extra);
            }
            P.tile_cap += c;
        }
    }
    // DEM cells of width >= 2 Rmax + skin
    const double cs = std::max(2.0 * Rmax + P.skin, 1.0);
    P.ncx = std::max(1, (int)std::floor(p->nx / cs));
    P.ncy = std::max(1, (int)std::floor(p->ny / cs));
    P.ncz = p->dim == 3 ? std::max(1, (int)std::floor(p->nz / cs)) : 1;
    P.cwx = (double)p->nx / P.ncx;
    P.cwy = (double)p->ny / P.ncy;
    P.cwz = p->dim == 3 ? (double)p->nz / P.ncz : 1.0;
    P.ncells = P.ncx * P.ncy * P.ncz;
    // layout
    const long long npa = std::max(np, 1);
    size_t sz[R_COUNT];
    const size_t fbytes = (size_t)P.Q * P.Ns * P.ssize, gbytes = (size_t)P.QG * P.Ns * P.ssize;
    // an f copy also holds pibm_fields' output (rho, u, T: five compute-type
    // arrays) while it is idle, which is larger for 16-bit 2D storage
    const size_t fcopy = std::max<size_t>(fbytes, (size_t)5 * (size_t)P.Ns * P.tsize);
    sz[R_FA] = fcopy; sz[R_GA] = gbytes; sz[R_FB] = fcopy; sz[R_GB] = gbytes;
    sz[R_PART0] = sz[R_PART1] = npa * sizeof(DevParticle);
    sz[R_REACT] = npa * sizeof(DevReact);
    sz[R_TMPL] = std::max(P.ntmpl_mk, 1LL) * sizeof(double4);
    sz[R_TMPL_START] = (P.tmpls.size() + 1) * sizeof(int);
    sz[R_TMPL_REXT] = (P.tmpls.size() + 1) * sizeof(double);
    sz[R_MK_START] = (npa + 1) * sizeof(int);
    sz[R_TP_START] = P.tp_start.size() * sizeof(int);
    sz[R_TP_BOX] = std::max<size_t>(P.tp_box.size(), 6) * sizeof(double);
    sz[R_GP_START] = P.gp_start.size() * sizeof(int);
    sz[R_GP_BASE] = P.gp_base.size() * sizeof(int);
    sz[R_MK] = std::max(P.nmk, 1LL) * (p->storage == PIBM_STORE_F64 ? sizeof(MarkerRec<double>) : sizeof(MarkerRec<float>));
    sz[R_TCOUNT] = (size_t)P.ntiles * sizeof(int);
    sz[R_TSTART] = (size_t)(P.ntiles + 1) * sizeof(int);
    sz[R_TFILL] = (size_t)P.ntiles * sizeof(int);
    sz[R_TITEMS] = std::max(P.tile_cap, 1LL) * sizeof(int2);
    // a second set of tile lists: the two-stream step bins the next step into it
    sz[R_TCOUNT1] = sz[R_TCOUNT]; sz[R_TSTART1] = sz[R_TSTART]; sz[R_TFILL1] = sz[R_TFILL]; sz[R_TITEMS1] = sz[R_TITEMS];
    sz[R_CCOUNT] = (size_t)P.ncells * sizeof(int);
    sz[R_CSTART] = (size_t)(P.ncells + 1) * sizeof(int);
    sz[R_CFILL] = (size_t)P.ncells * sizeof(int);
    sz[R_CITEMS] = npa * sizeof(int);
    sz[R_NBR] = npa * MAXN * sizeof(int);
    sz[R_NBRN] = npa * sizeof(int);
    sz[R_XREF] = npa * 3 * sizeof(double);
    sz[R_HID0] = sz[R_HID1] = npa * MAXC * sizeof(int);
    sz[R_HXI0] = sz[R_HXI1] = npa * MAXC * 3 * sizeof(double);
    sz[R_HN0] = sz[R_HN1] = npa * sizeof(int);
    sz[R_FEAT] = npa * 16 * sizeof(float);
    sz[R_TARG] = npa * 4 * sizeof(float);
    sz[R_AUX] = npa * 4 * sizeof(float);
    sz[R_XBF] = npa * 16 * sizeof(uint16_t);
    sz[R_YMLP] = npa * 4 * sizeof(float);
    sz[R_NORM] = 80 * sizeof(float);          // 40 normalisation values, then 16 + 16 range bounds
    sz[R_CNTR] = 64;                               // [0] tile items, [1] cell items
    sz[R_ERR] = 64;
    size_t o = 0;
    for (int r = 0; r < R_COUNT; ++r) { P.off[r] = o; o += up(sz[r]); }
    P.off[R_COUNT] = o;
    return PIBM_OK;
}

int check_particles(const pibm_params *p, const pibm_particle *pt, int np)
{
    const int nn[3] = {p->nx, p->ny, p->nz};
    double Rmax = 0;
    for (int i = 0; i < np; ++i) {
        for (int d = 0; d < p->dim; ++d) {
            if (!std::isfinite(pt[i].x[d]) || !std::isfinite(pt[i].u[d])) return PIBM_EINVAL;
            if (!p->periodic[d] && (pt[i].x[d] - pt[i].R < -0.5 || pt[i].x[d] + pt[i].R > nn[d] - 0.5))
                return PIBM_EINVAL;
        }
        if (!(pt[i].rho_r > 0)) return PIBM_EINVAL;
        Rmax = std::max(Rmax, pt[i].R);
    }
    // overlap check on a uniform grid of cells >= 2 Rmax
    const double cs = std::max(2.0 * Rmax, 1.0);
    int nc[3] = {1, 1, 1};
    for (int d = 0; d < p->dim; ++d) nc[d] = std::max(1, (int)std::floor(nn[d] / cs));
    auto cell = [&](const double *x, int *c) {
        for (int d = 0; d < 3; ++d) {
            if (d >= p->dim) { c[d] = 0; continue; }
            double y = x[d] + 0.5;
            if (p->periodic[d]) { y = std::fmod(y, (double)nn[d]); if (y < 0) y += nn[d]; }
            int v = (int)std::floor(y / ((double)nn[d] / nc[d]));
            c[d] = std::min(std::max(v, 0), nc[d] - 1);
        }
    };
    std::vector<std::vector<int>> cells((size_t)nc[0] * nc[1] * nc[2]);
    for (int i = 0; i < np; ++i) {
        int c[3];
        cell(pt[i].x, c);
        cells[((size_t)c[2] * nc[1] + c[1]) * nc[0] + c[0]].push_back(i);
    }
    for (int i = 0; i < np; ++i) {
        int c[3];
        cell(pt[i].x, c);
        for (int dz = (p->dim == 3 ? -1 : 0); dz <= (p->dim == 3 ? 1 : 0); ++dz)
            for (int dy = -1; dy <= 1; ++dy)
                for (int dx = -1; dx <= 1; ++dx) {
                    int cc[3] = {c[0] + dx, c[1] + dy, c[2] + dz}, ok = 1;
                    for (int d = 0; d < 3; ++d) {
                        if (cc[d] < 0 || cc[d] >= nc[d]) {
                            if (d < p->dim && p->periodic[d]) cc[d] = (cc[d] + nc[d]) % nc[d];
                            else ok = 0;
                        }
                    }
                    if (!ok) continue;
                    for (int j : cells[((size_t)cc[2] * nc[1] + cc[1]) * nc[0] + cc[0]]) {
                        if (j <= i) continue;
                        double d2 = 0;
                        for (int d = 0; d < p->dim; ++d) {
                            double dd = pt[j].x[d] - pt[i].x[d];
                            if (p->periodic[d]) {
                                if (dd > 0.5 * nn[d]) dd -= nn[d];
                                else if (dd < -0.5 * nn[d]) dd += nn[d];
                            }
                            d2 += dd * dd;
                        }
                        const double lim = pt[i].R + pt[j].R - 1e-9;
                        if (d2 < lim * lim) return PIBM_EOVERLAP;
                    }
                }
    }
    return PIBM_OK;
}

}  // namespace

struct pibm_ctx {
    pibm_params p;
    Plan P;
    Derived d;
    hipStream_t stream;
    // Temperature the g deviations are stored from: T_ref, except with 16-bit
    // storage, where it is the middle of the temperatures the case sets at
    // the start (fluid, walls, particles), so that the stored (g - w T_s) / w
    // stay within half the temperature range and keep the finest spacing.
    double T_store = 0.0;
    // Second stream on the same device: binning runs beside the marker
    // kernel and the DEM sub-steps beside the lattice kernel.  Each step forks
    // from `stream` and joins back into it, so all work stays ordered with
    // respect to the caller's stream.
    bool two = false;              // the step uses the second stream
    hipStream_t side = nullptr;
    hipEvent_t ev_start = nullptr, ev_bin = nullptr, ev_mk = nullptr, ev_join = nullptr;
    char *ws;
    size_t ws_bytes;
    int cur;        // lattice copy holding the current state (0 = A, 1 = B)
    int pcur;       // particle buffer holding the current state
    int hcur;       // contact-history buffer holding the current state
    int cells_ok;   // the cell list was built from the current particle state
    int tcur = 0;   // tile-list set the lattice kernel reads (0: R_TCOUNT.., 1: R_TCOUNT1..)
    int tiles_next = 0;   // the other set holds the lists of the current particle state
    long long step;
    int sticky;
    int device_lost;
    pibm_mlp *closure = nullptr;   // learned closure in the one-point mode (not owned)
    bool closure_range = false;    // particles with features outside a range keep the point exchange
    // phase profiling: pairs of events recorded around each phase's launches
    unsigned prof_mask = 0;        // phases timed (bit 1 << PIBM_PHASE_*)
    std::vector<hipEvent_t> ev_free;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> ev_rec[PIBM_NPHASE];
    void *r(int reg) const { return ws + P.off[reg]; }
    ~pibm_ctx() {
        if (side) (void)hipStreamSynchronize(side);
        for (hipEvent_t e : {ev_start, ev_bin, ev_mk, ev_join})
            if (e) (void)hipEventDestroy(e);
        if (side) (void)hipStreamDestroy(side);
    }
};

namespace {

template <class T> LbmArgs<T> lbm_args(const pibm_ctx *c)
{
    LbmArgs<T> a{};
    a.nx = c->p.nx; a.ny = c->p.ny; a.nz = c->p.nz;
    for (int d = 0; d < 3; ++d) a.per[d] = c->p.periodic[d] ? 1 : 0;
    a.Ns = c->P.Ns;
    a.ntx = c->P.ntx; a.nty = c->P.nty; a.ntz = c->P.ntz; a.ntiles = c->P.ntiles;
    a.omf = 1.0 / c->d.tau_f;
    a.omg = 1.0 / c->d.tau_g;
    a.gf = 1.0 - 0.5 / c->d.tau_f;
    a.gg = 1.0 - 0.5 / c->d.tau_g;
    a.gbeta = c->d.gbeta;
    a.Tref = c->T_store;
    a.dTb = c->T_store - c->p.T_ref;
    for (int k = 0; k < 6; ++k) a.tw[k] = c->p.T_wall[k] - c->T_store;
    const int src = c->cur;
    a.fA = c->r(src ? R_FB : R_FA);
    a.gA = c->r(src ? R_GB : R_GA);
    a.fB = c->r(src ? R_FA : R_FB);
    a.gB = c->r(src ? R_GA : R_GB);
    a.tile_start = (const int *)c->r(c->tcur ? R_TSTART1 : R_TSTART);
    a.tile_count = (const int *)c->r(c->tcur ? R_TCOUNT1 : R_TCOUNT);
    a.tile_items = (const int2 *)c->r(c->tcur ? R_TITEMS1 : R_TITEMS);
    a.mk = (const MarkerRec<T> *)c->r(R_MK);
    a.err = (int *)c->r(R_ERR);
    a.macro = nullptr;
    a.step = (uint32_t)c->step;
    a.seed = mix32((uint32_t)c->step * 0xc2b2ae3du + 0x85ebca77u);
    return a;
}

// Cell lists of at most this many particles and cells are built by one
// workgroup in one launch instead of four launches.
constexpr int ONE_WG_PARTICLES = 256, ONE_WG_LISTS = 16384;

int hip_ok(pibm_ctx *c, hipError_t e)
{
    if (e == hipSuccess) return PIBM_OK;
    if (c) c->device_lost = 1;
    return PIBM_EDEVICE;
}

int build_cells(pibm_ctx *c, hipStream_t s);

template <int DIM, class SF>
int launch_markers(pibm_ctx *c, bool reactions)
{
    using T = typename SF::T;
    if (c->P.np == 0) return PIBM_OK;
    int st;
    if ((st = build_cells(c, c->stream))) return st;   // the order of the workgroups (the DEM reuses the list)
    MkArgs<T> m{};
    m.lb = lbm_args<T>(c);
    m.part = (const DevParticle *)c->r(c->pcur ? R_PART1 : R_PART0);
    m.tmpl = (const double4 *)c->r(R_TMPL);
    m.tmpl_start = (const int *)c->r(R_TMPL_START);
    m.tmpl_rext = (const double *)c->r(R_TMPL_REXT);
    m.mk_start = (const int *)c->r(R_MK_START);
    m.order = (const int *)c->r(R_CITEMS);
    m.mk = (MarkerRec<T> *)c->r(R_MK);
    m.react = reactions ? (DevReact *)c->r(R_REACT) : nullptr;
    m.kappa = c->p.kappa_T;
    m.Tref = c->T_store;
    if (c->p.interp_order == 4)
        hipLaunchKernelGGL((k_markers<DIM, SF, 4>), dim3(c->P.np), dim3(256), 0, c->stream, m);
    else
        hipLaunchKernelGGL((k_markers<DIM, SF, 2>), dim3(c->P.np), dim3(256), 0, c->stream, m);
    return hip_ok(c, hipGetLastError());
}

template <int DIM, class SF>
int launch_features(pibm_ctx *c, bool raw, bool for_network)
{
    using T = typename SF::T;
    if (c->P.np == 0) return PIBM_OK;
    int st;
    if ((st = build_cells(c, c->stream))) return st;
    FeatArgs<T> f{};
    f.lb = lbm_args<T>(c);
    f.ncx = c->P.ncx; f.ncy = c->P.ncy; f.ncz = c->P.ncz;
    f.cwx = c->P.cwx; f.cwy = c->P.cwy; f.cwz = c->P.cwz;
    f.cell_start = (const int *)c->r(R_CSTART);
    f.cell_count = (const int *)c->r(R_CCOUNT);
    f.cell_items = (const int *)c->r(R_CITEMS);
    f.part = (const DevParticle *)c->r(c->pcur ? R_PART1 : R_PART0);
    f.np = c->P.np;
    f.nu = c->d.nu;
    f.alpha = c->d.alpha;
    f.gbeta = c->d.gbeta;
    f.feat = raw ? (float *)c->r(R_FEAT) : nullptr;
    f.aux = (float *)c->r(R_AUX);
    f.xbf = for_network ? (uint16_t *)c->r(R_XBF) : nullptr;
    f.norm = (const float *)c->r(R_NORM);
    hipLaunchKernelGGL((k_features<DIM, SF>), dim3(c->P.np), dim3(FEAT_THREADS), 0, c->stream, f);
    return hip_ok(c, hipGetLastError());
}

// The learned closure in place of the Lagrangian-point exchange: features of
// the current state, the network, and its outputs as point forces and heat.
// With a feature range set, the point exchange runs first for every particle
// and the closure replaces its record and reactions only where every feature
// lies in the range.
template <int DIM, class SF>
int launch_closure(pibm_ctx *c)
{
    using T = typename SF::T;
    if (c->P.np == 0) return PIBM_OK;
    int st;
    if (c->closure_range && (st = launch_markers<DIM, SF>(c, true))) return st;
    if ((st = launch_features<DIM, SF>(c, c->closure_range, true))) return st;
    if ((st = pibm_mlp_forward_on(c->closure, c->r(R_XBF), (float *)c->r(R_YMLP), c->P.np, c->stream))) return st;
    const float *norm = (const float *)c->r(R_NORM);
    hipLaunchKernelGGL((k_closure<DIM, T>), dim3((c->P.np + 127) / 128), dim3(128), 0, c->stream,
                       (const DevParticle *)c->r(c->pcur ? R_PART1 : R_PART0), c->P.np, (const float *)c->r(R_YMLP),
                       norm, (const float *)c->r(R_AUX), c->closure_range ? (const float *)c->r(R_FEAT) : nullptr,
                       norm + 40, c->d.nu, c->d.alpha, c->p.kappa_T, (MarkerRec<T> *)c->r(R_MK),
                       (DevReact *)c->r(R_REACT), (int *)c->r(R_ERR));
    return hip_ok(c, hipGetLastError());
}

BinArgs bin_args(pibm_ctx *c, int set)
{
    BinArgs b{};
    b.dim = c->p.dim; b.nx = c->p.nx; b.ny = c->p.ny; b.nz = c->p.nz;
    for (int d = 0; d < 3; ++d) b.per[d] = c->p.periodic[d] ? 1 : 0;
    b.TX = c->P.TX; b.TY = c->P.TY; b.TZ = c->P.TZ;
    b.ntx = c->P.ntx; b.nty = c->P.nty; b.ntz = c->P.ntz;
    b.np = c->P.np;
    b.part = (const DevParticle *)c->r(c->pcur ? R_PART1 : R_PART0);
    b.tp_start = (const int *)c->r(R_TP_START);
    b.tp_box = (const double *)c->r(R_TP_BOX);
    b.gp_base = (const int *)c->r(R_GP_BASE);
    b.gp_start = (const int *)c->r(R_GP_START);
    b.cap = c->P.tile_cap;
    b.tile_count = (int *)c->r(set ? R_TCOUNT1 : R_TCOUNT);
    b.tile_start = (int *)c->r(set ? R_TSTART1 : R_TSTART);
    b.tile_fill = (int *)c->r(set ? R_TFILL1 : R_TFILL);
    b.tile_items = (int2 *)c->r(set ? R_TITEMS1 : R_TITEMS);
    b.err = (int *)c->r(R_ERR);
    return b;
}

// Tile lists of the current particle state into set `set`.
int launch_bin(pibm_ctx *c, hipStream_t s, int set)
{
    if (c->P.np == 0) return PIBM_OK;
    BinArgs b = bin_args(c, set);
    const int nt = c->P.ntiles;
    int *cntr = (int *)c->r(R_CNTR);
    if (c->P.np <= BIN_ONE_WG_PARTICLES && nt <= BIN_ONE_WG_TILES) {   // few particles and tiles: one launch
        hipLaunchKernelGGL(k_bin_one_wg, dim3(1), dim3(1024), 0, s, b, nt, cntr);
        return hip_ok(c, hipGetLastError());
    }
    hipLaunchKernelGGL(k_zero2, dim3(std::min(1024, (nt + 256) / 256)), dim3(256), 0, s, b.tile_count, (long long)nt,
                       cntr, 1LL);
    const int gb = (c->P.np + BIN_THREADS / 64 - 1) / (BIN_THREADS / 64);
    hipLaunchKernelGGL((k_bin<false>), dim3(gb), dim3(BIN_THREADS), 0, s, b);
    hipLaunchKernelGGL(k_alloc, dim3((nt + 255) / 256), dim3(256), 0, s, (const int *)b.tile_count, b.tile_start,
                       b.tile_fill, nt, cntr);
    hipLaunchKernelGGL((k_bin<true>), dim3(gb), dim3(BIN_THREADS), 0, s, b);

    return hip_ok(c, hipGetLastError());
}

template <int DIM, class SF, bool MACRO>
int launch_lbm(pibm_ctx *c)
{
    using T = typename SF::T;
    LbmArgs<T> a = lbm_args<T>(c);
    if (MACRO) a.macro = (T *)c->r(c->cur ? R_FA : R_FB);   // the idle copy holds the output
    hipLaunchKernelGGL((k_lbm<DIM, SF, MACRO>), dim3(c->P.ntiles), dim3(LBM_THREADS), 0, c->stream, a);
    return hip_ok(c, hipGetLastError());
}

DemArgs dem_args(pibm_ctx *c)
{
    DemArgs a{};
    a.dim = c->p.dim; a.nx = c->p.nx; a.ny = c->p.ny; a.nz = c->p.nz;
    for (int d = 0; d < 3; ++d) a.per[d] = c->p.periodic[d] ? 1 : 0;
    a.np = c->P.np;
    a.ncx = c->P.ncx; a.ncy = c->P.ncy; a.ncz = c->P.ncz;
    a.cwx = c->P.cwx; a.cwy = c->P.cwy; a.cwz = c->P.cwz;
    a.skin = c->P.skin;
    a.react = (const DevReact *)c->r(R_REACT);
    a.cell_count = (int *)c->r(R_CCOUNT);
    a.cell_start = (int *)c->r(R_CSTART);
    a.cell_fill = (int *)c->r(R_CFILL);
    a.cell_items = (int *)c->r(R_CITEMS);
    a.nbr = (int *)c->r(R_NBR);
    a.nbr_n = (int *)c->r(R_NBRN);
    a.xref = (double *)c->r(R_XREF);
    const double E = c->p.E_star, nu = c->p.poisson;
    a.E = E;
    a.G = (1.0 - nu) * E / (2.0 * (2.0 - nu));
    a.mu = c->p.mu_fric;
    a.dts = 1.0 / c->p.n_sub;
    a.gravity = c->p.gravity;
    a.beta_p = c->p.beta_p;
    a.c_r = c->p.c_r;
    a.Tref = c->p.T_ref;
    a.err = (int *)c->r(R_ERR);
    return a;
}

// Cell list of the current particle state (kept until the state changes).
int build_cells(pibm_ctx *c, hipStream_t s)
{
    if (c->P.np == 0 || c->cells_ok) return PIBM_OK;
    DemArgs a = dem_args(c);
    const int gb = (c->P.np + 127) / 128;
    a.cur = (const DevParticle *)c->r(c->pcur ? R_PART1 : R_PART0);
    int *cntr = (int *)c->r(R_CNTR) + 1;
    if (c->P.np <= ONE_WG_PARTICLES && c->P.ncells <= ONE_WG_LISTS) {   // few particles: one launch
        hipLaunchKernelGGL(k_cells_one_wg, dim3(1), dim3(ONE_WG), 0, s, a, (int)c->P.ncells, cntr);
        c->cells_ok = 1;
        return hip_ok(c, hipGetLastError());
    }
    hipLaunchKernelGGL(k_zero2, dim3(std::min(1024, (c->P.ncells + 256) / 256)), dim3(256), 0, s,
                       a.cell_count, (long long)c->P.ncells, cntr, 1LL);
    hipLaunchKernelGGL((k_cells<false>), dim3(gb), dim3(128), 0, s, a);
    hipLaunchKernelGGL(k_alloc, dim3((c->P.ncells + 255) / 256), dim3(256), 0, s, (const int *)a.cell_count,
                       a.cell_start, a.cell_fill, c->P.ncells, cntr);
    hipLaunchKernelGGL((k_cells<true>), dim3(gb), dim3(128), 0, s, a);
    c->cells_ok = 1;
    return hip_ok(c, hipGetLastError());
}

// Few particles, cells and tiles: the cell list and the tile lists (set
// `set`) of the current particle state in one launch.  Binning reads only
// the particle state, so on one stream it can precede the exchange.
bool cells_bin_fused(const pibm_ctx *c)
{
    return c->P.np > 0 && !c->cells_ok && c->P.np <= ONE_WG_PARTICLES && c->P.ncells <= ONE_WG_LISTS &&
           c->P.np <= BIN_ONE_WG_PARTICLES && c->P.ntiles <= BIN_ONE_WG_TILES;
}
int launch_cells_bin(pibm_ctx *c, hipStream_t s, int set)
{
    DemArgs a = dem_args(c);
    a.cur = (const DevParticle *)c->r(c->pcur ? R_PART1 : R_PART0);
    const BinArgs b = bin_args(c, set);
    int *cntr = (int *)c->r(R_CNTR);
    hipLaunchKernelGGL(k_cells_bin_one_wg, dim3(1), dim3(ONE_WG), 0, s, a, (int)c->P.ncells, cntr + 1, b,
                       c->P.ntiles, cntr);
    c->cells_ok = 1;
    return hip_ok(c, hipGetLastError());
}

int launch_dem(pibm_ctx *c, hipStream_t s)
{
    if (c->P.np == 0) return PIBM_OK;
    int st;
    if ((st = build_cells(c, s))) return st;
    DemArgs a = dem_args(c);
    a.cur = (const DevParticle *)c->r(c->pcur ? R_PART1 : R_PART0);
    hipLaunchKernelGGL(k_neighbours, dim3((c->P.np + NBR_THREADS / 64 - 1) / (NBR_THREADS / 64)), dim3(NBR_THREADS), 0,
                       s, a);
    if (c->P.np <= DEM_ONE_WG) {   // few particles: every sub-step in one launch
        DemOneWg f{};
        f.a = a;
        f.part[0] = (DevParticle *)c->r(c->pcur ? R_PART1 : R_PART0);
        f.part[1] = (DevParticle *)c->r(c->pcur ? R_PART0 : R_PART1);
        f.hid[0] = (int *)c->r(c->hcur ? R_HID1 : R_HID0);
        f.hid[1] = (int *)c->r(c->hcur ? R_HID0 : R_HID1);
        f.hxi[0] = (double *)c->r(c->hcur ? R_HXI1 : R_HXI0);
        f.hxi[1] = (double *)c->r(c->hcur ? R_HXI0 : R_HXI1);
        f.hn[0] = (int *)c->r(c->hcur ? R_HN1 : R_HN0);
        f.hn[1] = (int *)c->r(c->hcur ? R_HN0 : R_HN1);
        f.n_sub = c->p.n_sub;
        const int threads = (c->P.np + 63) / 64 * 64;
        if (c->P.np <= DEM_LDS) hipLaunchKernelGGL(k_dem_one_wg_lds, dim3(1), dim3(threads), 0, s, f);
        else hipLaunchKernelGGL(k_dem_one_wg, dim3(1), dim3(threads), 0, s, f);
        if (c->p.n_sub & 1) { c->pcur ^= 1; c->hcur ^= 1; }
        c->cells_ok = 0;
        return hip_ok(c, hipGetLastError());
    }
    for (int k = 0; k < c->p.n_sub; ++k) {
        a.cur = (const DevParticle *)c->r(c->pcur ? R_PART1 : R_PART0);
        a.nxt = (DevParticle *)c->r(c->pcur ? R_PART0 : R_PART1);
        a.hid_in = (const int *)c->r(c->hcur ? R_HID1 : R_HID0);
        a.hxi_in = (const double *)c->r(c->hcur ? R_HXI1 : R_HXI0);
        a.hn_in = (const int *)c->r(c->hcur ? R_HN1 : R_HN0);
        a.hid_out = (int *)c->r(c->hcur ? R_HID0 : R_HID1);
        a.hxi_out = (double *)c->r(c->hcur ? R_HXI0 : R_HXI1);
        a.hn_out = (int *)c->r(c->hcur ? R_HN0 : R_HN1);
        a.last = k == c->p.n_sub - 1;
        hipLaunchKernelGGL(k_dem, dim3((c->P.np + 127) / 128), dim3(128), 0, s, a);
        c->pcur ^= 1;
        c->hcur ^= 1;
        c->cells_ok = 0;
    }
    return hip_ok(c, hipGetLastError());
}

hipEvent_t take_event(pibm_ctx *c)
{
    if (!c->ev_free.empty()) {
        hipEvent_t e = c->ev_free.back();
        c->ev_free.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

// Records an event pair around one phase when profiling is on.
struct PhaseTimer {
    pibm_ctx *c;
    int phase;
    hipStream_t s;
    hipEvent_t a = nullptr, b = nullptr;
    PhaseTimer(pibm_ctx *ctx, int ph, hipStream_t st) : c(ctx), phase(ph), s(st) {
        if (((c->prof_mask >> ph) & 1u) && (a = take_event(c)) && (b = take_event(c))) (void)hipEventRecord(a, s);
    }
    PhaseTimer(pibm_ctx *ctx, int ph) : PhaseTimer(ctx, ph, ctx->stream) {}
    ~PhaseTimer() {
        if (a && b) {
            (void)hipEventRecord(b, s);
            c->ev_rec[phase].emplace_back(a, b);
        } else {
            if (a) c->ev_free.push_back(a);
            if (b) c->ev_free.push_back(b);
        }
    }
};

int rec(pibm_ctx *c, hipEvent_t ev, hipStream_t s) { return hip_ok(c, hipEventRecord(ev, s)); }
int wait(pibm_ctx *c, hipStream_t s, hipEvent_t ev) { return hip_ok(c, hipStreamWaitEvent(s, ev, 0)); }

// One step: exchange, binning, lattice, DEM, in this order on the caller's
// stream, or on two streams.  Binning reads only the particle state, so it runs
// beside the exchange (markers or closure).  The DEM reads the particle state
// and the exchange's reactions and writes the other particle buffer and the
// contact history, none of which the lattice kernel touches, so it runs
// beside the lattice kernel:
//   stream: exchange --(mk)-- [wait(bin)] -- lattice -- wait(join)
//   side:   [wait(start) -- bin --(bin)--] wait(mk) -- DEM, next cell list, next bin --(join)
// From the second step on, the bracketed binning is skipped: the previous
// step binned into the idle tile-list set beside its lattice kernel.
// Binning precedes the DEM on the side stream, so the particle buffer it
// reads is overwritten only after it finished.
template <int DIM, class SF>
int step_impl(pibm_ctx *c, int n)
{
    if (!c->two) {
        for (int k = 0; k < n; ++k) {
            int st;
            const bool fused = cells_bin_fused(c);
            if (fused) { PhaseTimer t(c, PIBM_PHASE_BIN); if ((st = launch_cells_bin(c, c->stream, c->tcur))) return st; }
            {
                PhaseTimer t(c, PIBM_PHASE_MARKERS);
                if ((st = c->closure ? launch_closure<DIM, SF>(c) : launch_markers<DIM, SF>(c, true))) return st;
            }
            if (!fused) { PhaseTimer t(c, PIBM_PHASE_BIN); if ((st = launch_bin(c, c->stream, c->tcur))) return st; }
            { PhaseTimer t(c, PIBM_PHASE_LATTICE); if ((st = launch_lbm<DIM, SF, false>(c))) return st; }
            { PhaseTimer t(c, PIBM_PHASE_DEM); if ((st = launch_dem(c, c->stream))) return st; }
            c->cur ^= 1;
            c->step++;
        }
        return PIBM_OK;
    }
    const bool parts = c->P.np > 0;
    for (int k = 0; k < n; ++k) {
        int st;
        // the previous step binned this one into the idle set, beside its lattice kernel
        const bool binned = parts && c->tiles_next;
        if (binned) { c->tcur ^= 1; c->tiles_next = 0; }
        if (parts && !binned) {
            if ((st = rec(c, c->ev_start, c->stream)) || (st = wait(c, c->side, c->ev_start))) return st;
            { PhaseTimer t(c, PIBM_PHASE_BIN, c->side); if ((st = launch_bin(c, c->side, c->tcur))) return st; }
            if ((st = rec(c, c->ev_bin, c->side))) return st;
        }
        {
            PhaseTimer t(c, PIBM_PHASE_MARKERS);
            if ((st = c->closure ? launch_closure<DIM, SF>(c) : launch_markers<DIM, SF>(c, true))) return st;
        }
        if (parts) {
            if ((st = rec(c, c->ev_mk, c->stream)) || (st = wait(c, c->side, c->ev_mk))) return st;
            {
                PhaseTimer t(c, PIBM_PHASE_DEM, c->side);
                if ((st = launch_dem(c, c->side))) return st;
                // the next step's cell list from the new state, beside the lattice kernel
                // (nothing reads the list until the next exchange)
                if ((st = build_cells(c, c->side))) return st;
            }
            // the next step's tile lists into the idle set (its last reader, the
            // previous lattice kernel, finished before this exchange)
            { PhaseTimer t(c, PIBM_PHASE_BIN, c->side); if ((st = launch_bin(c, c->side, c->tcur ^ 1))) return st; }
            c->tiles_next = 1;
            if ((st = rec(c, c->ev_join, c->side))) return st;
            if (!binned && (st = wait(c, c->stream, c->ev_bin))) return st;
        }
        { PhaseTimer t(c, PIBM_PHASE_LATTICE); if ((st = launch_lbm<DIM, SF, false>(c))) return st; }
        if (parts && (st = wait(c, c->stream, c->ev_join))) return st;
        c->cur ^= 1;
        c->step++;
    }
    return PIBM_OK;
}

template <int DIM, class SF>
int macro_impl(pibm_ctx *c)
{
    int st;
    if ((st = c->closure ? launch_closure<DIM, SF>(c) : launch_markers<DIM, SF>(c, false))) return st;
    c->tiles_next = 0;             // rebinning here; the next step bins again
    if ((st = launch_bin(c, c->stream, c->tcur))) return st;
    return launch_lbm<DIM, SF, true>(c);
}

// FP32 / FP64 instances: flow lattice (D2Q9, D3Q19 or D3Q15) x thermal model
// (D2Q5 / D3Q7 linear, or the flow lattice with the quadratic equilibrium)
template <template <int, class> class F, class SF, typename... A>
int dispatch_lattices(pibm_ctx *c, A... args)
{
    const bool qt = c->p.thermal_model == 1;
    if (c->p.dim == 2) return qt ? F<2, OnQuadT<SF>>::run(c, args...) : F<2, SF>::run(c, args...);
    if (c->p.lattice == 15) return qt ? F<3, OnQuadT<OnQ15<SF>>>::run(c, args...) : F<3, OnQ15<SF>>::run(c, args...);
    return qt ? F<3, OnQuadT<SF>>::run(c, args...) : F<3, SF>::run(c, args...);
}

template <template <int, class> class F, typename... A>
int dispatch(pibm_ctx *c, A... args)
{
    const bool d3 = c->p.dim == 3;
    switch (c->p.storage) {
    case PIBM_STORE_F32: return dispatch_lattices<F, StF32>(c, args...);
    case PIBM_STORE_F64: return dispatch_lattices<F, StF64>(c, args...);
    case PIBM_STORE_F16DEV: return d3 ? F<3, StF16>::run(c, args...) : F<2, StF16>::run(c, args...);
    default: return d3 ? F<3, StBF16>::run(c, args...) : F<2, StBF16>::run(c, args...);
    }
}

template <int DIM, class SF> struct StepOp { static int run(pibm_ctx *c, int n) { return step_impl<DIM, SF>(c, n); } };

// Features of the current state, the resolved exchange's reactions for it,
// and the targets in the same slip frame.
template <int DIM, class SF>
int features_impl(pibm_ctx *c)
{
    int st;
    if ((st = launch_features<DIM, SF>(c, true, false))) return st;
    if ((st = launch_markers<DIM, SF>(c, true))) return st;
    hipLaunchKernelGGL((k_targets<DIM>), dim3((c->P.np + 127) / 128), dim3(128), 0, c->stream,
                       (const DevParticle *)c->r(c->pcur ? R_PART1 : R_PART0), c->P.np, (const DevReact *)c->r(R_REACT),
                       (const float *)c->r(R_AUX), c->d.nu, c->d.alpha, (float *)c->r(R_TARG));
    return hip_ok(c, hipGetLastError());
}
template <int DIM, class SF> struct FeatOp { static int run(pibm_ctx *c) { return features_impl<DIM, SF>(c); } };
template <int DIM, class SF> struct MacroOp { static int run(pibm_ctx *c) { return macro_impl<DIM, SF>(c); } };
template <int DIM, class SF> struct InitOp {
    static int run(pibm_ctx *c) {
        using T = typename SF::T;
        const int g = (int)std::min<long long>(4096, (c->P.N + 255) / 256);
        hipLaunchKernelGGL((k_init<SF, LatOf<DIM, SF>>), dim3(g), dim3(256), 0, c->stream, c->r(R_FA), c->r(R_GA),
                           c->P.N, c->P.Ns, (T)(c->p.T_init - c->T_store));
        return hip_ok(c, hipGetLastError());
    }
};

// ---- host conversions between absolute doubles and stored deviations ----
float half_to_float(uint16_t h) { _Float16 v; std::memcpy(&v, &h, 2); return (float)v; }
uint16_t float_to_half(float f) { _Float16 v = (_Float16)f; uint16_t h; std::memcpy(&h, &v, 2); return h; }
float bf16_to_float(uint16_t h) { uint32_t u = (uint32_t)h << 16; float f; std::memcpy(&f, &u, 4); return f; }
uint16_t float_to_bf16(float f)
{
    uint32_t u;
    std::memcpy(&u, &f, 4);
    if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u | 0x00400000u) >> 16);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

double stored_to_dev(const pibm_ctx *c, const char *buf, size_t i, double w)
{
    switch (c->p.storage) {
    case PIBM_STORE_F32: return ((const float *)buf)[i];
    case PIBM_STORE_F64: return ((const double *)buf)[i];
    case PIBM_STORE_F16DEV: return (double)(half_to_float(((const uint16_t *)buf)[i]) * (float)w);
    default: return (double)(bf16_to_float(((const uint16_t *)buf)[i]) * (float)w);
    }
}

void dev_to_stored(const pibm_ctx *c, char *buf, size_t i, double v, double w)
{
    switch (c->p.storage) {
    case PIBM_STORE_F32: ((float *)buf)[i] = (float)v; break;
    case PIBM_STORE_F64: ((double *)buf)[i] = v; break;
    case PIBM_STORE_F16DEV: ((uint16_t *)buf)[i] = float_to_half((float)v * (float)(1.0 / w)); break;
    default: ((uint16_t *)buf)[i] = float_to_bf16((float)v * (float)(1.0 / w)); break;
    }
}

double wf(int dim, int lattice, int q)
{
    return dim == 2 ? Lat<2>::w(q) : (lattice == 15 ? LatT<3, 15>::w(q) : Lat<3>::w(q));
}
double wgt(int dim, int lattice, int thermal_model, int q)
{
    return thermal_model == 1 ? wf(dim, lattice, q) : (dim == 2 ? Lat<2>::wg(q) : Lat<3>::wg(q));
}

DevParticle to_dev(const pibm_particle &q, int tmpl)
{
    DevParticle d{};
    for (int k = 0; k < 3; ++k) { d.x[k] = q.x[k]; d.u[k] = q.u[k]; d.om[k] = q.omega[k]; d.th[k] = q.theta[k]; }
    d.R = q.R; d.rho_r = q.rho_r; d.T = q.T; d.flags = q.flags; d.tmpl = tmpl;
    return d;
}

int upload_particles(pibm_ctx *c, const pibm_particle *pt, int n)
{
    std::vector<DevParticle> dp(std::max(n, 1));
    for (int i = 0; i < n; ++i) dp[i] = to_dev(pt[i], c->P.ptmpl[i]);
    c->cells_ok = 0;
    c->tiles_next = 0;
    if (n == 0) return PIBM_OK;
    hipError_t e = hipMemcpyAsync(c->r(c->pcur ? R_PART1 : R_PART0), dp.data(), sizeof(DevParticle) * n,
                                  hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    return hip_ok(c, e);
}

int status_from_err(int e)
{
    if (e & (ERR_CONTACTS | ERR_NEIGHBOURS | ERR_TILES)) return PIBM_ENOMEM;
    if (e) return PIBM_EUNSTABLE;
    return PIBM_OK;
}

int sync_impl(pibm_ctx *c)
{
    int e = 0;
    hipError_t he = hipMemcpyAsync(&e, c->r(R_ERR), sizeof(int), hipMemcpyDeviceToHost, c->stream);
    if (he == hipSuccess) he = hipStreamSynchronize(c->stream);
    if (he != hipSuccess) return hip_ok(c, he);
    if (e && !c->sticky) c->sticky = status_from_err(e);
    return c->sticky;
}

}  // namespace

// ============================================================================
// C ABI
// ============================================================================
extern "C" {

size_t pibm_workspace_bytes(const pibm_params *p, const pibm_particle *pt, int n)
{
    Plan P;
    if (make_plan(p, pt, n, P) != PIBM_OK) return 0;
    return P.off[R_COUNT];
}

int pibm_init(pibm_ctx **out, const pibm_params *p, const pibm_particle *pt, int n, void *ws, size_t ws_bytes,
              void *stream)
{
    if (!out) return PIBM_EINVAL;
    *out = nullptr;
    pibm_ctx *c = new (std::nothrow) pibm_ctx();
    if (!c) return PIBM_EINVAL;
    int st = make_plan(p, pt, n, c->P);
    if (st == PIBM_OK) st = check_particles(p, pt, n);
    if (st == PIBM_OK && (!ws || ((uintptr_t)ws % ALIGN) != 0 || ws_bytes < c->P.off[R_COUNT])) st = PIBM_EINVAL;
    if (st != PIBM_OK) { delete c; return st; }
    c->p = *p;
    c->d = derive(*p);
    c->T_store = p->T_ref;
    if (p->storage == PIBM_STORE_F16DEV || p->storage == PIBM_STORE_BF16DEV) {
        double lo = p->T_init, hi = p->T_init;
        for (int f = 0; f < 2 * p->dim; ++f)
            if (!p->periodic[f / 2]) { lo = std::min(lo, p->T_wall[f]); hi = std::max(hi, p->T_wall[f]); }
        for (int i = 0; i < n; ++i) { lo = std::min(lo, pt[i].T); hi = std::max(hi, pt[i].T); }
        c->T_store = 0.5 * (lo + hi);
    }
    c->stream = (hipStream_t)stream;
    c->ws = (char *)ws;
    c->ws_bytes = ws_bytes;
    c->cur = 0; c->pcur = 0; c->hcur = 0; c->step = 0; c->sticky = 0; c->device_lost = 0; c->cells_ok = 0;
    c->two = c->P.np > 0 && (p->streams == 2 || (p->streams == 0 && c->P.N >= (1LL << 22)));
    if (c->two) {   // the side stream and the fork/join events, on the device of the caller's stream
        int dev = 0, cur = 0;
        hipError_t e = hipStreamGetDevice(c->stream, &dev);
        if (e == hipSuccess) e = hipGetDevice(&cur);
        if (e == hipSuccess && dev != cur) e = hipSetDevice(dev);
        if (e == hipSuccess) e = hipStreamCreateWithFlags(&c->side, hipStreamNonBlocking);
        for (hipEvent_t *ev : {&c->ev_start, &c->ev_bin, &c->ev_mk, &c->ev_join})
            if (e == hipSuccess) e = hipEventCreateWithFlags(ev, hipEventDisableTiming);
        if (dev != cur) (void)hipSetDevice(cur);
        if (e != hipSuccess) { delete c; return PIBM_EDEVICE; }
    }
    // templates, marker offsets
    std::vector<double> tm((size_t)std::max(c->P.ntmpl_mk, 1LL) * 4, 0.0);
    std::vector<int> ts(c->P.tmpls.size() + 1, 0);
    std::vector<double> rext(c->P.tmpls.size() + 1, 0.0);
    size_t k = 0;
    for (size_t t = 0; t < c->P.tmpls.size(); ++t) {
        ts[t] = (int)(k / 4);
        std::copy(c->P.tmpls[t].off.begin(), c->P.tmpls[t].off.end(), tm.begin() + k);
        k += c->P.tmpls[t].off.size();
        rext[t] = p->marker_mode == PIBM_MARKERS_POINT ? 0.0 : c->P.tmpls[t].R;
    }
    ts[c->P.tmpls.size()] = (int)(k / 4);
    hipError_t e = hipMemcpyAsync(c->r(R_TMPL), tm.data(), tm.size() * sizeof(double), hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(c->r(R_TMPL_START), ts.data(), ts.size() * sizeof(int), hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(c->r(R_TMPL_REXT), rext.data(), rext.size() * sizeof(double), hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(c->r(R_MK_START), c->P.mk_start.data(), c->P.mk_start.size() * sizeof(int), hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(c->r(R_TP_START), c->P.tp_start.data(), c->P.tp_start.size() * sizeof(int), hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess && !c->P.tp_box.empty())
        e = hipMemcpyAsync(c->r(R_TP_BOX), c->P.tp_box.data(), c->P.tp_box.size() * sizeof(double), hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(c->r(R_GP_START), c->P.gp_start.data(), c->P.gp_start.size() * sizeof(int), hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(c->r(R_GP_BASE), c->P.gp_base.data(), c->P.gp_base.size() * sizeof(int), hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) { delete c; return PIBM_EDEVICE; }
    // zeroed small state: tile starts (no particles => empty lists), history counts, error word
    const int zero_regions[] = {R_TSTART, R_TCOUNT, R_TSTART1, R_TCOUNT1, R_CCOUNT, R_CITEMS, R_CNTR, R_HN0, R_HN1, R_ERR, R_REACT};
    for (int r : zero_regions) {
        const size_t bytes = c->P.off[r + 1] - c->P.off[r];
        hipLaunchKernelGGL(k_fill_int, dim3(std::max<size_t>(1, std::min<size_t>(1024, (bytes / 4 + 255) / 256))), dim3(256), 0,
                           c->stream, (int *)c->r(r), (long long)(bytes / 4), 0);
    }
    st = dispatch<InitOp>(c);
    if (st == PIBM_OK) st = upload_particles(c, pt, n);
    if (st == PIBM_OK) st = hip_ok(c, hipStreamSynchronize(c->stream));
    if (st != PIBM_OK) { delete c; return st; }
    *out = c;
    return PIBM_OK;
}

int pibm_step(pibm_ctx *c, int n)
{
    if (!c || n < 0) return PIBM_EINVAL;
    if (c->device_lost) return PIBM_EDEVICE;
    if (c->sticky) return c->sticky;         // the watchdog tripped: no further launches
    return dispatch<StepOp>(c, n);
}

int pibm_sync(pibm_ctx *c)
{
    if (!c) return PIBM_EINVAL;
    if (c->device_lost) return PIBM_EDEVICE;
    return sync_impl(c);
}

int pibm_particles(pibm_ctx *c, pibm_particle *out, double *fth, int cap)
{
    if (!c || (!out && cap > 0) || cap < c->P.np) return PIBM_EINVAL;
    if (c->device_lost) return PIBM_EDEVICE;
    const int n = c->P.np;
    std::vector<DevParticle> dp(std::max(n, 1));
    std::vector<DevReact> dr(std::max(n, 1));
    if (n) {
        hipError_t e = hipMemcpyAsync(dp.data(), c->r(c->pcur ? R_PART1 : R_PART0), sizeof(DevParticle) * n,
                                      hipMemcpyDeviceToHost, c->stream);
        if (e == hipSuccess) e = hipMemcpyAsync(dr.data(), c->r(R_REACT), sizeof(DevReact) * n, hipMemcpyDeviceToHost, c->stream);
        if (e != hipSuccess) return hip_ok(c, e);
    }
    const int st = sync_impl(c);
    if (c->device_lost) return PIBM_EDEVICE;
    for (int i = 0; i < n; ++i) {
        pibm_particle &q = out[i];
        for (int k = 0; k < 3; ++k) { q.x[k] = dp[i].x[k]; q.u[k] = dp[i].u[k]; q.omega[k] = dp[i].om[k]; q.theta[k] = dp[i].th[k]; }
        q.R = dp[i].R; q.rho_r = dp[i].rho_r; q.T = dp[i].T; q.flags = dp[i].flags; q.reserved = 0;
        if (fth) {
            double *o = fth + 8 * (size_t)i;
            for (int k = 0; k < 3; ++k) { o[k] = dr[i].F[k]; o[3 + k] = dr[i].tq[k]; }
            o[6] = dr[i].H; o[7] = dr[i].dTA;
        }
    }
    return st;
}

int pibm_set_particles(pibm_ctx *c, const pibm_particle *pt, int n)
{
    if (!c || n != c->P.np || (n && !pt)) return PIBM_EINVAL;
    for (int i = 0; i < n; ++i)
        if (pt[i].R != c->P.tmpls[c->P.ptmpl[i]].R) return PIBM_EINVAL;
    int st = check_particles(&c->p, pt, n);
    if (st) return st;
    return upload_particles(c, pt, n);
}

int pibm_fields(pibm_ctx *c, double *rho, double *u, double *T)
{
    if (!c) return PIBM_EINVAL;
    if (c->device_lost) return PIBM_EDEVICE;
    int st = dispatch<MacroOp>(c);
    if (st) return st;
    const size_t ts = c->P.tsize, Ns = (size_t)c->P.Ns, N = (size_t)c->P.N;
    std::vector<char> h(5 * Ns * ts);
    hipError_t e = hipMemcpyAsync(h.data(), c->r(c->cur ? R_FA : R_FB), h.size(), hipMemcpyDeviceToHost, c->stream);
    if (e != hipSuccess) return hip_ok(c, e);
    st = sync_impl(c);
    if (c->device_lost) return PIBM_EDEVICE;
    auto get = [&](int k, size_t n) -> double {
        return ts == 8 ? ((const double *)h.data())[k * Ns + n] : (double)((const float *)h.data())[k * Ns + n];
    };
    for (size_t n = 0; n < N; ++n) {
        if (rho) rho[n] = get(0, n);
        if (u) { u[3 * n] = get(1, n); u[3 * n + 1] = get(2, n); u[3 * n + 2] = get(3, n); }
        if (T) T[n] = get(4, n);
    }
    return st;
}

int pibm_features(pibm_ctx *c, float *x, float *t)
{
    if (!c) return PIBM_EINVAL;
    if (c->device_lost) return PIBM_EDEVICE;
    if (c->sticky) return c->sticky;
    if (c->P.np == 0) return PIBM_OK;
    int st = dispatch<FeatOp>(c);
    if (st) return st;
    const size_t np = (size_t)c->P.np;
    hipError_t e = hipSuccess;
    if (x) e = hipMemcpyAsync(x, c->r(R_FEAT), np * 16 * sizeof(float), hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess && t) e = hipMemcpyAsync(t, c->r(R_TARG), np * 4 * sizeof(float), hipMemcpyDeviceToHost, c->stream);
    if (e != hipSuccess) return hip_ok(c, e);
    return sync_impl(c);
}

int pibm_set_closure(pibm_ctx *c, pibm_mlp *m, const float *norm)
{
    if (!c) return PIBM_EINVAL;
    if (c->device_lost) return PIBM_EDEVICE;
    if (!m) { c->closure = nullptr; c->closure_range = false; return PIBM_OK; }
    if (c->p.marker_mode != PIBM_MARKERS_POINT || !norm) return PIBM_EINVAL;
    for (int i = 0; i < 40; ++i)
        if (!std::isfinite(norm[i])) return PIBM_EINVAL;
    for (int i = 0; i < 16; ++i)
        if (!(norm[16 + i] > 0.f)) return PIBM_EINVAL;
    for (int i = 0; i < 4; ++i)
        if (!(norm[36 + i] > 0.f)) return PIBM_EINVAL;
    hipError_t e = hipMemcpyAsync(c->r(R_NORM), norm, 40 * sizeof(float), hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return hip_ok(c, e);
    c->closure = m;
    c->closure_range = false;
    return PIBM_OK;
}

int pibm_set_closure_range(pibm_ctx *c, const float *lo, const float *hi)
{
    if (!c) return PIBM_EINVAL;
    if (c->device_lost) return PIBM_EDEVICE;
    if (!lo && !hi) { c->closure_range = false; return PIBM_OK; }
    if (!c->closure || !lo || !hi) return PIBM_EINVAL;
    float b[32];
    for (int i = 0; i < 16; ++i) {
        if (std::isnan(lo[i]) || std::isnan(hi[i])) return PIBM_EINVAL;
        b[i] = lo[i];
        b[16 + i] = hi[i];
    }
    hipError_t e = hipMemcpyAsync((float *)c->r(R_NORM) + 40, b, sizeof b, hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return hip_ok(c, e);
    c->closure_range = true;
    return PIBM_OK;
}

int pibm_get_populations(pibm_ctx *c, double *f, double *g)
{
    if (!c || !f || !g) return PIBM_EINVAL;
    if (c->device_lost) return PIBM_EDEVICE;
    const int dim = c->p.dim, Q = c->P.Q, QG = c->P.QG;
    const size_t Ns = (size_t)c->P.Ns, N = (size_t)c->P.N, ss = c->P.ssize;
    std::vector<char> hf(Q * Ns * ss), hg(QG * Ns * ss);
    hipError_t e = hipMemcpyAsync(hf.data(), c->r(c->cur ? R_FB : R_FA), hf.size(), hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(hg.data(), c->r(c->cur ? R_GB : R_GA), hg.size(), hipMemcpyDeviceToHost, c->stream);
    if (e != hipSuccess) return hip_ok(c, e);
    const int st = sync_impl(c);
    if (c->device_lost) return PIBM_EDEVICE;
    for (int q = 0; q < Q; ++q)
        for (size_t n = 0; n < N; ++n) f[q * N + n] = wf(dim, c->p.lattice, q) + stored_to_dev(c, hf.data(), q * Ns + n, wf(dim, c->p.lattice, q));
    for (int q = 0; q < QG; ++q)
        for (size_t n = 0; n < N; ++n)
            g[q * N + n] = wgt(dim, c->p.lattice, c->p.thermal_model, q) * c->T_store + stored_to_dev(c, hg.data(), q * Ns + n, wgt(dim, c->p.lattice, c->p.thermal_model, q));
    return st;
}

int pibm_set_populations(pibm_ctx *c, const double *f, const double *g)
{
    if (!c || !f || !g) return PIBM_EINVAL;
    if (c->device_lost) return PIBM_EDEVICE;
    const int dim = c->p.dim, Q = c->P.Q, QG = c->P.QG;
    const size_t Ns = (size_t)c->P.Ns, N = (size_t)c->P.N, ss = c->P.ssize;
    std::vector<char> hf(Q * Ns * ss, 0), hg(QG * Ns * ss, 0);
    for (int q = 0; q < Q; ++q)
        for (size_t n = 0; n < N; ++n) dev_to_stored(c, hf.data(), q * Ns + n, f[q * N + n] - wf(dim, c->p.lattice, q), wf(dim, c->p.lattice, q));
    for (int q = 0; q < QG; ++q)
        for (size_t n = 0; n < N; ++n)
            dev_to_stored(c, hg.data(), q * Ns + n, g[q * N + n] - wgt(dim, c->p.lattice, c->p.thermal_model, q) * c->T_store, wgt(dim, c->p.lattice, c->p.thermal_model, q));
    hipError_t e = hipMemcpyAsync(c->r(c->cur ? R_FB : R_FA), hf.data(), hf.size(), hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(c->r(c->cur ? R_GB : R_GA), hg.data(), hg.size(), hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    return hip_ok(c, e);
}

long long pibm_num_nodes(const pibm_ctx *c) { return c ? c->P.N : 0; }
long long pibm_num_markers(const pibm_ctx *c) { return c ? c->P.nmk : 0; }
long long pibm_step_count(const pibm_ctx *c) { return c ? c->step : 0; }

int pibm_derived(const pibm_ctx *c, double *out)
{
    if (!c || !out) return PIBM_EINVAL;
    out[0] = c->d.tau_f; out[1] = c->d.tau_g; out[2] = c->d.gbeta; out[3] = c->d.nu; out[4] = c->d.alpha;
    return PIBM_OK;
}

// ---- checkpoint blob: header, then raw device regions ----
namespace {
struct BlobHeader {
    char magic[8];
    int version;
    int cur, pcur, hcur;
    long long step;
    pibm_params p;
    long long N, np;
    double T_store;                // the populations' g offset (pibm_ctx::T_store)
};
const int blob_regions[] = {R_FA, R_GA, R_FB, R_GB, R_PART0, R_PART1, R_REACT, R_HID0, R_HXI0, R_HN0, R_HID1, R_HXI1, R_HN1};
}

int pibm_save(pibm_ctx *c, void *buf, size_t cap, size_t *used)
{
    if (!c || !used) return PIBM_EINVAL;
    size_t total = sizeof(BlobHeader);
    for (int r : blob_regions) total += c->P.off[r + 1] - c->P.off[r];
    *used = total;
    if (!buf) return PIBM_OK;
    if (cap < total) return PIBM_EINVAL;
    BlobHeader h{};
    std::memcpy(h.magic, "PIBMCKP", 8);
    h.version = 2; h.cur = c->cur; h.pcur = c->pcur; h.hcur = c->hcur; h.step = c->step; h.p = c->p;
    h.T_store = c->T_store;
    h.N = c->P.N; h.np = c->P.np;
    std::memcpy(buf, &h, sizeof h);
    char *o = (char *)buf + sizeof h;
    for (int r : blob_regions) {
        const size_t b = c->P.off[r + 1] - c->P.off[r];
        hipError_t e = hipMemcpyAsync(o, c->r(r), b, hipMemcpyDeviceToHost, c->stream);
        if (e != hipSuccess) return hip_ok(c, e);
        o += b;
    }
    return hip_ok(c, hipStreamSynchronize(c->stream));
}

int pibm_load(pibm_ctx *c, const void *buf, size_t n)
{
    if (!c || !buf || n < sizeof(BlobHeader)) return PIBM_EINVAL;
    BlobHeader h;
    std::memcpy(&h, buf, sizeof h);
    if (std::memcmp(h.magic, "PIBMCKP", 8) != 0 || h.version != 2) return PIBM_ESTATE;
    if (std::memcmp(&h.p, &c->p, sizeof(pibm_params)) != 0 || h.N != c->P.N || h.np != c->P.np) return PIBM_ESTATE;
    size_t total = sizeof(BlobHeader);
    for (int r : blob_regions) total += c->P.off[r + 1] - c->P.off[r];
    if (n < total) return PIBM_EINVAL;
    const char *o = (const char *)buf + sizeof h;
    for (int r : blob_regions) {
        const size_t b = c->P.off[r + 1] - c->P.off[r];
        hipError_t e = hipMemcpyAsync(c->r(r), o, b, hipMemcpyHostToDevice, c->stream);
        if (e != hipSuccess) return hip_ok(c, e);
        o += b;
    }
    c->cur = h.cur; c->pcur = h.pcur; c->hcur = h.hcur; c->step = h.step; c->cells_ok = 0; c->tiles_next = 0;
    c->T_store = h.T_store;
    return hip_ok(c, hipStreamSynchronize(c->stream));
}

int pibm_profile(pibm_ctx *c, int enable)
{
    if (!c) return PIBM_EINVAL;
    c->prof_mask = enable ? (1u << PIBM_NPHASE) - 1u : 0u;
    return PIBM_OK;
}

int pibm_profile_phases(pibm_ctx *c, unsigned phase_mask)
{
    if (!c || (phase_mask >> PIBM_NPHASE)) return PIBM_EINVAL;
    c->prof_mask = phase_mask;
    return PIBM_OK;
}

int pibm_profile_read(pibm_ctx *c, double *ms, long long *count)
{
    if (!c || !ms || !count) return PIBM_EINVAL;
    if (c->device_lost) return PIBM_EDEVICE;
    hipError_t e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return hip_ok(c, e);
    for (int ph = 0; ph < PIBM_NPHASE; ++ph) {
        double acc = 0.0;
        for (auto &pr : c->ev_rec[ph]) {
            float t = 0.0f;
            if (hipEventElapsedTime(&t, pr.first, pr.second) == hipSuccess) acc += t;
            c->ev_free.push_back(pr.first);
            c->ev_free.push_back(pr.second);
        }
        ms[ph] = acc;
        count[ph] = (long long)c->ev_rec[ph].size();
        c->ev_rec[ph].clear();
    }
    return PIBM_OK;
}

int pibm_destroy(pibm_ctx *c)
{
    if (!c) return PIBM_OK;
    for (int ph = 0; ph < PIBM_NPHASE; ++ph)
        for (auto &pr : c->ev_rec[ph]) c->ev_free.insert(c->ev_free.end(), {pr.first, pr.second});
    for (hipEvent_t e : c->ev_free) (void)hipEventDestroy(e);
    delete c;
    return PIBM_OK;
}

const char *pibm_strerror(int s)
{
    switch (s) {
    case PIBM_OK: return "ok";
    case PIBM_EINVAL: return "invalid argument (parameters, sizes, pointers or workspace)";
    case PIBM_ENOMEM: return "device capacity exceeded (contact slots or neighbour list)";
    case PIBM_EDEVICE: return "HIP runtime error";
    case PIBM_EUNSTABLE: return "watchdog: NaN or |u| > 0.4, stale neighbour list, or particle outside the domain";
    case PIBM_EOVERLAP: return "initial particles overlap";
    case PIBM_ESTATE: return "checkpoint does not match this context";
    default: return "unknown status";
    }
}

}  // extern "C"
