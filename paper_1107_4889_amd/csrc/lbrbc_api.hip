// lbrbc_api.hip -- C ABI of the MI355X library: arena layout, host-side geometry tables,
// step orchestration on the caller's stream, getters/setters, checkpoints, timing.
#include <algorithm>
#include <array>
#include <cmath>
#include <mutex>
#include <cstring>
#include <string>
#include <type_traits>
#include <vector>

#include "../../include/lbrbc.h"
#include "lbrbc_device.h"
#include "lbrbc_internal.h"

using namespace lbrbc;

namespace {

constexpr size_t ALIGN = 256;
constexpr int OBS_BLOCKS = 1024;
constexpr int MAX_TIMED = 4096;

size_t up(size_t v) { return (v + ALIGN - 1) / ALIGN * ALIGN; }

// automatic layout choice: the compact layout (only the 64-node row segments holding fluid are
// stored) when fewer than this fraction of all row segments hold fluid (the straight tubes:
// 80-94%, dense; the Y-bifurcation in its box: a few per cent, compact)
constexpr double COMPACT_MAX_FRACTION = 0.6;

int storage_bytes(int s) { return s == LB_F64 ? 8 : (s == LB_F32 ? 4 : 2); }
int real_bytes(int s) { return s == LB_F64 ? 8 : 4; }
// u and sigma elements: the compute precision, or 16 bits (BF16, or FP16 times 2^12) for the
// 16-bit storages, whose velocity record is padded to four elements
int field_bytes(int s) { return storage_bytes(s); }
int vel_stride(int s) { return field_bytes(s) == 2 ? 4 : 3; }
constexpr double FIELD16_SCALE_HOST = FIELD16_SCALE;   // the device's FP16 field scale

// ---- host geometry tables --------------------------------------------------------------------
struct Geometry {
    long long nodes = 0;             // lattice nodes nx ny nz
    long long N = 0, ld = 0, n_fluid = 0;   // storage slots (nodes, or 64 per stored segment)
    bool compact = false;
    int nbx = 1;                     // 64-node column segments per row
    std::vector<uint32_t> nodeword;  // per storage slot
    std::vector<int> wall_xyz;       // solid nodes with a fluid D3Q19 neighbour
    std::vector<long long> wn_node;  // wall-adjacent fluid nodes: storage index
    std::vector<long long> wn_dense; //   and lattice index x + nx (y + ny z)
    std::vector<double> wn_nrm;
    std::vector<int> planes;         // open-boundary plane nodes: (k, k of the inner neighbour
                                     // or -1 when solid, x | y << 16, z)
    std::vector<int> segs;           // compact layout: (x0, y, z, 0) per stored segment,
    std::vector<int> segnb;          //   27 neighbour segments each,
    std::vector<int> segmap;         //   stored segment per column segment, or -1
    // storage index of lattice node n (x + nx (y + ny z)), -1 when not stored
    long long store_of(long long n, int nx, int ny) const
    {
        if (!compact) return n;
        const long long x = n % nx, row = n / nx;
        const int sg = segmap[(size_t)((x >> 6) + (long long)nbx * row)];
        (void)ny;
        return sg < 0 ? -1 : ((long long)sg << 6) | (x & 63);
    }
    int ncell[3] = {1, 1, 1};
    double cedge[3] = {1, 1, 1};
    int wncell[3] = {1, 1, 1};        // grid of the wall points, edge >= the cell-wall cut-off
    double wcedge[3] = {1, 1, 1};
    double rc = 0;
    std::vector<int> wcell_off, wcell_ids;
    int tile_max = 0;
    int cand_cap = 0;
    int ent_shift = 0;
};

// FNV-1a over the layout and the node words (in storage order)
unsigned long long geometry_hash(const Geometry& g)
{
    unsigned long long h = 1469598103934665603ull;
    h ^= g.compact ? 1u : 0u;
    h *= 1099511628211ull;
    for (uint32_t w : g.nodeword)
        for (int b = 0; b < 4; ++b) {
            h ^= (w >> (8 * b)) & 0xffu;
            h *= 1099511628211ull;
        }
    return h;
}

// Capacity of the one-wavefront map pass: the largest number of candidate nodes (the
// covered x-range of every support-tile row, computed as the kernel does) over 4096
// orientations and sub-node offsets from a fixed generator, with 20% and 64 nodes of margin;
// at least tile_max^2 (the pass also keeps two row tables there) and at most tile_max^3 (the
// tile). A cell that still has more takes the full-tile pass, so the bound needs no proof.
int candidate_capacity_sampled(const double* xi, int tm);

// the sampled bound depends on xi and tile_max only: kept per process
int candidate_capacity(const double* xi, int tm)
{
    static std::mutex mu;
    static std::vector<std::pair<std::array<double, 4>, int>> memo;
    const std::array<double, 4> key = {xi[0], xi[1], xi[2], (double)tm};
    std::lock_guard<std::mutex> lock(mu);
    for (const auto& kv : memo)
        if (kv.first == key) return kv.second;
    const int cap = candidate_capacity_sampled(xi, tm);
    memo.emplace_back(key, cap);
    return cap;
}

int candidate_capacity_sampled(const double* xi, int tm)
{
    uint64_t x = 0x9E3779B97F4A7C15ull;
    auto next = [&]() {   // xorshift64*, uniform in (0, 1)
        x ^= x >> 12;
        x ^= x << 25;
        x ^= x >> 27;
        return ((double)((x * 0x2545F4914F6CDD1Dull) >> 11) + 0.5) / 9007199254740992.0;
    };
    int most = 0;
    std::vector<int> lo_r, hi_r;
    for (int k = 0; k < 4096; ++k) {
        // uniform rotation from a unit quaternion (normal deviates by Box-Muller)
        double q[4];
        for (int a = 0; a < 4; a += 2) {
            const double r1 = std::sqrt(-2.0 * std::log(next())), t = 6.283185307179586 * next();
            q[a] = r1 * std::cos(t);
            q[a + 1] = r1 * std::sin(t);
        }
        const double qn = std::sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
        const double w = q[0] / qn, i = q[1] / qn, j = q[2] / qn, l = q[3] / qn;
        const double Q[9] = {1 - 2 * (j * j + l * l), 2 * (i * j - w * l), 2 * (i * l + w * j),
                             2 * (i * j + w * l), 1 - 2 * (i * i + l * l), 2 * (j * l - w * i),
                             2 * (i * l - w * j), 2 * (j * l + w * i), 1 - 2 * (i * i + j * j)};
        double R[3];
        for (int a = 0; a < 3; ++a) R[a] = 64.0 + next();
        int lo[3], sz[3];
        for (int a = 0; a < 3; ++a) {
            const double ext = std::fabs(Q[3 * a]) * xi[0] + std::fabs(Q[3 * a + 1]) * xi[1] +
                               std::fabs(Q[3 * a + 2]) * xi[2];
            lo[a] = (int)std::floor(R[a] - ext) - 1;
            sz[a] = (int)std::ceil(R[a] + ext) + 1 - lo[a] + 1;
        }
        if (sz[0] > tm || sz[1] > tm || sz[2] > tm) continue;
        const int rows = sz[1] * sz[2];
        lo_r.assign(rows, 0);
        hi_r.assign(rows, 0);
        const double X0 = R[0] - lo[0];
        for (int r = 0; r < rows; ++r) {
            const double dy = lo[1] + r % sz[1] - R[1], dz = lo[2] + r / sz[1] - R[2];
            double xa = -1e30, xb = 1e30;
            for (int a = 0; a < 3; ++a) {
                const double qa = Q[a], b = Q[3 + a] * dy + Q[6 + a] * dz;
                if (std::fabs(qa) > 1e-12) {
                    const double u0 = (-xi[a] - b) / qa, u1 = (xi[a] - b) / qa;
                    xa = std::max(xa, std::min(u0, u1));
                    xb = std::min(xb, std::max(u0, u1));
                } else if (std::fabs(b) >= xi[a] + 1e-9) {
                    xa = 1e30;
                }
            }
            lo_r[r] = sz[0];
            hi_r[r] = -1;
            if (xa <= xb) {
                lo_r[r] = std::max(0, (int)std::floor(X0 + xa - 1e-7) + 1);
                hi_r[r] = std::min(sz[0] - 1, (int)std::ceil(X0 + xb + 1e-7) - 1);
            }
        }
        int tot = 0;
        for (int r = 0; r < rows; ++r) {
            const int ty = r % sz[1], tz = r / sz[1];
            int a = sz[0], b = -1;
            if (lo_r[r] <= hi_r[r]) {
                a = lo_r[r] - 1;
                b = hi_r[r] + 1;
            }
            if (ty > 0) { a = std::min(a, lo_r[r - 1]); b = std::max(b, hi_r[r - 1]); }
            if (ty + 1 < sz[1]) { a = std::min(a, lo_r[r + 1]); b = std::max(b, hi_r[r + 1]); }
            if (tz > 0) { a = std::min(a, lo_r[r - sz[1]]); b = std::max(b, hi_r[r - sz[1]]); }
            if (tz + 1 < sz[2]) { a = std::min(a, lo_r[r + sz[1]]); b = std::max(b, hi_r[r + sz[1]]); }
            tot += std::max(0, std::min(b, sz[0] - 1) - std::max(a, 0) + 1);
        }
        most = std::max(most, tot);
    }
    const int cap = ((int)(1.2 * most) + 64 + 63) / 64 * 64;
    return std::min(std::max(cap, tm * tm), tm * tm * tm);
}

long long node_at(const lb_config& c, int x, int y, int z)
{
    if (x < 0 || x >= c.nx) { if (!c.periodic[0]) return -1; x = ((x % c.nx) + c.nx) % c.nx; }
    if (y < 0 || y >= c.ny) { if (!c.periodic[1]) return -1; y = ((y % c.ny) + c.ny) % c.ny; }
    if (z < 0 || z >= c.nz) { if (!c.periodic[2]) return -1; z = ((z % c.nz) + c.nz) % c.nz; }
    return (long long)x + (long long)c.nx * ((long long)y + (long long)c.ny * z);
}

std::string validate(const lb_config& c, int n_rbc)
{
    if (c.nx < 1 || c.ny < 1 || c.nz < 1) return "lattice dimensions must be positive";
    if (c.storage < LB_F64 || c.storage > LB_F16) return "unknown storage";
    if (!(c.tau0 > 0.5)) return "tau0 must exceed 1/2";
    if (c.forcing != 0 && c.forcing != 1) return "forcing must be 0 or 1";
    if (c.map_cap < 0 || c.map_cap > CAP_MAX) return "map_cap must be in 0..12";
    if (c.bf16_nearest != 0 && c.bf16_nearest != 1) return "bf16_nearest must be 0 or 1";
    for (int a = 0; a < 3; ++a)
        if (!std::isfinite(c.ext_force[a]) || !std::isfinite(c.ext_torque[a]))
            return "ext_force and ext_torque must be finite";
    if (c.storage == LB_F16) {
        // a power of two (scaling and unscaling are then exact in float) between 2^10, below
        // which slow flows underflow into FP16 subnormals without any error, and 2^40
        int e = 0;
        if (!(c.f16_scale > 0) || !std::isfinite(c.f16_scale) || std::frexp(c.f16_scale, &e) != 0.5 ||
            e < 11 || e > 41)
            return "f16_scale must be a power of two between 2^10 and 2^40";
    }
    if (c.cand_cap < 0) return "cand_cap must be non-negative";
    if (c.open_z && c.periodic[2]) return "open z faces need a non-periodic z axis";
    for (int a = 0; a < 3; ++a) {
        if (!std::isfinite(c.wall_u_lo[a]) || !std::isfinite(c.wall_u_hi[a]))
            return "wall velocities must be finite";
        if (c.open_z && (c.wall_u_lo[a] != 0.0 || c.wall_u_hi[a] != 0.0))
            return "moving walls and open z faces together are not supported";
    }
    if (c.open_z && c.nz < 3) return "open z faces need nz >= 3";
    if (c.open_z && (c.nx > 65535 || c.ny > 32767)) return "open z faces need nx < 65536 and ny < 32768";
    if (c.layout < 0 || c.layout > 2) return "layout must be 0 (automatic), 1 (dense) or 2 (compact)";
    {
        // The kernels address every per-node plane (populations, u, sigma, coverage counts
        // and slots) as a base plus a 32-bit byte offset node * element size: the padded plane
        // must stay below 4 GiB. FP64 planes hold 8-byte elements, the others at most 4.
        const long long N = (long long)c.nx * c.ny * c.nz;
        const long long elem = c.storage == LB_F64 ? 8 : 4;
        if ((N + 4096) * elem >= (1LL << 32))
            return c.storage == LB_F64 ? "at most 2^29 - 4096 nodes with FP64 storage (32-bit plane offsets)"
                                       : "at most 2^30 - 4096 nodes (32-bit plane offsets)";
    }
    if (n_rbc < 0) return "negative cell count";
    if (n_rbc >= (1 << 27)) return "at most 2^27 - 1 cells (coverage sort keys)";
    if (n_rbc > 0) {
        if (!(c.mass > 0) || !(c.inertia[0] > 0) || !(c.inertia[1] > 0) || !(c.inertia[2] > 0))
            return "mass and inertia must be positive";
        if (!(c.xi[0] > 0) || !(c.xi[1] > 0) || !(c.xi[2] > 0)) return "xi must be positive";
        if (!(c.axes[0] > 0) || !(c.axes[1] > 0) || !(c.axes[2] > 0)) return "axes must be positive";
        if (!(c.eps0 > 0)) return "eps0 must be positive";
        if (c.kappa < 0) return "kappa must be non-negative";
    }
    return "";
}

std::string build_geometry(const lb_config& c, const uint8_t* solid, int n_rbc, Geometry& g)
{
    g.nodes = (long long)c.nx * c.ny * c.nz;
    std::vector<uint32_t> dense((size_t)g.nodes, 0u);   // node words in lattice order
    std::vector<long long> plane_nodes;
    auto is_fluid = [&](int x, int y, int z) {
        long long m = node_at(c, x, y, z);
        return m >= 0 && !solid[m];
    };
    for (int z = 0; z < c.nz; ++z)
        for (int y = 0; y < c.ny; ++y)
            for (int x = 0; x < c.nx; ++x) {
                const long long n = (long long)x + (long long)c.nx * ((long long)y + (long long)c.ny * z);
                if (solid[n]) {
                    bool adj = false;
                    for (int p = 1; p < 19; ++p)
                        if (is_fluid(x + cx_(p), y + cy_(p), z + cz_(p))) adj = true;
                    if (adj) {
                        g.wall_xyz.push_back(x);
                        g.wall_xyz.push_back(y);
                        g.wall_xyz.push_back(z);
                    }
                    continue;
                }
                uint32_t w = NW_FLUID;
                double nv[3] = {0, 0, 0};
                bool wadj = false;
                for (int p = 1; p < 19; ++p) {
                    if (!is_fluid(x - cx_(p), y - cy_(p), z - cz_(p))) w |= 1u << p;
                    const long long m = node_at(c, x + cx_(p), y + cy_(p), z + cz_(p));
                    if (m >= 0 && solid[m]) {
                        wadj = true;
                        nv[0] += w_(p) * cx_(p);
                        nv[1] += w_(p) * cy_(p);
                        nv[2] += w_(p) * cz_(p);
                    }
                }
                if (wadj) {
                    w |= NW_WALLADJ;
                    const double len = std::sqrt(nv[0] * nv[0] + nv[1] * nv[1] + nv[2] * nv[2]);
                    g.wn_dense.push_back(n);
                    for (int a = 0; a < 3; ++a) g.wn_nrm.push_back(len > 0 ? nv[a] / len : 0.0);
                }
                if (c.open_z && (z == 0 || z == c.nz - 1)) {
                    w |= NW_OPEN;
                    plane_nodes.push_back(n);
                }
                // inner neighbour of an open-plane node (z = 1 above the inlet, z = nz - 2
                // below the outlet)
                if (c.open_z && ((z == 1 && !solid[n - (long long)c.nx * c.ny]) ||
                                 (z == c.nz - 2 && !solid[n + (long long)c.nx * c.ny])))
                    w |= NW_OPEN_INNER;
                dense[n] = w;
                g.n_fluid++;
            }
    // storage layout: the 64-node row segments that hold a fluid node decide between the dense
    // layout (every node stored, index x + nx (y + ny z)) and the compact one
    {
        const int nbx = (c.nx + 63) / 64;
        g.nbx = nbx;
        const long long ncol = (long long)nbx * c.ny * c.nz;
        std::vector<int> smap((size_t)ncol, -1);
        int active = 0;
        for (long long col = 0; col < ncol; ++col) {
            const long long row = col / nbx, x0 = 64 * (col - row * nbx);
            const long long n0 = row * c.nx;
            for (long long x = x0; x < std::min<long long>(c.nx, x0 + 64); ++x)
                if (dense[(size_t)(n0 + x)] & NW_FLUID) {
                    smap[(size_t)col] = active++;
                    break;
                }
        }
        g.compact = c.layout == 2 || (c.layout == 0 && active > 0 &&
                                      (double)active < COMPACT_MAX_FRACTION * (double)ncol);
        if (g.compact) {
            g.segmap.swap(smap);
            g.segs.assign((size_t)active * 4, 0);
            g.segnb.assign((size_t)active * 27, -1);
            for (long long col = 0; col < ncol; ++col) {
                const int sg = g.segmap[(size_t)col];
                if (sg < 0) continue;
                const long long row = col / nbx;
                const int x0 = (int)(64 * (col - row * nbx)), y = (int)(row % c.ny), z = (int)(row / c.ny);
                g.segs[4 * (size_t)sg + 0] = x0;
                g.segs[4 * (size_t)sg + 1] = y;
                g.segs[4 * (size_t)sg + 2] = z;
                // x of the neighbouring column segments: the node before x0, the first node past
                // the segment's last node (both wrapped on a periodic x axis, else outside)
                const int xl = x0 - 1, xr = std::min(x0 + 64, c.nx);
                const int xs[3] = {xl >= 0 ? xl : (c.periodic[0] ? c.nx - 1 : -1), x0,
                                   xr < c.nx ? xr : (c.periodic[0] ? 0 : -1)};
                for (int dz = -1; dz <= 1; ++dz)
                    for (int dy = -1; dy <= 1; ++dy)
                        for (int dx = -1; dx <= 1; ++dx) {
                            int Y = y + dy, Z = z + dz;
                            const int X = xs[dx + 1];
                            if (X < 0) continue;
                            if (Y < 0 || Y >= c.ny) {
                                if (!c.periodic[1]) continue;
                                Y = (Y + c.ny) % c.ny;
                            }
                            if (Z < 0 || Z >= c.nz) {
                                if (!c.periodic[2]) continue;
                                Z = (Z + c.nz) % c.nz;
                            }
                            g.segnb[27 * (size_t)sg + (dx + 1) + 3 * (dy + 1) + 9 * (dz + 1)] =
                                g.segmap[(size_t)((X >> 6) + (long long)nbx * (Y + (long long)c.ny * Z))];
                        }
            }
            g.N = 64LL * active;
            g.nodeword.assign((size_t)g.N, 0u);
            for (int sg = 0; sg < active; ++sg) {
                const int x0 = g.segs[4 * (size_t)sg], y = g.segs[4 * (size_t)sg + 1], z = g.segs[4 * (size_t)sg + 2];
                const long long n0 = (long long)c.nx * ((long long)y + (long long)c.ny * z);
                for (int x = x0; x < std::min(c.nx, x0 + 64); ++x)
                    g.nodeword[64 * (size_t)sg + (x - x0)] = dense[(size_t)(n0 + x)];
            }
        } else {
            g.N = g.nodes;
            g.nodeword.swap(dense);
        }
        // plane stride: a multiple of 256 B plus an odd number of 256-B blocks, so that planes
        // read together do not start at power-of-two distances (HBM channel spread)
        const long long G = 256 / storage_bytes(c.storage);
        g.ld = (g.N + 2 * G - 1) / (2 * G) * (2 * G) + G;
        g.wn_node.resize(g.wn_dense.size());
        for (size_t k = 0; k < g.wn_dense.size(); ++k) g.wn_node[k] = g.store_of(g.wn_dense[k], c.nx, c.ny);
        const long long nxy = (long long)c.nx * c.ny;
        for (long long n : plane_nodes) {
            const long long z = n / nxy, rem = n - z * nxy, y = rem / c.nx, x = rem - y * c.nx;
            const long long ni = z == 0 ? n + nxy : n - nxy;
            const long long ki = solid[ni] ? -1 : g.store_of(ni, c.nx, c.ny);
            g.planes.insert(g.planes.end(), {(int)g.store_of(n, c.nx, c.ny), (int)ki, (int)(x | (y << 16)), (int)z});
        }
    }
    // cell grid: r_c bounds every Gay-Berne cut-off (cell-cell and cell-wall)
    const double amax = std::max(c.axes[0], std::max(c.axes[1], c.axes[2]));
    const double amin = std::min(c.axes[0], std::min(c.axes[1], c.axes[2]));
    const double sm = std::sqrt(4.0 * amin * amin);
    const double shift = std::pow(2.0, 1.0 / 6.0) - 1.0;
    const double rc_cc = std::sqrt(4.0 * amax * amax) + shift * sm;
    const double rc_cw = std::sqrt(2.0 * (amax * amax + c.a_wall * c.a_wall)) + shift * c.sigmin_wall;
    g.rc = std::max(rc_cc, rc_cw);
    const int L[3] = {c.nx, c.ny, c.nz};
    for (int a = 0; a < 3; ++a) {
        int m = (int)std::floor(L[a] / g.rc);
        if (m < 1) m = 1;
        g.ncell[a] = m;
        g.cedge[a] = (double)L[a] / m;
    }
    // wall points in a grid of their own: its edge bounds only the cell-wall cut-off, so the
    // 27 neighbour cells of a cell centre hold about three times fewer points than the cell
    // grid's would
    for (int a = 0; a < 3; ++a) {
        int m = (int)std::floor(L[a] / rc_cw);
        if (m < 1) m = 1;
        g.wncell[a] = m;
        g.wcedge[a] = (double)L[a] / m;
    }
    const int nc = g.wncell[0] * g.wncell[1] * g.wncell[2];
    const int nwall = (int)g.wall_xyz.size() / 3;
    std::vector<int> cnt(nc, 0), wc(nwall);
    auto cell_of = [&](double v, int a) {
        int q = (int)std::floor(v / g.wcedge[a]);
        return std::min(std::max(q, 0), g.wncell[a] - 1);
    };
    for (int k = 0; k < nwall; ++k) {
        wc[k] = cell_of(g.wall_xyz[3 * k], 0) +
                g.wncell[0] * (cell_of(g.wall_xyz[3 * k + 1], 1) + g.wncell[1] * cell_of(g.wall_xyz[3 * k + 2], 2));
        cnt[wc[k]]++;
    }
    g.wcell_off.assign(nc + 1, 0);
    for (int q = 0; q < nc; ++q) g.wcell_off[q + 1] = g.wcell_off[q] + cnt[q];
    g.wcell_ids.assign(std::max(nwall, 1), 0);
    std::fill(cnt.begin(), cnt.end(), 0);
    for (int k = 0; k < nwall; ++k) g.wcell_ids[g.wcell_off[wc[k]] + cnt[wc[k]]++] = k;
    // support tile bound (support box plus one node on each side, plus rounding)
    const double r = std::sqrt(c.xi[0] * c.xi[0] + c.xi[1] * c.xi[1] + c.xi[2] * c.xi[2]);
    g.tile_max = 2 * (int)std::ceil(r) + 5;
    if (n_rbc > 0) {
        // The full-tile map pass keeps tile_max^3 kernel values, a flag byte each and a
        // 2-byte position list in LDS, next to about 3.5 KiB of fixed arrays; the
        // one-wavefront pass keeps cand_cap candidates. Both within 64 KiB per workgroup.
        g.cand_cap = candidate_capacity(c.xi, g.tile_max);
        // test hook: a smaller capacity sends more cells to the full-tile pass
        if (c.cand_cap > 0)
            g.cand_cap = std::min(std::max(c.cand_cap, g.tile_max * g.tile_max),
                                  g.tile_max * g.tile_max * g.tile_max);
        // Coverage entries per cell: covered nodes lie within one node (on each axis) of the
        // support box 2 xi; each such lattice node's unit cube lies in the box grown by 1.5 on
        // each axis, which lies in the box grown by the ball of radius 1.5 sqrt(3). Steiner's
        // formula bounds that volume, hence the count; the power of two above it is reserved.
        {
            const double a = 2 * c.xi[0], b = 2 * c.xi[1], d = 2 * c.xi[2], rr = 1.5 * std::sqrt(3.0);
            const double vol = a * b * d + 2 * (a * b + b * d + d * a) * rr + M_PI * (a + b + d) * rr * rr +
                               4.0 / 3.0 * M_PI * rr * rr * rr;
            g.ent_shift = 0;
            while ((double)(1 << g.ent_shift) < vol) ++g.ent_shift;
            if (((long long)n_rbc << g.ent_shift) >= (1ll << 31))
                return "too many cells for 32-bit coverage entries at this support size";
        }
        const int rb = real_bytes(c.storage);
        if (g.tile_max > 20 || map_couple_tile_lds(g.tile_max, rb) + 4096 > 65536 ||
            map_couple_lds(g.tile_max, g.cand_cap, rb) > 65536)
            return "shape-function support too large for the LDS tile";
        for (int a = 0; a < 3; ++a)
            if (c.periodic[a] && L[a] < g.tile_max + 2) return "periodic axis shorter than a support tile";
        for (int a = 0; a < 3; ++a)
            if (c.periodic[a] && L[a] <= 2.0 * g.rc) return "periodic axis shorter than twice the cut-off";
    }
    return "";
}

// ---- arena layout --------------------------------------------------------------------------
struct Layout {
    size_t fA, fB, u, sig, gdbg, tdbg, nodeword, map_ids[2], map_vals[2], cnt[2], ovf, st, cp, gat, cellid, cell_cnt, cell_off,
        cell_part, cell_ids, wall_xyz, wcell_off, wcell_ids, wn_node, wn_nrm, wss, wss_acc, planes, segs, segnb,
        segmap, partials, obs_out, err, step_ctr, slot, total;
};

Layout layout(const lb_config& c, const Geometry& g, int n_rbc)
{
    Layout L{};
    const size_t ss = storage_bytes(c.storage), rs = real_bytes(c.storage);
    const int cap = c.map_cap == 0 ? CAP_MAX : c.map_cap;
    const size_t nc = (size_t)g.ncell[0] * g.ncell[1] * g.ncell[2];
    const size_t nwall = g.wall_xyz.size() / 3, nwn = g.wn_node.size();
    const size_t ld = (size_t)g.ld;
    size_t o = 0;
    auto take = [&](size_t bytes) {
        size_t at = o;
        o += up(std::max<size_t>(bytes, 1));
        return at;
    };
    L.fA = take(19 * ld * ss);
    L.fB = take(19 * ld * ss);
    const size_t fs = field_bytes(c.storage);
    L.u = take(vel_stride(c.storage) * ld * fs);
    L.sig = take(6 * ld * fs);
    L.gdbg = take(3 * ld * rs);
    L.tdbg = take(ld * rs);
    L.nodeword = take(ld * 4);
    // two coverage sets, alternating with the step's parity
    for (int p = 0; p < 2; ++p) {
        L.map_ids[p] = take(n_rbc > 0 ? (size_t)cap * ld * 4 : 4);
        // coverage entries: four values in the compute precision, or in 16 bits for the
        // 16-bit storages
        L.map_vals[p] = take(n_rbc > 0 ? ((size_t)n_rbc << g.ent_shift) * 4 * (fs == 2 ? 2 : rs) : 4);
        L.cnt[p] = take(ld * 4);   // read at every fluid node, with or without cells
    }
    L.ovf = take(((size_t)n_rbc + 1) * 4);
    L.st = take(n_rbc * sizeof(RbcState));
    L.cp = take(n_rbc * sizeof(RbcCouple));
    L.gat = take(n_rbc * (rs == 8 ? sizeof(Gather<double>) : sizeof(Gather<float>)));
    L.cellid = take(n_rbc * 4);
    L.cell_cnt = take(nc * 4);
    L.cell_off = take((nc + 1) * 4);
    L.cell_part = take((nc + CELL_SCAN_CHUNK - 1) / CELL_SCAN_CHUNK * 4);
    L.cell_ids = take(n_rbc * 4);
    L.wall_xyz = take(nwall * 3 * 4);
    L.wcell_off = take(((size_t)g.wncell[0] * g.wncell[1] * g.wncell[2] + 1) * 4);
    L.wcell_ids = take(std::max<size_t>(nwall, 1) * 4);
    L.wn_node = take(nwn * 8);
    L.wn_nrm = take(nwn * 3 * 8);
    L.wss = take(nwn * 8);
    L.wss_acc = take(nwn * 8);
    L.planes = take(g.planes.size() * 4);
    L.segs = take(g.segs.size() * 4);
    L.segnb = take(g.segnb.size() * 4);
    L.segmap = take(g.segmap.size() * 4);
    L.partials = take(6 * OBS_BLOCKS * 8);
    L.obs_out = take(8 * 8);
    L.err = take(4);
    L.step_ctr = take(8);
    L.slot = take(sizeof(SlotDesc));
    L.total = o;
    return L;
}

}  // namespace

// ---- scratch of rbc_collide_static, the entry point that allocates nothing ----------------------
// Its cell list lives in this file-scope device array instead of the context's arena: one copy
// per GPU, held until the process ends. Host code never uses the array's name as an address:
// lb_init resolves the array's device address once per device (with that device current) and
// every use goes through that pointer.
constexpr int STATIC_MAX_CELLS = 1 << 18;    // 262,144 cells
constexpr int STATIC_MAX_GRID = 1 << 20;     // 1,048,576 grid cells of the cell list
constexpr size_t STATIC_SCRATCH_INTS = 2 * (size_t)STATIC_MAX_CELLS + 2 * (size_t)STATIC_MAX_GRID + 1 +
                                       (STATIC_MAX_GRID + CELL_SCAN_CHUNK - 1) / CELL_SCAN_CHUNK;
static __device__ __align__(256) int scratch[STATIC_SCRATCH_INTS];

namespace {
constexpr int SCRATCH_MAX_DEVICES = 64;
std::mutex g_scratch_mu;
int* g_scratch_ptr[SCRATCH_MAX_DEVICES] = {};

// device address of `scratch` on device dev (which must be current)
hipError_t resolve_scratch(int dev)
{
    if (dev < 0 || dev >= SCRATCH_MAX_DEVICES) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch_ptr[dev]) return hipSuccess;
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e == hipSuccess) g_scratch_ptr[dev] = static_cast<int*>(p);
    return e;
}
}  // namespace

struct lb_ctx_s {
    lb_config cfg;
    KParams kp;
    Geometry geo;
    unsigned long long geo_hash = 0;
    int device = 0;   // the GPU current at lb_init
    Layout lay;
    hipStream_t stream = nullptr;
    // Side stream (default priority) for the cells' own work, for large cell counts: the
    // Gay-Berne forces (independent of the map pass), then, once the map pass is done, the
    // kick and, within one lb_step call, the next step's first half and cell list, all
    // overlapping the stream-collide. Events order the two streams.
    hipStream_t side = nullptr;
    bool side_owned = false;   // created by lb_init (else the caller's, from lb_set_side_stream)
    hipEvent_t ev_cells = nullptr, ev_gb = nullptr, ev_map = nullptr;
    // the current step's first half, cell list and Gay-Berne are already on the side stream
    bool cells_ahead = false;
    char* base = nullptr;
    void *fA = nullptr, *fB = nullptr;
    // per coverage set: counts possibly nonzero (left by rbc_couple, or by a step whose
    // stream-collide could not clear them); cleared before that set's next map pass
    bool dirty[2] = {false, false};
    // the set the last map pass filled (rbc_get_map and the spread probe read it)
    int map_parity = 0;
    CellBuffers cb{};
    long long step = 0;
    int nrbc = 0;
    bool poisoned = false;
    unsigned fault = 0;
    int wss_on = 0;
    long long wss_count = 0;
    std::string last_error;
    // timing of the stream-collide kernel and of whole steps
    bool timing = false;
    std::vector<hipEvent_t> ev_pool;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> sc_pairs, map_pairs;
    hipEvent_t step_t0 = nullptr, step_t1 = nullptr;
    int timed_steps = 0;
    bool step_t0_set = false;

    template <typename T>
    T* at(size_t off) { return reinterpret_cast<T*>(base + off); }
    // the cell buffers with coverage set p (the fused launches use set 0, written at init)
    CellBuffers par(int p)
    {
        CellBuffers b = cb;
        b.map_ids = at<int>(lay.map_ids[p]);
        b.map_vals = at<void>(lay.map_vals[p]);
        b.cnt = at<uint32_t>(lay.cnt[p]);
        return b;
    }
    // stored segments of the compact layout (0 in the dense one)
    int nseg() const { return (int)(geo.segs.size() / 4); }
    // 0 while the current populations are in buffer A, 1 in buffer B (flips every step)
    int ab_parity() { return fA == at<void>(lay.fA) ? 0 : 1; }
};

namespace {

// cell count from which a context forks the map-independent work onto a side stream
constexpr int SIDE_STREAM_MIN_CELLS = 2048;

void release_side(lb_ctx c)
{
    if (c->side) (void)hipStreamSynchronize(c->side);
    for (hipEvent_t* ev : {&c->ev_cells, &c->ev_gb, &c->ev_map})
        if (*ev) {
            (void)hipEventDestroy(*ev);
            *ev = nullptr;
        }
    if (c->side && c->side_owned) (void)hipStreamDestroy(c->side);
    c->side = nullptr;
    c->side_owned = false;
}

// message of the last lb_init / lb_query_footprint failure (no context exists then)
std::string g_init_error;

lb_status fail(lb_ctx c, lb_status s, const std::string& msg)
{
    if (c) c->last_error = msg;
    else g_init_error = msg;
    return s;
}

lb_status init_fail(lb_ctx c, lb_status s, const std::string& msg)
{
    delete c;
    g_init_error = msg;
    return s;
}

#define HIPCHK(ctx, expr)                                                                        \
    do {                                                                                         \
        hipError_t e_ = (expr);                                                                  \
        if (e_ != hipSuccess)                                                                    \
            return fail(ctx, LB_EHIP, std::string(#expr) + ": " + hipGetErrorString(e_));       \
    } while (0)

// dispatch on the storage type
template <typename F>
void with_types(int storage, F&& f)
{
    switch (storage) {
    case LB_F64: f((double*)nullptr, (double*)nullptr); break;
    case LB_F32: f((float*)nullptr, (float*)nullptr); break;
    case LB_BF16: f((bf16_t*)nullptr, (float*)nullptr); break;
    default: f((_Float16*)nullptr, (float*)nullptr); break;
    }
}

// host conversions of one stored population value to/from the shifted float value
double load_stored(const void* p, size_t i, int storage, double inv)
{
    switch (storage) {
    case LB_F64: return ((const double*)p)[i];
    case LB_F32: return ((const float*)p)[i];
    case LB_BF16: {
        uint32_t u = (uint32_t)((const uint16_t*)p)[i] << 16;
        float f;
        std::memcpy(&f, &u, 4);
        return f;
    }
    default: return (double)(float)((const _Float16*)p)[i] * inv;
    }
}

void store_value(void* p, size_t i, int storage, double v, double scale)
{
    switch (storage) {
    case LB_F64: ((double*)p)[i] = v; break;
    case LB_F32: ((float*)p)[i] = (float)v; break;
    case LB_BF16: {
        float f = (float)v;
        uint32_t u;
        std::memcpy(&u, &f, 4);
        uint16_t r = ((u & 0x7f800000u) == 0x7f800000u && (u & 0x007fffffu))
                         ? 0x7fc0
                         : (uint16_t)((u + 0x7fffu + ((u >> 16) & 1u)) >> 16);
        ((uint16_t*)p)[i] = r;
        break;
    }
    default: ((_Float16*)p)[i] = (_Float16)(float)(v * scale); break;
    }
}

double load_real(const void* p, size_t i, int storage)
{
    return storage == LB_F64 ? ((const double*)p)[i] : (double)((const float*)p)[i];
}
void store_real(void* p, size_t i, int storage, double v)
{
    if (storage == LB_F64) ((double*)p)[i] = v;
    else ((float*)p)[i] = (float)v;
}
// one element of u or sigma (the same roundings as the device's field stores)
double load_field(const void* p, size_t i, int storage)
{
    if (field_bytes(storage) != 2) return load_real(p, i, storage);
    return load_stored(p, i, storage, 1.0 / FIELD16_SCALE_HOST);
}
void store_field(void* p, size_t i, int storage, double v)
{
    if (field_bytes(storage) != 2) store_real(p, i, storage, v);
    else store_value(p, i, storage, v, FIELD16_SCALE_HOST);
}

lb_status check_fault(lb_ctx c)
{
    unsigned e = 0;
    HIPCHK(c, hipStreamSynchronize(c->stream));
    HIPCHK(c, hipMemcpy(&e, c->cb.err, 4, hipMemcpyDeviceToHost));
    if (e) {
        c->fault |= e;
        c->poisoned = true;
        if (e & ERR_OVERLAP) return fail(c, LB_EOVERLAP, "Gay-Berne pair at rho <= 0 (singular overlap)");
        if (e & ERR_UNSTABLE) return fail(c, LB_EUNSTABLE, "non-finite or non-positive density, or |u| > 0.3");
        return fail(c, LB_ECAPACITY, "coverage slots per node or support tile exhausted");
    }
    return LB_OK;
}

// cell list, coverage map and interpolation onto the cells (one pass per cell), into the
// coverage set of the next step
template <typename RT>
void enqueue_cells_map_couple(lb_ctx c)
{
    hipStream_t s = c->stream;
    const int p = (int)(c->step & 1);
    const CellBuffers b = c->par(p);
    launch_cell_list(b, c->kp, s);
    launch_clear_counts(b.cnt, c->kp.N, b.ovf, s);
    launch_map_couple<RT>(b, c->kp, s);
    c->dirty[p] = true;
    c->map_parity = p;
}

// One step. With a side stream the cells' work runs there: after the map pass, the kick and,
// unless this is the last step of the call (`last`), the next step's first half, cell list
// and Gay-Berne forces, all while the stream-collide runs; the map pass waits for the cell
// list. The last step joins the side stream back, so a call leaves whole steps behind.
void enqueue_step(lb_ctx c, bool last)
{
    hipStream_t s = c->stream;
    const KParams& kp = c->kp;
    c->cb.u = c->at<void>(c->lay.u);
    c->cb.sig = c->at<void>(c->lay.sig);
    // this step's coverage set
    const int p = (int)(c->step & 1);
    const CellBuffers b = c->par(p);
    // The stream-collide clears the counts of the set it reads, except at the open planes and
    // their inner neighbours, whose counts the boundary kernel reads after it and then
    // clears. With nz = 3 both planes extrapolate from the same layer (two readers), so the
    // counts stay and are cleared before that set's next map pass, as after rbc_couple.
    const bool sc_clears = c->geo.planes.empty() || c->cfg.nz > 3;
    with_types(c->cfg.storage, [&](auto* sp, auto* rp) {
        using ST = std::remove_pointer_t<decltype(sp)>;
        using RT = std::remove_pointer_t<decltype(rp)>;
        const bool forked = c->nrbc > 0 && c->side;
        if (c->nrbc > 0) {
            // rb1 + cell list, map + interpolation (which writes F^hyd, T^hyd and the gather
            // records), Gay-Berne, kick
            if (!forked) {
                launch_rb1_cell_list(c->cb, kp, s);
            } else if (!c->cells_ahead) {
                launch_rb1_cell_list(c->cb, kp, s);
                (void)hipEventRecord(c->ev_cells, s);
                (void)hipStreamWaitEvent(c->side, c->ev_cells, 0);
                launch_gay_berne(c->cb, kp, c->side);
            } else {
                (void)hipStreamWaitEvent(s, c->ev_cells, 0);
            }
            if (c->dirty[p])
                launch_clear_counts(b.cnt, kp.N, b.ovf, s);
            hipEvent_t m0 = nullptr, m1 = nullptr;
            if (c->timing && (int)c->map_pairs.size() < MAX_TIMED && c->ev_pool.size() >= 4) {
                m0 = c->ev_pool.back();
                c->ev_pool.pop_back();
                m1 = c->ev_pool.back();
                c->ev_pool.pop_back();
                (void)hipEventRecord(m0, s);
            }
            launch_map_couple<RT>(b, kp, s);
            if (m0) {
                (void)hipEventRecord(m1, s);
                c->map_pairs.emplace_back(m0, m1);
            }
            c->map_parity = p;
            if (!forked) {
                launch_gay_berne(c->cb, kp, s);
                launch_rb_second_half(c->cb, kp, s);
            } else {
                (void)hipEventRecord(c->ev_map, s);
                (void)hipStreamWaitEvent(c->side, c->ev_map, 0);
                launch_rb_second_half(c->cb, kp, c->side);
                c->cells_ahead = !last;
                if (!last) {
                    launch_rb1_cell_list(c->cb, kp, c->side);
                    (void)hipEventRecord(c->ev_cells, c->side);
                    launch_gay_berne(c->cb, kp, c->side);
                } else {
                    (void)hipEventRecord(c->ev_gb, c->side);
                }
            }
        }
        hipEvent_t e0 = nullptr, e1 = nullptr;
        if (c->timing && (int)c->sc_pairs.size() < MAX_TIMED && c->ev_pool.size() >= 2) {
            e0 = c->ev_pool.back();
            c->ev_pool.pop_back();
            e1 = c->ev_pool.back();
            c->ev_pool.pop_back();
            (void)hipEventRecord(e0, s);
        }
        launch_stream_collide<ST, RT>(c->fA, c->fB, b.nodeword, b.map_ids, b.map_vals, b.cnt,
                                      c->cb.gat, c->at<void>(c->lay.u), c->at<void>(c->lay.sig), kp,
                                      c->cb.err, sc_clears && c->nrbc > 0, c->cb.tab, c->nseg(), c->cb.step_ctr,
                                      c->ab_parity(), s);
        if (e0) {
            (void)hipEventRecord(e1, s);
            c->sc_pairs.emplace_back(e0, e1);
        }
        if (!c->geo.planes.empty())
            launch_open_bc<ST, RT>(c->fA, c->fB, b.nodeword, c->at<int4>(c->lay.planes),
                                   (int)c->geo.planes.size() / 4, b.map_ids, b.map_vals, b.cnt, c->cb.gat,
                                   c->at<void>(c->lay.u), c->at<void>(c->lay.sig), kp, c->cb.tab,
                                   sc_clears && c->nrbc > 0, c->cb.step_ctr, c->ab_parity(), s);
        if (c->wss_on)
            launch_wss<RT>(c->at<void>(c->lay.sig), c->at<long long>(c->lay.wn_node),
                           c->at<double>(c->lay.wn_nrm), (int)c->geo.wn_node.size(), kp, nullptr,
                           c->at<double>(c->lay.wss_acc), 1, s);
        if (forked && last) (void)hipStreamWaitEvent(s, c->ev_gb, 0);
    });
    if (c->wss_on) c->wss_count++;
    // the stream-collide (and the boundary kernel) cleared the counts of this step's set
    c->dirty[p] = c->nrbc > 0 && !sc_clears;
    std::swap(c->fA, c->fB);
    c->step++;
}

// Contexts whose steps one fused launch per stage can carry together: the same stream and
// storage type, no open boundary, no WSS accumulation, no kernel timing.
bool fusable(lb_ctx c, lb_ctx first)
{
    return c->stream == first->stream && c->cfg.storage == first->cfg.storage && c->geo.planes.empty() &&
           !c->wss_on && !c->timing;
}

// A second stream (default priority) per device for the fused batches' cell work, as the side
// stream of a single context: after the map passes, the Gay-Berne stage and the kick (it needs
// both) run beside the stream-collide; the next step's first stage waits for the kick. Events
// fork and join it. Created on the first batch call of a device (never during a capture); the
// mutex keeps one host thread at a time enqueuing with the shared events. A batch call ends
// joined.
struct FusedSide {
    std::mutex mu;
    hipStream_t side = nullptr;
    hipEvent_t mapped = nullptr, join = nullptr;
    bool ready = false;
};

FusedSide* fused_side(int dev)
{
    static std::mutex create_mu;
    static FusedSide table[SCRATCH_MAX_DEVICES];
    if (dev < 0 || dev >= SCRATCH_MAX_DEVICES) return nullptr;
    std::lock_guard<std::mutex> lock(create_mu);
    FusedSide& f = table[dev];
    if (!f.ready) {
        int cur = 0;
        if (hipGetDevice(&cur) != hipSuccess || cur != dev) return nullptr;
        if (hipStreamCreateWithFlags(&f.side, hipStreamNonBlocking) != hipSuccess) return nullptr;
        if (hipEventCreateWithFlags(&f.mapped, hipEventDisableTiming) != hipSuccess ||
            hipEventCreateWithFlags(&f.join, hipEventDisableTiming) != hipSuccess)
            return nullptr;
        f.ready = true;
    }
    return &f;
}

// one step of n contexts (n <= FUSE_MAX): rb1 + binning, scan, scatter, sort, count clearing,
// map + interpolation (and the overflow pass), Gay-Berne, second half, stream-collide; each stage
// is one launch over all contexts. With fs, the Gay-Berne stage and the kick run on its stream.
void enqueue_fused_step(lb_ctx* cs, int n, FusedSide* fs)
{
    hipStream_t s = cs[0]->stream;
    // the previous step's kick (a no-op wait at the first step of a batch: already joined)
    if (fs) (void)hipStreamWaitEvent(s, fs->join, 0);
    FusedArgs fa;
    fa.n = n;
    fa.field16 = cs[0]->kp.field16;
    fa.parity = 0;
    size_t lds_map = 0, lds_tile = 0;
    for (int i = 0; i < n; ++i) {
        lb_ctx c = cs[i];
        fa.slot[i] = c->at<SlotDesc>(c->lay.slot);
        if (c->fA != c->at<void>(c->lay.fA)) fa.parity |= 1ull << i;
        const int rb = real_bytes(c->cfg.storage);
        if (c->nrbc > 0) {
            lds_map = std::max(lds_map, map_couple_lds(c->kp.tile_max, c->kp.cand_cap, rb));
            lds_tile = std::max(lds_tile, map_couple_tile_lds(c->kp.tile_max, rb));
        }
    }
    auto starts = [&](int stage) {
        int tot = 0;
        for (int i = 0; i < n; ++i) {
            fa.start[i] = tot;
            tot += fused_blocks(cs[i]->kp, stage);
        }
        fa.start[n] = tot;
    };
    with_types(cs[0]->cfg.storage, [&](auto* sp, auto* rp) {
        using ST = std::remove_pointer_t<decltype(sp)>;
        using RT = std::remove_pointer_t<decltype(rp)>;
        for (int stage : {FS_CELLS_A, FS_SCAN, FS_SCATTER, FS_SORT}) {
            starts(stage);
            launch_fused_cells<RT>(fa, stage, 0, s);
        }
        // counts left by a single-context step are cleared here; otherwise the previous fused
        // stream-collide has cleared them
        {
            int tot = 0;
            for (int i = 0; i < n; ++i) {
                fa.start[i] = tot;
                tot += cs[i]->dirty[0] ? fused_blocks(cs[i]->kp, FS_CLEAR) : 0;
            }
            fa.start[n] = tot;
            launch_fused_lattice<ST, RT>(fa, FS_CLEAR, s);
        }
        starts(FS_MAP);
        launch_fused_cells<RT>(fa, FS_MAP, lds_map, s);
        starts(FS_MAP_TILE);
        launch_fused_cells<RT>(fa, FS_MAP_TILE, lds_tile, s);
        if (fs) {
            // the Gay-Berne stage and the kick run beside the stream-collide (beside the map
            // passes they held the overflow pass's blocks back)
            (void)hipEventRecord(fs->mapped, s);
            (void)hipStreamWaitEvent(fs->side, fs->mapped, 0);
            starts(FS_GB);
            launch_fused_cells<RT>(fa, FS_GB, 0, fs->side);
            starts(FS_RB2);
            launch_fused_cells<RT>(fa, FS_RB2, 0, fs->side);
            (void)hipEventRecord(fs->join, fs->side);
        } else {
            starts(FS_GB);
            launch_fused_cells<RT>(fa, FS_GB, 0, s);
            starts(FS_RB2);
            launch_fused_cells<RT>(fa, FS_RB2, 0, s);
        }
        starts(FS_STREAM);
        launch_fused_lattice<ST, RT>(fa, FS_STREAM, s);
    });
    for (int i = 0; i < n; ++i) {
        std::swap(cs[i]->fA, cs[i]->fB);
        cs[i]->step++;
        cs[i]->dirty[0] = false;
        cs[i]->map_parity = 0;
    }
}

}  // namespace

extern "C" {

lb_status lb_query_footprint(const lb_config* cfg, const uint8_t* solid, int n_rbc, size_t* bytes)
{
    if (!cfg || !solid || !bytes) return fail(nullptr, LB_EINVAL, "null argument");
    std::string msg = validate(*cfg, n_rbc);
    Geometry g;
    if (msg.empty()) msg = build_geometry(*cfg, solid, n_rbc, g);
    if (!msg.empty()) return fail(nullptr, LB_EINVAL, msg);
    *bytes = layout(*cfg, g, n_rbc).total;
    return LB_OK;
}

lb_status lb_init(const lb_config* cfg, const uint8_t* solid, const lb_rbc* cells, int n_rbc,
                  void* arena, size_t arena_bytes, void* hip_stream, lb_ctx* out)
{
    if (!cfg || !solid || !out || (n_rbc > 0 && !cells) || !arena) return LB_EINVAL;
    *out = nullptr;
    lb_ctx c = new lb_ctx_s();
    c->cfg = *cfg;
    if (c->cfg.map_cap == 0) c->cfg.map_cap = CAP_MAX;
    std::string msg = validate(c->cfg, n_rbc);
    if (msg.empty()) msg = build_geometry(c->cfg, solid, n_rbc, c->geo);
    if (!msg.empty()) return init_fail(c, LB_EINVAL, msg);
    if ((reinterpret_cast<uintptr_t>(arena) % ALIGN) != 0)
        return init_fail(c, LB_EINVAL, "arena must be 256-byte aligned");
    c->lay = layout(c->cfg, c->geo, n_rbc);
    c->geo_hash = geometry_hash(c->geo);
    if (arena_bytes < c->lay.total) return init_fail(c, LB_ENOMEM, "arena smaller than the footprint");
    c->stream = (hipStream_t)hip_stream;
    c->base = (char*)arena;
    {
        hipError_t e0 = hipGetDevice(&c->device);
        if (e0 == hipSuccess) e0 = resolve_scratch(c->device);
        if (e0 != hipSuccess)
            return init_fail(c, LB_EHIP, std::string("static scratch address: ") + hipGetErrorString(e0));
    }
    c->nrbc = n_rbc;
    const lb_config& C = c->cfg;
    const Geometry& g = c->geo;
    KParams& kp = c->kp;
    std::memset(&kp, 0, sizeof kp);
    kp.nx = C.nx; kp.ny = C.ny; kp.nz = C.nz;
    for (int a = 0; a < 3; ++a) kp.per[a] = C.periodic[a] ? 1 : 0;
    kp.N = g.N;
    kp.ld = g.ld;
    kp.nbx = g.nbx;
    kp.compact = g.compact ? 1 : 0;
    kp.forcing = C.forcing;
    kp.cap = C.map_cap;
    kp.tau0 = C.tau0; kp.delta = C.delta_visc; kp.kappa = C.kappa;
    kp.kappa_int = (C.kappa == std::floor(C.kappa) && C.kappa >= 0 && C.kappa <= 64) ? (int)C.kappa : -1;
    for (int a = 0; a < 3; ++a) {
        kp.gext[a] = C.g_ext[a];
        kp.inertia[a] = C.inertia[a];
        kp.xi[a] = C.xi[a];
        kp.axes[a] = C.axes[a];
        kp.ncell[a] = g.ncell[a];
        kp.cedge[a] = g.cedge[a];
        kp.wncell[a] = g.wncell[a];
        kp.wcedge[a] = g.wcedge[a];
    }
    kp.gammaT = C.gammaT; kp.gammaR = C.gammaR; kp.alpha = C.alpha; kp.mass = C.mass;
    kp.vort_scale = C.vort_scale;
    for (int a = 0; a < 3; ++a) {
        kp.ext_force[a] = C.ext_force[a];
        kp.ext_torque[a] = C.ext_torque[a];
    }
    kp.eps0 = C.eps0; kp.a_wall = C.a_wall; kp.sigmin_wall = C.sigmin_wall;
    kp.wall_particles = C.wall_particles;
    kp.open_z = C.open_z; kp.rho_in = C.rho_in; kp.rho_out = C.rho_out;
    kp.f16_scale = C.storage == LB_F16 ? (float)C.f16_scale : 1.0f;
    kp.f16_inv = 1.0f / kp.f16_scale;
    kp.nrbc = n_rbc;
    kp.rc = g.rc;
    {
        const double amax = std::max(C.axes[0], std::max(C.axes[1], C.axes[2]));
        const double amin = std::min(C.axes[0], std::min(C.axes[1], C.axes[2]));
        const double shift = std::pow(2.0, 1.0 / 6.0) - 1.0;
        kp.rc_pair = std::sqrt(4.0 * amax * amax) + shift * std::sqrt(4.0 * amin * amin);
        kp.rc_wall = std::sqrt(2.0 * (amax * amax + C.a_wall * C.a_wall)) + shift * C.sigmin_wall;
    }
    kp.tile_max = g.tile_max;
    kp.cand_cap = g.cand_cap;
    kp.bf16_sr = C.storage == LB_BF16 && !C.bf16_nearest ? 1 : 0;
    kp.field16 = C.storage == LB_BF16 ? 1 : (C.storage == LB_F16 ? 2 : 0);
    kp.moving_walls = 0;
    for (int a = 0; a < 3; ++a) {
        kp.uw_lo[a] = C.wall_u_lo[a];
        kp.uw_hi[a] = C.wall_u_hi[a];
        if (C.wall_u_lo[a] != 0.0 || C.wall_u_hi[a] != 0.0) kp.moving_walls = 1;
    }
    kp.ent_shift = g.ent_shift;

    const Layout& L = c->lay;
    c->fA = c->at<void>(L.fA);
    c->fB = c->at<void>(L.fB);
    CellBuffers& b = c->cb;
    b.st = c->at<RbcState>(L.st);
    b.cp = c->at<RbcCouple>(L.cp);
    b.gat = c->at<void>(L.gat);
    b.cellid = c->at<int>(L.cellid);
    b.cell_cnt = c->at<int>(L.cell_cnt);
    b.cell_off = c->at<int>(L.cell_off);
    b.cell_part = c->at<int>(L.cell_part);
    b.cell_ids = c->at<int>(L.cell_ids);
    b.wall_xyz = c->at<int>(L.wall_xyz);
    b.wcell_off = c->at<int>(L.wcell_off);
    b.wcell_ids = c->at<int>(L.wcell_ids);
    b.nodeword = c->at<uint32_t>(L.nodeword);
    b.map_ids = c->at<int>(L.map_ids[0]);
    b.map_vals = c->at<void>(L.map_vals[0]);
    b.cnt = c->at<uint32_t>(L.cnt[0]);
    b.ovf = c->at<int>(L.ovf);
    b.u = c->at<void>(L.u);
    b.sig = c->at<void>(L.sig);
    b.err = c->at<unsigned>(L.err);
    b.tab.seg = c->at<int4>(L.segs);
    b.tab.nb = c->at<int>(L.segnb);
    b.tab.map = c->at<int>(L.segmap);
    b.step_ctr = c->at<unsigned>(L.step_ctr);

    hipStream_t s = c->stream;
    auto h2d = [&](size_t off, const void* src, size_t bytes) {
        return bytes ? hipMemcpyAsync(c->base + off, src, bytes, hipMemcpyHostToDevice, s) : hipSuccess;
    };
    // rest state: shifted populations zero, fields zero
    hipError_t e = hipMemsetAsync(c->base, 0, L.total, s);
    if (e != hipSuccess) return init_fail(c, LB_EHIP, std::string("hipMemsetAsync: ") + hipGetErrorString(e));
    std::vector<uint32_t> nw(g.ld, 0u);
    std::copy(g.nodeword.begin(), g.nodeword.end(), nw.begin());
    e = e ? e : h2d(L.nodeword, nw.data(), nw.size() * 4);
    e = e ? e : h2d(L.wall_xyz, g.wall_xyz.data(), g.wall_xyz.size() * 4);
    e = e ? e : h2d(L.wcell_off, g.wcell_off.data(), g.wcell_off.size() * 4);
    e = e ? e : h2d(L.wcell_ids, g.wcell_ids.data(), g.wcell_ids.size() * 4);
    e = e ? e : h2d(L.wn_node, g.wn_node.data(), g.wn_node.size() * 8);
    e = e ? e : h2d(L.wn_nrm, g.wn_nrm.data(), g.wn_nrm.size() * 8);
    e = e ? e : h2d(L.planes, g.planes.data(), g.planes.size() * 4);
    e = e ? e : h2d(L.segs, g.segs.data(), g.segs.size() * 4);
    e = e ? e : h2d(L.segnb, g.segnb.data(), g.segnb.size() * 4);
    e = e ? e : h2d(L.segmap, g.segmap.data(), g.segmap.size() * 4);
    std::vector<RbcState> hs(n_rbc);
    for (int i = 0; i < n_rbc; ++i) {
        RbcState& r = hs[i];
        std::memset(&r, 0, sizeof r);
        for (int a = 0; a < 3; ++a) {
            double v = cells[i].R[a];
            if (C.periodic[a]) {
                const double Lh = a == 0 ? C.nx : (a == 1 ? C.ny : C.nz);
                if (v >= Lh) v -= Lh;
                else if (v < 0.0) v += Lh;
            }
            r.R[a] = v;
            r.V[a] = cells[i].V[a];
            r.Om[a] = cells[i].Omega[a];
        }
        for (int a = 0; a < 9; ++a) r.Q[a] = cells[i].Q[a];
    }
    e = e ? e : h2d(L.st, hs.data(), hs.size() * sizeof(RbcState));
    // the context's record for fused multi-lattice launches
    SlotDesc sd;
    std::memset(&sd, 0, sizeof sd);
    sd.kp = kp;
    sd.b = b;
    sd.fA = c->fA;
    sd.fB = c->fB;
    e = e ? e : h2d(L.slot, &sd, sizeof sd);
    if (e != hipSuccess) return init_fail(c, LB_EHIP, std::string("hipMemcpyAsync: ") + hipGetErrorString(e));
    if (n_rbc > 0) {
        // start-up: F^comb(0) = F^mech(0), tau^comb(0) = tau^mech(0) (fluid at rest)
        launch_cell_list(b, kp, s);
        launch_gay_berne(b, kp, s);
        launch_init_combined(b, kp, s);
    }
    e = hipGetLastError();
    if (e != hipSuccess) return init_fail(c, LB_EHIP, std::string("kernel launch: ") + hipGetErrorString(e));
    e = hipStreamSynchronize(s);
    if (e != hipSuccess) return init_fail(c, LB_EHIP, std::string("hipStreamSynchronize: ") + hipGetErrorString(e));
    // (on the context's stream: a copy on the null stream would wait for other streams)
    unsigned err = 0;
    e = hipMemcpyAsync(&err, b.err, 4, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return init_fail(c, LB_EHIP, std::string("hipMemcpy: ") + hipGetErrorString(e));
    if (err & ERR_OVERLAP) return init_fail(c, LB_EOVERLAP, "Gay-Berne pair at rho <= 0 in the initial state");
    if (n_rbc >= SIDE_STREAM_MIN_CELLS) {
        e = hipStreamCreateWithFlags(&c->side, hipStreamNonBlocking);
        c->side_owned = e == hipSuccess;
        for (hipEvent_t* ev : {&c->ev_cells, &c->ev_gb, &c->ev_map})
            if (e == hipSuccess) e = hipEventCreateWithFlags(ev, hipEventDisableTiming);
        if (e != hipSuccess) {
            release_side(c);
            return init_fail(c, LB_EHIP, std::string("side stream: ") + hipGetErrorString(e));
        }
    }
    *out = c;
    return LB_OK;
}

lb_status lb_step(lb_ctx c, int nsteps)
{
    if (!c || nsteps < 0) return LB_EINVAL;
    if (c->poisoned) return fail(c, LB_ESTATE, "context poisoned by a device fault");
    if (c->timing && !c->step_t0_set && nsteps > 0) {
        (void)hipEventRecord(c->step_t0, c->stream);
        c->step_t0_set = true;
    }
    for (int k = 0; k < nsteps; ++k) enqueue_step(c, k + 1 == nsteps);
    if (c->timing && nsteps > 0) {
        (void)hipEventRecord(c->step_t1, c->stream);
        c->timed_steps += nsteps;
    }
    HIPCHK(c, hipGetLastError());
    return LB_OK;
}

lb_status lb_batch_step(lb_ctx* ctxs, const int* nsteps, int n)
{
    if (!ctxs || !nsteps || n < 0) return LB_EINVAL;
    if (n == 0) return LB_OK;
    int most = 0;
    bool fuse = n > 1;
    for (int i = 0; i < n; ++i) {
        if (!ctxs[i] || nsteps[i] < 0) return LB_EINVAL;
        if (ctxs[i]->poisoned) return LB_ESTATE;
        most = std::max(most, nsteps[i]);
        fuse = fuse && fusable(ctxs[i], ctxs[0]);
    }
    if (fuse) {
        FusedSide* fs = fused_side(ctxs[0]->device);
        std::unique_lock<std::mutex> lock;
        if (fs) lock = std::unique_lock<std::mutex>(fs->mu);
        std::vector<lb_ctx> act;
        for (int k = 0; k < most; ++k) {
            act.clear();
            for (int i = 0; i < n; ++i)
                if (k < nsteps[i]) act.push_back(ctxs[i]);
            for (size_t g = 0; g < act.size(); g += FUSE_MAX)
                enqueue_fused_step(act.data() + g, (int)std::min<size_t>(FUSE_MAX, act.size() - g), fs);
        }
        if (fs) (void)hipStreamWaitEvent(ctxs[0]->stream, fs->join, 0);
    } else {
        for (int k = 0; k < most; ++k)
            for (int i = 0; i < n; ++i)
                if (k < nsteps[i]) enqueue_step(ctxs[i], k + 1 == nsteps[i]);
    }
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? LB_OK : LB_EHIP;
}

}  // extern "C"

// A captured sequence of fused steps over a fixed set of contexts (serving).
struct lb_graph_s {
    std::vector<lb_ctx> ctxs;
    int nsteps = 0;
    hipStream_t stream = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipEvent_t done = nullptr;   // recorded after every replay; destruction waits for it
};

extern "C" {

lb_status lb_batch_capture(lb_ctx* ctxs, int n, int nsteps, lb_graph* out)
{
    if (!ctxs || !out || n < 1 || nsteps < 2 || (nsteps & 1)) return LB_EINVAL;
    *out = nullptr;
    for (int i = 0; i < n; ++i) {
        if (!ctxs[i]) return LB_EINVAL;
        if (ctxs[i]->poisoned) return fail(ctxs[i], LB_ESTATE, "context poisoned by a device fault");
        if (!fusable(ctxs[i], ctxs[0]))
            return fail(ctxs[i], LB_EINVAL, "lb_batch_capture: the contexts must share one stream and "
                                            "one storage, without open boundaries, WSS accumulation or timing");
        for (int j = 0; j < i; ++j)
            if (ctxs[j] == ctxs[i]) return fail(ctxs[i], LB_EINVAL, "lb_batch_capture: a context twice");
    }
    hipStream_t s = ctxs[0]->stream;
    struct Saved {
        void *fA, *fB;
        long long step;
        bool dirty0;
        int map_parity;
    };
    std::vector<Saved> sv(n);
    for (int i = 0; i < n; ++i) {
        lb_ctx c = ctxs[i];
        sv[i] = {c->fA, c->fB, c->step, c->dirty[0], c->map_parity};
        // every replay first clears the coverage counts of every context, whatever the host
        // did in between (e.g. rbc_couple): counts left clean are read and left as they are
        c->dirty[0] = true;
    }
    // the side stream of the Gay-Berne stage exists before the capture starts
    FusedSide* fs = fused_side(ctxs[0]->device);
    std::unique_lock<std::mutex> lock;
    if (fs) lock = std::unique_lock<std::mutex>(fs->mu);
    // an error left by earlier work of this thread would read as a launch error of the capture
    const hipError_t pending = hipGetLastError();
    if (pending != hipSuccess) {
        for (int i = 0; i < n; ++i) ctxs[i]->dirty[0] = sv[i].dirty0;
        return fail(ctxs[0], LB_EHIP, std::string("lb_batch_capture: error pending before the capture: ") +
                                          hipGetErrorString(pending));
    }
    hipError_t e = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) {
        for (int i = 0; i < n; ++i) ctxs[i]->dirty[0] = sv[i].dirty0;
        return fail(ctxs[0], LB_EHIP, std::string("hipStreamBeginCapture: ") + hipGetErrorString(e));
    }
    // the first launch error (launch checks are synchronous, also under capture)
    hipError_t launch_err = hipSuccess;
    for (int k = 0; k < nsteps && launch_err == hipSuccess; ++k) {
        for (int g = 0; g < n; g += FUSE_MAX) enqueue_fused_step(ctxs + g, std::min(FUSE_MAX, n - g), fs);
        launch_err = hipGetLastError();
    }
    // the last kick rejoins the capturing stream
    if (fs) (void)hipStreamWaitEvent(s, fs->join, 0);
    hipGraph_t graph = nullptr;
    e = hipStreamEndCapture(s, &graph);
    if (launch_err != hipSuccess && e == hipSuccess) e = launch_err;
    // nothing ran: the host state is what it was (an even step count returns the buffers)
    for (int i = 0; i < n; ++i) {
        lb_ctx c = ctxs[i];
        c->fA = sv[i].fA;
        c->fB = sv[i].fB;
        c->step = sv[i].step;
        c->dirty[0] = sv[i].dirty0;
        c->map_parity = sv[i].map_parity;
    }
    if (e != hipSuccess || !graph) {
        if (graph) (void)hipGraphDestroy(graph);
        return fail(ctxs[0], LB_EHIP,
                    std::string("hipStreamEndCapture: ") + hipGetErrorString(e) +
                        (launch_err != hipSuccess ? std::string("; first launch error: ") + hipGetErrorString(launch_err)
                                                  : std::string()));
    }
    hipGraphExec_t exec = nullptr;
    e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        (void)hipGraphDestroy(graph);
        return fail(ctxs[0], LB_EHIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
    }
    hipEvent_t done = nullptr;
    e = hipEventCreateWithFlags(&done, hipEventDisableTiming);
    if (e != hipSuccess) {
        (void)hipGraphExecDestroy(exec);
        (void)hipGraphDestroy(graph);
        return fail(ctxs[0], LB_EHIP, std::string("hipEventCreate: ") + hipGetErrorString(e));
    }
    lb_graph g = new lb_graph_s();
    g->done = done;
    g->ctxs.assign(ctxs, ctxs + n);
    g->nsteps = nsteps;
    g->stream = s;
    g->graph = graph;
    g->exec = exec;
    *out = g;
    return LB_OK;
}

lb_status lb_graph_launch(lb_graph g)
{
    if (!g) return LB_EINVAL;
    for (lb_ctx c : g->ctxs) {
        if (c->poisoned) return fail(c, LB_ESTATE, "context poisoned by a device fault");
        if (c->stream != g->stream) return fail(c, LB_EINVAL, "context moved off the captured stream");
    }
    hipError_t e = hipGraphLaunch(g->exec, g->stream);
    if (e == hipSuccess) e = hipEventRecord(g->done, g->stream);
    if (e != hipSuccess) return fail(g->ctxs[0], LB_EHIP, std::string("hipGraphLaunch: ") + hipGetErrorString(e));
    for (lb_ctx c : g->ctxs) {
        c->step += g->nsteps;
        c->dirty[0] = false;
        c->map_parity = 0;
    }
    return LB_OK;
}

void lb_graph_destroy(lb_graph g)
{
    if (!g) return;
    // the last replay must have finished before its executable goes
    if (g->done) {
        (void)hipEventSynchronize(g->done);
        (void)hipEventDestroy(g->done);
    }
    if (g->exec) (void)hipGraphExecDestroy(g->exec);
    if (g->graph) (void)hipGraphDestroy(g->graph);
    delete g;
}

lb_status rbc_couple(lb_ctx c)
{
    if (!c) return LB_EINVAL;
    with_types(c->cfg.storage, [&](auto*, auto* rp) {
        using RT = std::remove_pointer_t<decltype(rp)>;
        if (c->nrbc > 0) enqueue_cells_map_couple<RT>(c);
        const CellBuffers b = c->par(c->map_parity);
        launch_spread_field<RT>(b.nodeword, b.map_ids, b.map_vals, b.cnt, c->cb.gat,
                                c->at<void>(c->lay.gdbg), c->at<void>(c->lay.tdbg), c->kp, c->stream);
    });
    HIPCHK(c, hipGetLastError());
    return LB_OK;
}

lb_status rbc_collide(lb_ctx c, double* F, double* T)
{
    if (!c) return LB_EINVAL;
    if (c->nrbc == 0) return LB_OK;
    launch_cell_list(c->cb, c->kp, c->stream);
    launch_gay_berne(c->cb, c->kp, c->stream);
    lb_status st = check_fault(c);
    std::vector<RbcCouple> cp(c->nrbc);
    HIPCHK(c, hipMemcpy(cp.data(), c->cb.cp, cp.size() * sizeof(RbcCouple), hipMemcpyDeviceToHost));
    for (int i = 0; i < c->nrbc; ++i)
        for (int a = 0; a < 3; ++a) {
            if (F) F[3 * i + a] = cp[i].Fm[a];
            if (T) T[3 * i + a] = cp[i].Tm[a];
        }
    return st;
}

lb_status lb_set_stream(lb_ctx c, void* hip_stream)
{
    if (!c || !hip_stream) return LB_EINVAL;
    c->stream = (hipStream_t)hip_stream;
    return LB_OK;
}

lb_status rbc_collide_static(lb_ctx c, double* F, double* T)
{
    if (!c) return LB_EINVAL;
    if (c->nrbc == 0) return LB_OK;
    if (!F || !T) return fail(c, LB_EINVAL, "rbc_collide_static needs device arrays F and T");
    if (c->poisoned) return fail(c, LB_ESTATE, "context poisoned by a device fault");
    const long long nc = (long long)c->kp.ncell[0] * c->kp.ncell[1] * c->kp.ncell[2];
    if (c->nrbc > STATIC_MAX_CELLS || nc > STATIC_MAX_GRID)
        return fail(c, LB_EINVAL, "rbc_collide_static: more than 262,144 cells or 1,048,576 grid cells "
                                  "(the size of its static scratch)");
    int* base = g_scratch_ptr[c->device];
    if (!base) return fail(c, LB_EHIP, "static scratch address not resolved for this device");
    CellBuffers b = c->cb;
    b.cellid = base;
    b.cell_ids = base + STATIC_MAX_CELLS;
    b.cell_cnt = base + 2 * (size_t)STATIC_MAX_CELLS;
    b.cell_off = b.cell_cnt + STATIC_MAX_GRID;
    b.cell_part = b.cell_off + STATIC_MAX_GRID + 1;
    // the counts the binning adds to start at zero whatever an earlier call left
    launch_zero_ints(b.cell_cnt, nc, c->stream);
    launch_cell_list(b, c->kp, c->stream);
    launch_gay_berne_out(b, c->kp, F, T, 3, c->stream);
    HIPCHK(c, hipGetLastError());
    return LB_OK;
}

lb_status lb_set_side_stream(lb_ctx c, void* hip_stream)
{
    if (!c) return LB_EINVAL;
    HIPCHK(c, hipStreamSynchronize(c->stream));
    release_side(c);
    c->cells_ahead = false;
    if (!hip_stream) return LB_OK;
    c->side = (hipStream_t)hip_stream;
    c->side_owned = false;
    for (hipEvent_t* ev : {&c->ev_cells, &c->ev_gb, &c->ev_map}) {
        hipError_t e = hipEventCreateWithFlags(ev, hipEventDisableTiming);
        if (e != hipSuccess) {
            release_side(c);
            return fail(c, LB_EHIP, std::string("side stream events: ") + hipGetErrorString(e));
        }
    }
    return LB_OK;
}

lb_status lb_sync(lb_ctx c)
{
    if (!c) return LB_EINVAL;
    return check_fault(c);
}

lb_status lb_observe(lb_ctx c, lb_observables* o)
{
    if (!c || !o) return LB_EINVAL;
    std::memset(o, 0, sizeof *o);
    with_types(c->cfg.storage, [&](auto* sp, auto* rp) {
        using ST = std::remove_pointer_t<decltype(sp)>;
        using RT = std::remove_pointer_t<decltype(rp)>;
        launch_observe<ST, RT>(c->fA, c->cb.nodeword, c->at<void>(c->lay.u), c->kp,
                               c->at<double>(c->lay.partials), OBS_BLOCKS, c->at<double>(c->lay.obs_out),
                               c->stream);
        launch_wss<RT>(c->at<void>(c->lay.sig), c->at<long long>(c->lay.wn_node),
                       c->at<double>(c->lay.wn_nrm), (int)c->geo.wn_node.size(), c->kp,
                       c->at<double>(c->lay.wss), nullptr, 0, c->stream);
    });
    lb_status st = check_fault(c);
    double r[6];
    HIPCHK(c, hipMemcpy(r, c->at<double>(c->lay.obs_out), sizeof r, hipMemcpyDeviceToHost));
    const size_t nwn = c->geo.wn_node.size();
    std::vector<double> w(nwn), acc(nwn);
    if (nwn) {
        HIPCHK(c, hipMemcpy(w.data(), c->at<double>(c->lay.wss), nwn * 8, hipMemcpyDeviceToHost));
        HIPCHK(c, hipMemcpy(acc.data(), c->at<double>(c->lay.wss_acc), nwn * 8, hipMemcpyDeviceToHost));
    }
    o->mass = r[0];
    o->momentum[0] = r[1];
    o->momentum[1] = r[2];
    o->momentum[2] = r[3];
    o->flow_rate = r[4] / c->cfg.nz;
    const double area = (double)c->geo.n_fluid / c->cfg.nz;
    const double Rt = std::sqrt(area / M_PI);
    o->eta_app = o->flow_rate != 0.0 ? M_PI * std::pow(Rt, 4.0) * c->cfg.g_ext[2] / (8.0 * o->flow_rate) : 0.0;
    double sum = 0, mx = 0, asum = 0;
    for (size_t k = 0; k < nwn; ++k) {
        sum += w[k];
        mx = std::max(mx, w[k]);
        asum += acc[k];
    }
    o->wss_mean = nwn ? sum / nwn : 0.0;
    o->wss_max = mx;
    o->wss_time_mean = (nwn && c->wss_count) ? asum / (double)nwn / (double)c->wss_count : 0.0;
    o->step = c->step;
    o->flags = c->fault;
    o->n_fluid = c->geo.n_fluid;
    o->n_wall_nodes = (int)nwn;
    o->n_rbc = c->nrbc;
    o->compact = c->geo.compact ? 1 : 0;
    o->n_stored = c->kp.N;
    return st;
}

lb_status lb_wall_shear_stress(lb_ctx c, int time, double* wss, long long* node, int* n)
{
    if (!c || !n) return LB_EINVAL;
    const int nwn = (int)c->geo.wn_node.size();
    *n = nwn;
    if (node)
        for (int k = 0; k < nwn; ++k) node[k] = c->geo.wn_dense[k];
    if (!wss) return LB_OK;
    if (time) {
        HIPCHK(c, hipStreamSynchronize(c->stream));
        std::vector<double> acc(nwn);
        if (nwn) HIPCHK(c, hipMemcpy(acc.data(), c->at<double>(c->lay.wss_acc), nwn * 8, hipMemcpyDeviceToHost));
        for (int k = 0; k < nwn; ++k) wss[k] = c->wss_count ? acc[k] / (double)c->wss_count : 0.0;
        return check_fault(c);
    }
    with_types(c->cfg.storage, [&](auto*, auto* rp) {
        using RT = std::remove_pointer_t<decltype(rp)>;
        launch_wss<RT>(c->at<void>(c->lay.sig), c->at<long long>(c->lay.wn_node),
                       c->at<double>(c->lay.wn_nrm), nwn, c->kp, c->at<double>(c->lay.wss), nullptr, 0,
                       c->stream);
    });
    lb_status st = check_fault(c);
    if (nwn) HIPCHK(c, hipMemcpy(wss, c->at<double>(c->lay.wss), nwn * 8, hipMemcpyDeviceToHost));
    return st;
}

lb_status lb_apparent_viscosity(lb_ctx c, double* eta)
{
    if (!c || !eta) return LB_EINVAL;
    lb_observables o;
    lb_status st = lb_observe(c, &o);
    *eta = o.eta_app;
    return st;
}

lb_status lb_wss_accumulate(lb_ctx c, int on)
{
    if (!c) return LB_EINVAL;
    if (on) {
        const size_t nwn = c->geo.wn_node.size();
        if (nwn) HIPCHK(c, hipMemsetAsync(c->at<double>(c->lay.wss_acc), 0, nwn * 8, c->stream));
        c->wss_count = 0;
    }
    c->wss_on = on ? 1 : 0;
    return LB_OK;
}

lb_status lb_get_fields(lb_ctx c, double* f, double* u, double* sigma, double* g, double* relax)
{
    if (!c) return LB_EINVAL;
    lb_status st = check_fault(c);
    const int S = c->cfg.storage;
    const size_t N = (size_t)c->geo.nodes, ld = (size_t)c->kp.ld;
    const size_t rs = real_bytes(S);
    // storage slot of every lattice node (-1: not stored, rest state and zero fields)
    std::vector<long long> ks(N);
    for (size_t n = 0; n < N; ++n) ks[n] = c->geo.store_of((long long)n, c->cfg.nx, c->cfg.ny);
    if (f) {
        std::vector<char> h(19 * ld * storage_bytes(S));
        HIPCHK(c, hipMemcpy(h.data(), c->fA, h.size(), hipMemcpyDeviceToHost));
        const double inv = S == LB_F16 ? 1.0 / c->cfg.f16_scale : 1.0;
        for (int p = 0; p < 19; ++p)
            for (size_t n = 0; n < N; ++n)
                f[p * N + n] = w_(p) + (ks[n] < 0 ? 0.0 : load_stored(h.data(), p * ld + ks[n], S, inv));
    }
    // the fields u and sigma: node-interleaved records of `stride` elements (element
    // k * stride + a); the debug planes g and T: compute precision, planes a * ld + k
    auto fields = [&](size_t off, int k, int stride, double* out) -> lb_status {
        std::vector<char> h(stride * ld * field_bytes(S));
        HIPCHK(c, hipMemcpy(h.data(), c->base + off, h.size(), hipMemcpyDeviceToHost));
        for (int a = 0; a < k; ++a)
            for (size_t n = 0; n < N; ++n)
                out[n * k + a] = ks[n] < 0 ? 0.0 : load_field(h.data(), (size_t)ks[n] * stride + a, S);
        return LB_OK;
    };
    auto planes = [&](size_t off, int k, double* out) -> lb_status {
        std::vector<char> h(k * ld * rs);
        HIPCHK(c, hipMemcpy(h.data(), c->base + off, h.size(), hipMemcpyDeviceToHost));
        for (int a = 0; a < k; ++a)
            for (size_t n = 0; n < N; ++n) out[n * k + a] = ks[n] < 0 ? 0.0 : load_real(h.data(), a * ld + ks[n], S);
        return LB_OK;
    };
    lb_status r;
    if (u && (r = fields(c->lay.u, 3, vel_stride(S), u)) != LB_OK) return r;
    if (sigma && (r = fields(c->lay.sig, 6, 6, sigma)) != LB_OK) return r;
    if (g && (r = planes(c->lay.gdbg, 3, g)) != LB_OK) return r;
    if (relax && (r = planes(c->lay.tdbg, 1, relax)) != LB_OK) return r;
    return st;
}

lb_status lb_set_fields(lb_ctx c, const double* f, const double* u, const double* sigma)
{
    if (!c) return LB_EINVAL;
    HIPCHK(c, hipStreamSynchronize(c->stream));
    const int S = c->cfg.storage;
    const size_t N = (size_t)c->geo.nodes, ld = (size_t)c->kp.ld;
    // nodes that are not stored (compact layout) are solid: their values are dropped
    std::vector<long long> ks(N);
    for (size_t n = 0; n < N; ++n) ks[n] = c->geo.store_of((long long)n, c->cfg.nx, c->cfg.ny);
    if (f) {
        std::vector<char> h(19 * ld * storage_bytes(S), 0);
        const double scale = S == LB_F16 ? c->cfg.f16_scale : 1.0;
        for (int p = 0; p < 19; ++p)
            for (size_t n = 0; n < N; ++n)
                if (ks[n] >= 0) store_value(h.data(), p * ld + ks[n], S, f[p * N + n] - w_(p), scale);
        HIPCHK(c, hipMemcpy(c->fA, h.data(), h.size(), hipMemcpyHostToDevice));
    }
    // u and sigma are node-interleaved records of `stride` elements on the device
    auto fields = [&](size_t off, int k, int stride, const double* in) -> lb_status {
        std::vector<char> h(stride * ld * field_bytes(S), 0);
        for (int a = 0; a < k; ++a)
            for (size_t n = 0; n < N; ++n)
                if (ks[n] >= 0) store_field(h.data(), (size_t)ks[n] * stride + a, S, in[n * k + a]);
        HIPCHK(c, hipMemcpy(c->base + off, h.data(), h.size(), hipMemcpyHostToDevice));
        return LB_OK;
    };
    lb_status r;
    if (u && (r = fields(c->lay.u, 3, vel_stride(S), u)) != LB_OK) return r;
    if (sigma && (r = fields(c->lay.sig, 6, 6, sigma)) != LB_OK) return r;
    HIPCHK(c, hipMemset(c->cb.err, 0, 4));
    c->poisoned = false;
    c->fault = 0;
    return LB_OK;
}

lb_status rbc_get_state(lb_ctx c, lb_rbc* out, int n)
{
    if (!c || (n > 0 && !out) || n > c->nrbc) return LB_EINVAL;
    lb_status st = check_fault(c);
    std::vector<RbcState> h(n);
    if (n) HIPCHK(c, hipMemcpy(h.data(), c->cb.st, n * sizeof(RbcState), hipMemcpyDeviceToHost));
    for (int i = 0; i < n; ++i) {
        for (int a = 0; a < 3; ++a) {
            out[i].R[a] = h[i].R[a];
            out[i].V[a] = h[i].V[a];
            out[i].Omega[a] = h[i].Om[a];
        }
        for (int a = 0; a < 9; ++a) out[i].Q[a] = h[i].Q[a];
    }
    return st;
}

lb_status rbc_set_state(lb_ctx c, const lb_rbc* in, int n)
{
    if (!c || n != c->nrbc || (n > 0 && !in)) return LB_EINVAL;
    HIPCHK(c, hipStreamSynchronize(c->stream));
    std::vector<RbcState> h(n);
    if (n) HIPCHK(c, hipMemcpy(h.data(), c->cb.st, n * sizeof(RbcState), hipMemcpyDeviceToHost));
    for (int i = 0; i < n; ++i) {
        for (int a = 0; a < 3; ++a) {
            h[i].R[a] = in[i].R[a];
            h[i].V[a] = in[i].V[a];
            h[i].Om[a] = in[i].Omega[a];
        }
        for (int a = 0; a < 9; ++a) h[i].Q[a] = in[i].Q[a];
    }
    if (n) HIPCHK(c, hipMemcpy(c->cb.st, h.data(), n * sizeof(RbcState), hipMemcpyHostToDevice));
    return LB_OK;
}

lb_status rbc_get_coupling(lb_ctx c, double* o, int n)
{
    if (!c || (n > 0 && !o) || n > c->nrbc) return LB_EINVAL;
    lb_status st = check_fault(c);
    std::vector<RbcState> hs(n);
    std::vector<RbcCouple> hc(n);
    if (n) {
        HIPCHK(c, hipMemcpy(hs.data(), c->cb.st, n * sizeof(RbcState), hipMemcpyDeviceToHost));
        HIPCHK(c, hipMemcpy(hc.data(), c->cb.cp, n * sizeof(RbcCouple), hipMemcpyDeviceToHost));
    }
    for (int i = 0; i < n; ++i) {
        double* r = o + 22 * i;
        r[0] = hc[i].S;
        for (int a = 0; a < 3; ++a) {
            r[1 + a] = hc[i].ut[a];
            r[4 + a] = hc[i].wt[a];
            r[7 + a] = hc[i].TS[a];
            r[10 + a] = hc[i].Fh[a];
            r[13 + a] = hc[i].Th[a];
            r[16 + a] = hs[i].Fc[a];
            r[19 + a] = hs[i].Tc[a];
        }
    }
    return st;
}

lb_status rbc_get_cells(lb_ctx c, int* ncell, int* off, int* ids)
{
    if (!c) return LB_EINVAL;
    lb_status st = check_fault(c);
    const int nc = c->kp.ncell[0] * c->kp.ncell[1] * c->kp.ncell[2];
    if (ncell)
        for (int a = 0; a < 3; ++a) ncell[a] = c->kp.ncell[a];
    if (off) HIPCHK(c, hipMemcpy(off, c->cb.cell_off, (nc + 1) * 4, hipMemcpyDeviceToHost));
    if (ids && c->nrbc) HIPCHK(c, hipMemcpy(ids, c->cb.cell_ids, c->nrbc * 4, hipMemcpyDeviceToHost));
    return st;
}

lb_status rbc_get_map(lb_ctx c, int* off, int* ids, long long* len)
{
    if (!c || !len) return LB_EINVAL;
    lb_status st = check_fault(c);
    const size_t N = (size_t)c->geo.nodes, NS = (size_t)c->kp.N, ld = (size_t)c->kp.ld;
    const CellBuffers b = c->par(c->map_parity);
    std::vector<uint32_t> cs(NS, 0u);
    if (c->nrbc && NS) HIPCHK(c, hipMemcpy(cs.data(), b.cnt, NS * 4, hipMemcpyDeviceToHost));
    // counts and slot columns in lattice order
    std::vector<uint32_t> cn(N, 0u);
    std::vector<long long> ks(N);
    for (size_t n = 0; n < N; ++n) {
        ks[n] = c->geo.store_of((long long)n, c->cfg.nx, c->cfg.ny);
        if (ks[n] >= 0) cn[n] = cs[(size_t)ks[n]];
    }
    long long tot = 0;
    for (size_t n = 0; n < N; ++n) tot += std::min<int>((int)cn[n], c->kp.cap);
    if (!ids) {
        *len = tot;
        if (off) {
            off[0] = 0;
            for (size_t n = 0; n < N; ++n) off[n + 1] = off[n] + std::min<int>((int)cn[n], c->kp.cap);
        }
        return st;
    }
    if (*len < tot) return LB_EINVAL;
    std::vector<int> slots;
    if (c->nrbc) {
        slots.resize((size_t)c->kp.cap * ld);
        HIPCHK(c, hipMemcpy(slots.data(), b.map_ids, slots.size() * 4, hipMemcpyDeviceToHost));
    }
    long long k = 0;
    if (off) off[0] = 0;
    for (size_t n = 0; n < N; ++n) {
        const int cnt = std::min<int>((int)cn[n], c->kp.cap);
        const long long k0 = k;
        for (int q = 0; q < cnt; ++q) ids[k++] = slots[(size_t)q * ld + (size_t)ks[n]] >> c->kp.ent_shift;
        std::sort(ids + k0, ids + k);
        if (off) off[n + 1] = (int)k;
    }
    *len = tot;
    return st;
}

// checkpoint: header, populations (storage precision), u, sigma (their element type and
// record layout), cell states, WSS sums. The header records the lattice shape, the FP16 scale,
// the BF16 rounding mode and a hash of the node words (geometry and boundary flags): a
// checkpoint loads only into a context whose stored values mean the same thing. Version 3: u and
// sigma of the 16-bit storages in 16 bits.
constexpr int CKPT_VERSION = 3;
struct CkptHeader {
    char magic[8];
    int version, storage, nrbc, nwn;
    long long N, step, wss_count;
    int wss_on, bf16_nearest;
    int nx, ny, nz, pad;
    double f16_scale;
    unsigned long long geom_hash;
};

lb_status lb_save(lb_ctx c, void* buf, size_t* bytes)
{
    if (!c || !bytes) return LB_EINVAL;
    const size_t ld = (size_t)c->kp.ld;
    const size_t fb = 19 * ld * storage_bytes(c->cfg.storage);
    const size_t ub = vel_stride(c->cfg.storage) * ld * field_bytes(c->cfg.storage),
                 sgb = 6 * ld * field_bytes(c->cfg.storage), rb = ub + sgb;
    const size_t sb = c->nrbc * sizeof(RbcState), wb = c->geo.wn_node.size() * 8;
    const size_t need = sizeof(CkptHeader) + fb + rb + sb + wb;
    if (!buf) {
        *bytes = need;
        return LB_OK;
    }
    if (*bytes < need) return LB_EINVAL;
    lb_status st = check_fault(c);
    CkptHeader h{};
    std::memcpy(h.magic, "LBRBCCK1", 8);
    h.version = CKPT_VERSION;
    h.storage = c->cfg.storage;
    h.bf16_nearest = c->cfg.bf16_nearest;
    h.nx = c->cfg.nx;
    h.ny = c->cfg.ny;
    h.nz = c->cfg.nz;
    h.f16_scale = c->cfg.storage == LB_F16 ? c->cfg.f16_scale : 0.0;
    h.geom_hash = c->geo_hash;
    h.nrbc = c->nrbc;
    h.nwn = (int)c->geo.wn_node.size();
    h.N = c->kp.N;
    h.step = c->step;
    h.wss_count = c->wss_count;
    h.wss_on = c->wss_on;
    char* p = (char*)buf;
    std::memcpy(p, &h, sizeof h);
    p += sizeof h;
    HIPCHK(c, hipMemcpy(p, c->fA, fb, hipMemcpyDeviceToHost));
    p += fb;
    HIPCHK(c, hipMemcpy(p, c->base + c->lay.u, ub, hipMemcpyDeviceToHost));
    HIPCHK(c, hipMemcpy(p + ub, c->base + c->lay.sig, sgb, hipMemcpyDeviceToHost));
    p += rb;
    if (sb) HIPCHK(c, hipMemcpy(p, c->cb.st, sb, hipMemcpyDeviceToHost));
    p += sb;
    if (wb) HIPCHK(c, hipMemcpy(p, c->at<double>(c->lay.wss_acc), wb, hipMemcpyDeviceToHost));
    *bytes = need;
    return st;
}

lb_status lb_load(lb_ctx c, const void* buf, size_t bytes)
{
    if (!c || !buf || bytes < sizeof(CkptHeader)) return LB_EINVAL;
    CkptHeader h;
    std::memcpy(&h, buf, sizeof h);
    const size_t ld = (size_t)c->kp.ld;
    const size_t fb = 19 * ld * storage_bytes(c->cfg.storage);
    const size_t ub = vel_stride(c->cfg.storage) * ld * field_bytes(c->cfg.storage),
                 sgb = 6 * ld * field_bytes(c->cfg.storage), rb = ub + sgb;
    const size_t sb = c->nrbc * sizeof(RbcState), wb = c->geo.wn_node.size() * 8;
    if (std::memcmp(h.magic, "LBRBCCK1", 8) != 0 || h.version != CKPT_VERSION)
        return fail(c, LB_EINVAL, "not a checkpoint of this library version");
    if (h.storage != c->cfg.storage || h.nrbc != c->nrbc || h.N != c->kp.N ||
        h.nwn != (int)c->geo.wn_node.size() || h.nx != c->cfg.nx || h.ny != c->cfg.ny ||
        h.nz != c->cfg.nz || h.bf16_nearest != c->cfg.bf16_nearest ||
        h.f16_scale != (c->cfg.storage == LB_F16 ? c->cfg.f16_scale : 0.0) || h.geom_hash != c->geo_hash ||
        bytes < sizeof h + fb + rb + sb + wb)
        return fail(c, LB_EINVAL, "checkpoint does not match this context (storage, scale, rounding, "
                                  "lattice shape, geometry or cell count)");
    HIPCHK(c, hipStreamSynchronize(c->stream));
    const char* p = (const char*)buf + sizeof h;
    HIPCHK(c, hipMemcpy(c->fA, p, fb, hipMemcpyHostToDevice));
    p += fb;
    HIPCHK(c, hipMemcpy(c->base + c->lay.u, p, ub, hipMemcpyHostToDevice));
    HIPCHK(c, hipMemcpy(c->base + c->lay.sig, p + ub, sgb, hipMemcpyHostToDevice));
    p += rb;
    if (sb) HIPCHK(c, hipMemcpy(c->cb.st, p, sb, hipMemcpyHostToDevice));
    p += sb;
    if (wb) HIPCHK(c, hipMemcpy(c->at<double>(c->lay.wss_acc), p, wb, hipMemcpyHostToDevice));
    c->step = h.step;
    {
        // the device step counter (the BF16 rounding's step term) continues from the saved step
        const unsigned ctr = (unsigned)h.step;
        HIPCHK(c, hipMemcpy(c->cb.step_ctr + c->ab_parity(), &ctr, 4, hipMemcpyHostToDevice));
    }
    c->wss_count = h.wss_count;
    c->wss_on = h.wss_on;
    HIPCHK(c, hipMemset(c->cb.err, 0, 4));
    c->poisoned = false;
    c->fault = 0;
    return LB_OK;
}

const char* lb_last_error(lb_ctx c) { return c ? c->last_error.c_str() : g_init_error.c_str(); }

lb_status lb_set_timing(lb_ctx c, int on)
{
    if (!c) return LB_EINVAL;
    HIPCHK(c, hipStreamSynchronize(c->stream));
    for (auto* pairs : {&c->sc_pairs, &c->map_pairs}) {
        for (auto& pr : *pairs) {
            c->ev_pool.push_back(pr.first);
            c->ev_pool.push_back(pr.second);
        }
        pairs->clear();
    }
    c->timed_steps = 0;
    c->step_t0_set = false;
    if (on && c->ev_pool.empty()) {
        for (int k = 0; k < 4 * MAX_TIMED; ++k) {
            hipEvent_t e;
            HIPCHK(c, hipEventCreate(&e));
            c->ev_pool.push_back(e);
        }
        HIPCHK(c, hipEventCreate(&c->step_t0));
        HIPCHK(c, hipEventCreate(&c->step_t1));
    }
    c->timing = on != 0;
    return LB_OK;
}

lb_status lb_kernel_time(lb_ctx c, double* sc_ms, double* step_ms)
{
    if (!c) return LB_EINVAL;
    HIPCHK(c, hipStreamSynchronize(c->stream));
    double tot = 0;
    for (auto& pr : c->sc_pairs) {
        float ms = 0;
        HIPCHK(c, hipEventElapsedTime(&ms, pr.first, pr.second));
        tot += ms;
    }
    if (sc_ms) *sc_ms = c->sc_pairs.empty() ? 0.0 : tot / c->sc_pairs.size();
    if (step_ms) {
        float ms = 0;
        if (c->timed_steps > 0 && c->step_t0_set) HIPCHK(c, hipEventElapsedTime(&ms, c->step_t0, c->step_t1));
        *step_ms = c->timed_steps > 0 ? ms / c->timed_steps : 0.0;
    }
    return LB_OK;
}

lb_status lb_map_time(lb_ctx c, double* map_ms)
{
    if (!c || !map_ms) return LB_EINVAL;
    HIPCHK(c, hipStreamSynchronize(c->stream));
    double tot = 0;
    for (auto& pr : c->map_pairs) {
        float ms = 0;
        HIPCHK(c, hipEventElapsedTime(&ms, pr.first, pr.second));
        tot += ms;
    }
    *map_ms = c->map_pairs.empty() ? 0.0 : tot / c->map_pairs.size();
    return LB_OK;
}

void lb_destroy(lb_ctx c)
{
    if (!c) return;
    (void)hipStreamSynchronize(c->stream);
    release_side(c);
    for (auto* pairs : {&c->sc_pairs, &c->map_pairs})
        for (auto& pr : *pairs) {
            (void)hipEventDestroy(pr.first);
            (void)hipEventDestroy(pr.second);
        }
    for (auto e : c->ev_pool) (void)hipEventDestroy(e);
    if (c->step_t0) (void)hipEventDestroy(c->step_t0);
    if (c->step_t1) (void)hipEventDestroy(c->step_t1);
    delete c;
}

}  // extern "C"
