// lb_kernels.hip -- per-node kernels: fused spreading + D3Q19 pull stream-collide,
// open z boundaries, the spread-field probe and the FP64 reductions (gfx950).
#include <climits>

#include "lbrbc_device.h"
#include "lbrbc_internal.h"

namespace lbrbc {

template <typename RT>
static MapPlanes<RT> map_planes(const int* ids, const void* vals, uint32_t* cnt, const KParams& kp)
{
    MapPlanes<RT> mp;
    for (int k = 0; k < CAP_MAX; ++k) mp.ids[k] = ids + (k < kp.cap ? (size_t)k * (size_t)kp.ld : 0);
    mp.vals0 = vals;
    mp.cnt = cnt;
    return mp;
}

// ---- spreading at one node (Sec. II B back-reaction G; Sec. II D, Eq. 23) -----------------
// g = g_ext - sum_i [F_i dhat_i - 1/2 T_i x grad(dhat_i)], theta = sum_i [1 - (1 - raw_i)^kappa]
// over the covering cells in ascending id order (a fixed order: bitwise repeatable). Each
// coverage slot holds an entry index e = (cell << ent_shift) | j, and entry e the (raw,
// grad raw) of that cell's j-th covered node, written by the per-cell pass; dhat = raw / S_i.
// The torque term carries the sign that hands the plasma -T_i of angular momentum.
//
// The slot words are read with branch-free loads (unused slots read the node's count, already
// in cache) so that all loads are in flight together; the entry indices, ascending in the cell,
// are sorted by a network sized to the wave's largest count (4, 8 or 12 slots).
template <int CN>
__device__ __forceinline__ void sort_keys(int* key)
{
#pragma unroll
    for (int r = 0; r < CN; ++r) {
#pragma unroll
        for (int k = (r & 1); k + 1 < CN; k += 2) {
            const int a = min(key[k], key[k + 1]), b = max(key[k], key[k + 1]);
            key[k] = a;
            key[k + 1] = b;
        }
    }
}

// FM: the field mode (entries in 16 bits for the 16-bit storages), or -1 to read it from kp
template <typename RT, int CN, int FM>
__device__ __forceinline__ void spread_slots(unsigned n, int cnt, const MapPlanes<RT>& mp,
                                             const Gather<RT>* __restrict__ gat, const KParams& kp,
                                             RT g[3], RT& theta)
{
    int key[CN];
#pragma unroll
    for (int k = 0; k < CN; ++k) {
        const int* a = (k < cnt) ? at32(mp.ids[k], n) : reinterpret_cast<const int*>(at32(mp.cnt, n));
        const int v = *a;
        key[k] = (k < cnt) ? v : INT_MAX;
    }
    sort_keys<CN>(key);
    for (int k = 0; k < cnt; ++k) {
        const int e = key[0];
#pragma unroll
        for (int j = 0; j + 1 < CN; ++j) key[j] = key[j + 1];
        const int i = e >> kp.ent_shift;
        RT r0, gx, gy, gz;
        load_entry<RT, FM>(mp.vals0, (size_t)e, kp, r0, gx, gy, gz);
        const Gather<RT>& G = gat[i];
        const RT invS = G.invS;
        const RT dh = r0 * invS;
        const RT gr0 = gx * invS, gr1 = gy * invS, gr2 = gz * invS;
        const RT T0 = G.T[0], T1 = G.T[1], T2 = G.T[2];
        g[0] -= G.F[0] * dh - RT(0.5) * (T1 * gr2 - T2 * gr1);
        g[1] -= G.F[1] * dh - RT(0.5) * (T2 * gr0 - T0 * gr2);
        g[2] -= G.F[2] * dh - RT(0.5) * (T0 * gr1 - T1 * gr0);
        theta += RT(1) - ipow_or_pow(RT(1) - r0, kp.kappa, kp.kappa_int);
    }
}

template <typename RT, int FM>
__device__ __forceinline__ void spread_at(unsigned n, uint32_t count, const MapPlanes<RT>& mp,
                                          const Gather<RT>* __restrict__ gat, const KParams& kp,
                                          RT g[3], RT& theta)
{
    g[0] = (RT)kp.gext[0];
    g[1] = (RT)kp.gext[1];
    g[2] = (RT)kp.gext[2];
    theta = RT(0);
    int cnt = (int)min(count, (uint32_t)kp.cap);
    // wave-uniform choice of the slot network
    if (!__any(cnt > 0)) return;
    if (!__any(cnt > 4)) spread_slots<RT, 4, FM>(n, cnt, mp, gat, kp, g, theta);
    else if (!__any(cnt > 8)) spread_slots<RT, 8, FM>(n, cnt, mp, gat, kp, g, theta);
    else spread_slots<RT, CAP_MAX, FM>(n, cnt, mp, gat, kp, g, theta);
}

// ---- pull sources in the compact layout -----------------------------------------------------
// The 27 neighbour segments of one stored segment, held in registers (scalar ones when the
// segment is wave-uniform). Entry e = (dx + 1) + 3 (dy + 1) + 9 (dz + 1).
struct SegNb {
    int e[27];
};
__device__ __forceinline__ void load_segnb(const int* __restrict__ nb, int s, SegNb& out)
{
#pragma unroll
    for (int j = 0; j < 27; ++j) out.e[j] = nb[27 * s + j];
}

// Storage index of the pull source x - c_P of node (x, y, z), storage k, in the segment that
// starts at x0: the source row is (y - c_y, z - c_z); along x it lies in the left neighbour
// segment when it falls before x0, in the right one when it passes the segment's last node (x0 + 63
// or the row's last node), else in the column of the node itself, at lane (x - c_x wrapped) mod 64.
// A source outside the box or in a segment that is not stored is solid: the node's own index is
// returned (any valid address: the bounce-back value replaces it).
template <int P>
__device__ __forceinline__ unsigned pull_src(unsigned k, int x, int x0, const SegNb& nb, const KParams& kp)
{
    constexpr int eb = 3 * (1 - cy_(P)) + 9 * (1 - cz_(P));
    int sn;
    if constexpr (cx_(P) > 0) sn = x == x0 ? nb.e[eb] : nb.e[eb + 1];
    else if constexpr (cx_(P) < 0) sn = (x == x0 + 63 || x == kp.nx - 1) ? nb.e[eb + 2] : nb.e[eb + 1];
    else sn = nb.e[eb + 1];
    int xs = x - cx_(P);
    xs += xs < 0 ? kp.nx : 0;
    xs -= xs >= kp.nx ? kp.nx : 0;
    return sn < 0 ? k : ((unsigned)sn << 6) | ((unsigned)xs & 63u);
}

// Dense layout (storage index n = x + nx (y + ny z)): the pull source offset is
// n - (c_x + nx c_y + nx ny c_z), wrapped by one period at the box faces on every axis, so the
// address is always inside the lattice (on a non-periodic face the source is a wall: the value
// read there is replaced by the bounce-back value)
template <int P>
__device__ __forceinline__ unsigned pull_off(unsigned n, int x, int y, int z, const KParams& kp)
{
    const unsigned sx = 1u, sy = (unsigned)kp.nx, sz = (unsigned)kp.nx * (unsigned)kp.ny;
    // offset change of the source along an axis: -c s normally, -c s (1 - L) across the face
    unsigned off = n;
    if (cx_(P)) off -= (unsigned)cx_(P) * ((x == (cx_(P) > 0 ? 0 : kp.nx - 1)) ? sx * (1u - (unsigned)kp.nx) : sx);
    if (cy_(P)) off -= (unsigned)cy_(P) * ((y == (cy_(P) > 0 ? 0 : kp.ny - 1)) ? sy * (1u - (unsigned)kp.ny) : sy);
    if (cz_(P)) off -= (unsigned)cz_(P) * ((z == (cz_(P) > 0 ? 0 : kp.nz - 1)) ? sz * (1u - (unsigned)kp.nz) : sz);
    return off;
}

// Where a node's pull sources are: in the dense layout from its coordinates, in the compact
// layout from its segment's neighbour table.
struct NodeAt {
    unsigned k;       // storage index
    int x, y, z;      // lattice coordinates
    int x0;           // compact layout: first x of the node's segment
    unsigned salt;    // step term of the BF16 stochastic rounding, shifted past the direction bits
};

// The step counter of a context: the stream-collide of step s (A/B parity par) reads
// ctr[par] = s and one of its threads writes ctr[par ^ 1] = s + 1 for the next step, so no
// launch reads the word it writes. The counter lives in device memory: captured graphs and fused
// launches advance it too. Its value salts the BF16 stochastic rounding (0 for other storages).
template <typename ST>
__device__ __forceinline__ unsigned step_salt(unsigned* ctr, int par, const KParams& kp, bool writer)
{
    unsigned v = 0;
    if (std::is_same<ST, bf16_t>::value && kp.bf16_sr) v = __builtin_amdgcn_readfirstlane(ctr[par]);
    if (writer) {
        const unsigned c = ctr[par];
        ctr[par ^ 1] = c + 1u;
    }
    return v << 5;
}

template <bool CMP, int P>
__device__ __forceinline__ unsigned source_of(const NodeAt& a, const SegNb& nb, const KParams& kp)
{
    if constexpr (CMP) return pull_src<P>(a.k, a.x, a.x0, nb, kp);
    else return pull_off<P>(a.k, a.x, a.y, a.z, kp);
}

// one population: a uniform plane base (scalar registers) plus a 32-bit per-lane offset;
// the bounce-back source is the opposite population at the node itself
template <typename ST, typename RT, bool CMP, int P>
__device__ __forceinline__ void pull_one(RT* f, const ST* __restrict__ fin, const NodeAt& a, uint32_t w,
                                         const SegNb& nb, const KParams& kp)
{
    constexpr int O = opp_(P);
    const bool bb = w & (1u << P);
    const ST* plane = fin + (size_t)(bb ? O : P) * (size_t)kp.ld;
    const unsigned off = bb ? a.k : source_of<CMP, P>(a, nb, kp);
    f[P] = Store<ST, RT>::ld(plane, off, kp.f16_inv);
}

template <typename ST, typename RT, bool CMP, int... Ps>
__device__ __forceinline__ void pull_all(RT* f, const ST* __restrict__ fin, const NodeAt& a, uint32_t w,
                                         const SegNb& nb, const KParams& kp, std::integer_sequence<int, Ps...>)
{
    (pull_one<ST, RT, CMP, Ps>(f, fin, a, w, nb, kp), ...);
}

// the 19 pull loads depend only on the position, so they issue without waiting for the node
// word; directions whose source is solid are then replaced by the opposite population at
// the node itself (halfway bounce-back)
template <typename ST, typename RT, bool CMP, typename PL, int... Ps>
__device__ __forceinline__ void pull_all_fast(RT* f, const PL& pl, const NodeAt& a, const SegNb& nb,
                                              const KParams& kp, std::integer_sequence<int, Ps...>)
{
    ((f[Ps] = Store<ST, RT>::ld(pl.src(Ps), source_of<CMP, Ps>(a, nb, kp), kp.f16_inv)), ...);
}

// Momentum a moving wall hands the population it reflects (Ladd's rule with wall density 1):
// 2 w_P (c_P . u_w) / c^2, u_w the velocity of the solid source row y - c_y (below the mid-plane
// y = ny/2: wall_u_lo, else wall_u_hi). Zero for resting walls.
template <typename RT, int P>
__device__ __forceinline__ RT moving_wall_term(int y, const KParams& kp)
{
    if (!kp.moving_walls) return RT(0);
    const double* uw = 2 * (y - cy_(P)) < kp.ny ? kp.uw_lo : kp.uw_hi;
    return RT(6.0 * w_(P) * ((double)cx_(P) * uw[0] + (double)cy_(P) * uw[1] + (double)cz_(P) * uw[2]));
}

template <typename ST, typename RT, typename PL, int... Ps>
__device__ __forceinline__ void bounce_back(RT* f, const PL& pl, unsigned n, uint32_t w, int y,
                                            const KParams& kp, std::integer_sequence<int, Ps...>)
{
    ((f[Ps] = (w & (1u << Ps)) ? Store<ST, RT>::ld(pl.src(opp_(Ps)), n, kp.f16_inv) + moving_wall_term<RT, Ps>(y, kp)
                               : f[Ps]), ...);
}

template <typename RT>
__device__ __forceinline__ RT feq_shift(int p, RT drho, RT rho, RT ux, RT uy, RT uz, RT usq)
{
    // shifted equilibrium f^eq - w (Eq. 3, c^2 = 1/3)
    const RT uc = RT(cx_(p)) * ux + RT(cy_(p)) * uy + RT(cz_(p)) * uz;
    return RT(w_(p)) * (drho + rho * (RT(3) * uc + RT(4.5) * uc * uc - RT(1.5) * usq));
}

// BGK with body force for the pair (P, P+1) of opposite speeds: the equilibrium and the
// force term split into parts even and odd in c, shared by the two directions. Lanes that
// do not hold a fluid node (live == false) store zero.
template <typename ST, typename RT, typename PL, int P>
__device__ __forceinline__ void collide_pair(const RT* f, const PL& pl, unsigned n,
                                             RT drho, RT rho, RT ux, RT uy, RT uz, RT usq,
                                             const RT g[3], RT gu, RT om, RT kf, RT k2, RT k3,
                                             const KParams& kp, bool live, bool put, unsigned slt)
{
    constexpr int Q = P + 1;
    const RT w = RT(w_(P));
    const RT uc = RT(cx_(P)) * ux + RT(cy_(P)) * uy + RT(cz_(P)) * uz;
    const RT gc = RT(cx_(P)) * g[0] + RT(cy_(P)) * g[1] + RT(cz_(P)) * g[2];
    const RT sym = w * (drho + rho * (RT(4.5) * uc * uc - RT(1.5) * usq));
    const RT asym = w * rho * RT(3) * uc;
    const RT fs = kf * w * (k2 * gc * uc - k3 * gu);
    const RT fa = kf * w * RT(3) * gc;
    if (put) {
        store_pop<ST, RT>(pl.dst(P), n, live ? f[P] - om * (f[P] - sym - asym) + fs + fa : RT(0), kp, P | slt);
        store_pop<ST, RT>(pl.dst(Q), n, live ? f[Q] - om * (f[Q] - sym + asym) + fs - fa : RT(0), kp, Q | slt);
    }
}

template <typename ST, typename RT, typename PL, int... Ps>
__device__ __forceinline__ void collide_pairs(const RT* f, const PL& pl, unsigned n,
                                              RT drho, RT rho, RT ux, RT uy, RT uz, RT usq,
                                              const RT g[3], RT gu, RT om, RT kf, RT k2, RT k3,
                                              const KParams& kp, bool live, bool put, unsigned slt,
                                              std::integer_sequence<int, Ps...>)
{
    (collide_pair<ST, RT, PL, 2 * Ps + 1>(f, pl, n, drho, rho, ux, uy, uz, usq, g, gu, om, kf, k2, k3, kp, live, put,
                                          slt), ...);
}

// ---- fused spreading + stream + collide (Sec. II A, Eqs. 1-8) -----------------------------
// One thread per node, a wavefront over 64 consecutive x (a tile row of the dense layout, or one
// stored row segment of the compact layout); SoA planes f[p*ld + k] of the shifted populations
// f - w, 32-bit storage offsets. A wavefront with no fluid node exits. In a wavefront that has one, every lane stores all
// 28 outputs (zero at solid and open-plane nodes, whose values are never read: pulls from
// solid sources are replaced by bounce-back, open planes are rewritten by the boundary
// kernel), so that each store writes whole cache lines: stores that leave part of a line
// unwritten, as at every wall crossing of a lattice row, measured markedly slower in HBM.
// CLEAR: also clear the coverage counts read here (every lane of the wavefront, whole lines),
// for the map pass that next uses this set of counts
template <typename ST, typename RT, typename PL, bool CLEAR, bool CMP>
__device__ __forceinline__ void stream_collide_node(const PL& pl, const uint32_t* __restrict__ nodeword,
                                                    const MapPlanes<RT>& mp,
                                                    const Gather<RT>* __restrict__ gat,
                                                    const KParams& kp, unsigned* __restrict__ err,
                                                    const NodeAt& at, const SegNb& nb)
{
    // (compact layout: lanes past the row's end hold node word 0, not live)
    const unsigned n = at.k;
    const int y = at.y;
    const uint32_t w = nodeword[n];
    const bool live = (w & NW_FLUID) && !(w & NW_OPEN);
    const unsigned long long lv = __ballot(live);
    if (!lv) return;
    const uint32_t cnum = *at32(mp.cnt, n);
    // A lane stores when its 128-B line (of S-byte elements) holds a fluid node of this
    // wavefront; the 64 lanes hold consecutive nodes.
    const int lane = (int)__lane_id();
    auto line_has_fluid = [&](unsigned S) {
        const int first = lane - (int)((n * S & 127u) / S);
        const int lo = max(first, 0), hi = min(first + (int)(128u / S) - 1, 63);
        const unsigned long long m = (hi == 63 ? ~0ull : (2ull << hi) - 1ull) & ~((1ull << lo) - 1ull);
        return (lv & m) != 0ull;
    };
    // u and sigma are node-interleaved, records that need not divide a line: the window of
    // lanes around this one is then approximate, and a live lane always stores
    using FT = typename PL::FT;
    const bool put_f = line_has_fluid((unsigned)sizeof(ST));
    const bool put_v = live || line_has_fluid(vel_stride<FT>() * (unsigned)sizeof(FT));
    const bool put_s = live || line_has_fluid(6u * (unsigned)sizeof(FT));
    RT f[19];
    if (live) {
        pull_all_fast<ST, RT, CMP>(f, pl, at, nb, kp, std::make_integer_sequence<int, 19>{});
        if (w & 0x7FFFEu) bounce_back<ST, RT>(f, pl, n, w, y, kp, std::make_integer_sequence<int, 19>{});
    } else {
#pragma unroll
        for (int p = 0; p < 19; ++p) f[p] = RT(0);
    }

    RT g[3], theta;
    spread_at<RT, field_mode_of<ST>()>(n, cnum, mp, gat, kp, g, theta);

    // moments of the shifted populations: density excess, momentum, second moments
    RT drho = RT(0), mx = RT(0), my = RT(0), mz = RT(0);
    RT pxx = RT(0), pyy = RT(0), pzz = RT(0), pxy = RT(0), pxz = RT(0), pyz = RT(0);
#pragma unroll
    for (int p = 0; p < 19; ++p) {
        drho += f[p];
        if (cx_(p)) mx += RT(cx_(p)) * f[p];
        if (cy_(p)) my += RT(cy_(p)) * f[p];
        if (cz_(p)) mz += RT(cz_(p)) * f[p];
        if (cx_(p)) pxx += f[p];
        if (cy_(p)) pyy += f[p];
        if (cz_(p)) pzz += f[p];
        if (cx_(p) * cy_(p)) pxy += RT(cx_(p) * cy_(p)) * f[p];
        if (cx_(p) * cz_(p)) pxz += RT(cx_(p) * cz_(p)) * f[p];
        if (cy_(p) * cz_(p)) pyz += RT(cy_(p) * cz_(p)) * f[p];
    }
    const RT rho = RT(1) + drho;
    const RT irho = recip(rho);
    const RT ux = (mx + RT(0.5) * g[0]) * irho;
    const RT uy = (my + RT(0.5) * g[1]) * irho;
    const RT uz = (mz + RT(0.5) * g[2]) * irho;
    const RT usq = ux * ux + uy * uy + uz * uz;
    const RT T = (RT)kp.tau0 + (RT)kp.delta * theta;
    const RT om = recip(T);
    const RT kf = kp.forcing == 1 ? RT(1) : RT(1) - RT(0.5) * om;
    const RT k2 = kp.forcing == 1 ? RT(4.5) : RT(9);      // 1/(2c^4) or 1/c^4
    const RT k3 = kp.forcing == 1 ? RT(1.5) : RT(3);      // c^2/(2c^4) or c^2/c^4
    const RT gu = g[0] * ux + g[1] * uy + g[2] * uz;

    // rest population, then the nine pairs of opposite speeds
    {
        const RT w0 = RT(w_(0));
        const RT fe0 = w0 * (drho - RT(1.5) * rho * usq);
        const RT F0 = -kf * w0 * k3 * gu;
        if (put_f) store_pop<ST, RT>(pl.dst(0), n, live ? f[0] - om * (f[0] - fe0) + F0 : RT(0), kp, at.salt);
    }
    collide_pairs<ST, RT>(f, pl, n, drho, rho, ux, uy, uz, usq, g, gu, om, kf, k2, k3, kp, live, put_f, at.salt,
                          std::make_integer_sequence<int, 9>{});

    // stress of the non-equilibrium part: sigma = -(1 - 1/(2T)) sum c c (f - f^eq), with
    // sum c c f^eq - w = drho/3 delta + rho u u
    const RT ks = -(RT(1) - RT(0.5) * om);
    const RT d3 = drho * RT(1.0 / 3.0);
    const RT z0 = RT(0);
    if (put_v) store_vel_nt(vel_of(pl.u, n), live ? ux : z0, live ? uy : z0, live ? uz : z0);
    if (put_s)
        store_str_nt(str_of(pl.sig, n), live ? ks * (pxx - d3 - rho * ux * ux) : z0,
                     live ? ks * (pyy - d3 - rho * uy * uy) : z0, live ? ks * (pzz - d3 - rho * uz * uz) : z0,
                     live ? ks * (pxy - rho * ux * uy) : z0, live ? ks * (pxz - rho * ux * uz) : z0,
                     live ? ks * (pyz - rho * uy * uz) : z0);
    // (the boundary kernel still reads, and then clears, the counts at the open planes and
    // at the nodes it extrapolates from)
    if (CLEAR && line_has_fluid(4u))
        __builtin_nontemporal_store((w & NW_OPEN_INNER) ? cnum : 0u, at32(mp.cnt, n));
    if (live && (!(rho > RT(0)) || !(usq <= RT(0.09)))) atomicOr(err, ERR_UNSTABLE);
}

// Block -> tile: the hardware deals consecutive blocks to the eight XCDs in turn, so block
// k + 8 t of a grid padded to a multiple of 8 is tile t of XCD k's contiguous share. Each XCD then
// sweeps one range of tiles (four stored segments each, in x, y, z order), and the cache lines
// that neighbouring segments share (the pulls across a segment's x faces) are fetched into one L2.
__device__ __forceinline__ unsigned xcd_tile()
{
    const unsigned per = gridDim.x / 8u;
    return (blockIdx.x % 8u) * per + blockIdx.x / 8u;
}

// one stored segment per wavefront, four per block; the segment's neighbour table is loaded
// once per wavefront into scalar registers
template <typename ST, typename RT, typename PL, bool CLEAR>
__device__ __forceinline__ void stream_collide_segment(const PL& pl, const uint32_t* __restrict__ nodeword,
                                                       const MapPlanes<RT>& mp,
                                                       const Gather<RT>* __restrict__ gat,
                                                       const KParams& kp, unsigned* __restrict__ err,
                                                       const SegTables& tab, int s, unsigned slt)
{
    s = __builtin_amdgcn_readfirstlane(s);
    const int4 sg = tab.seg[s];
    SegNb nb;
    load_segnb(tab.nb, s, nb);
    const NodeAt at{((unsigned)s << 6) | threadIdx.x, sg.x + (int)threadIdx.x, sg.y, sg.z, sg.x, slt};
    stream_collide_node<ST, RT, PL, CLEAR, true>(pl, nodeword, mp, gat, kp, err, at, nb);
}

// compact layout: one stored segment per wavefront, four per block
template <typename ST, typename RT, bool CLEAR>
__global__ __launch_bounds__(256) void k_stream_collide_cmp(
    const Planes<ST, RT> pl, const uint32_t* __restrict__ nodeword, const MapPlanes<RT> mp,
    const Gather<RT>* __restrict__ gat, KParams kp, unsigned* __restrict__ err, const SegTables tab,
    int nseg, unsigned* __restrict__ ctr, int par)
{
    const unsigned t = xcd_tile();
    const unsigned slt = step_salt<ST>(ctr, par, kp, t == 0 && threadIdx.x == 0 && threadIdx.y == 0);
    const int s = (int)t * 4 + (int)threadIdx.y;
    if (s < nseg) stream_collide_segment<ST, RT, Planes<ST, RT>, CLEAR>(pl, nodeword, mp, gat, kp, err, tab, s, slt);
}

// dense layout: tiles of 64 x 4 nodes (a wavefront spans 64 consecutive x). With FP32
// arithmetic the kernel is held to 72 VGPRs, seven wavefronts per SIMD (the 16-bit storages
// gained 3% over six; FP32 storage was unchanged)
template <typename ST, typename RT, bool CLEAR>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(sizeof(RT) == 4 ? 7 : 1))) void k_stream_collide(
    const Planes<ST, RT> pl, const uint32_t* __restrict__ nodeword, const MapPlanes<RT> mp,
    const Gather<RT>* __restrict__ gat, KParams kp, unsigned* __restrict__ err, unsigned nbx,
    unsigned nby, unsigned ntiles, unsigned* __restrict__ ctr, int par)
{
    const unsigned t = xcd_tile();
    if (t >= ntiles) return;
    const unsigned slt = step_salt<ST>(ctr, par, kp, t == 0 && threadIdx.x == 0 && threadIdx.y == 0);
    const unsigned r = t / nbx;
    const int x = (int)(t - r * nbx) * 64 + threadIdx.x;
    const int y = (int)(r % nby) * 4 + threadIdx.y;
    const int z = (int)(r / nby);
    if (x < kp.nx && y < kp.ny) {
        const NodeAt at{(unsigned)x + (unsigned)kp.nx * ((unsigned)y + (unsigned)kp.ny * (unsigned)z), x, y, z, 0,
                        slt};
        stream_collide_node<ST, RT, Planes<ST, RT>, CLEAR, false>(pl, nodeword, mp, gat, kp, err, at, SegNb{});
    }
}

// ---- open z faces: non-equilibrium extrapolation (Guo, Zheng & Shi 2002) ------------------
// planes[q] = (storage index of the plane node, storage index of its inner neighbour along z
// or -1 when that node is solid, x | y << 16, z)
template <typename ST, typename RT>
__global__ __launch_bounds__(256) void k_open_bc(
    const ST* __restrict__ fin, ST* __restrict__ fout, const uint32_t* __restrict__ nodeword,
    const int4* __restrict__ planes, int nplane, const MapPlanes<RT> mp,
    const Gather<RT>* __restrict__ gat, typename FieldOf<ST, RT>::T* __restrict__ uout,
    typename FieldOf<ST, RT>::T* __restrict__ sout, KParams kp,
    const SegTables tab, int clear_counts, unsigned* __restrict__ ctr, int par)
{
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= nplane) return;
    // the step term of this step's stream-collide (which has written only the other word)
    const unsigned slt = step_salt<ST>(ctr, par, kp, false);
    const int4 pq = planes[q];
    const unsigned n = (unsigned)pq.x;
    const int x = pq.z & 0xffff;
    const int z = pq.w;
    const bool inner_fluid = pq.y >= 0;
    const unsigned ni = inner_fluid ? (unsigned)pq.y : n;
    const uint32_t wi = inner_fluid ? nodeword[ni] : 0u;
    const RT rb = z == 0 ? (RT)kp.rho_in : (RT)kp.rho_out;
    RT gb[3], thb;
    const uint32_t cn = mp.cnt[n], cni = inner_fluid ? mp.cnt[ni] : 0u;
    spread_at<RT, field_mode_of<ST>()>(n, cn, mp, gat, kp, gb, thb);
    const RT om = RT(1) / ((RT)kp.tau0 + (RT)kp.delta * thb);
    const RT z0 = RT(0);
    store_str_nt(str_of(sout, n), z0, z0, z0, z0, z0, z0);
    // with clear_counts this thread is the only reader of the counts at n and ni (the inner
    // node of one plane node): it clears them for the next step's map pass once read
    if (clear_counts && cn) mp.cnt[n] = 0u;
    if (!(wi & NW_FLUID)) {
        for (int p = 0; p < 19; ++p)
            store_pop<ST, RT>(fout + (size_t)p * (size_t)kp.ld, (unsigned)n, RT(w_(p)) * (rb - RT(1)), kp,
                              (unsigned)p | slt);
        store_vel_nt(vel_of(uout, n), z0, z0, z0);
        return;
    }
    RT f[19];
    const int y = pq.z >> 16, zi = z == 0 ? 1 : kp.nz - 2;
    if (kp.compact) {
        const int si = (int)(ni >> 6);
        SegNb nb;
        load_segnb(tab.nb, si, nb);
        const NodeAt at{ni, x, y, zi, tab.seg[si].x};
        pull_all<ST, RT, true>(f, fin, at, wi, nb, kp, std::make_integer_sequence<int, 19>{});
    } else {
        const NodeAt at{ni, x, y, zi, 0};
        pull_all<ST, RT, false>(f, fin, at, wi, SegNb{}, kp, std::make_integer_sequence<int, 19>{});
    }
    RT gi[3], thi;
    spread_at<RT, field_mode_of<ST>()>(ni, cni, mp, gat, kp, gi, thi);
    if (clear_counts && cni) mp.cnt[ni] = 0u;
    RT drho = 0, mx = 0, my = 0, mz = 0;
    for (int p = 0; p < 19; ++p) {
        drho += f[p];
        mx += RT(cx_(p)) * f[p];
        my += RT(cy_(p)) * f[p];
        mz += RT(cz_(p)) * f[p];
    }
    const RT rho = RT(1) + drho;
    const RT ux = (mx + RT(0.5) * gi[0]) / rho, uy = (my + RT(0.5) * gi[1]) / rho,
             uz = (mz + RT(0.5) * gi[2]) / rho;
    const RT usq = ux * ux + uy * uy + uz * uz;
    for (int p = 0; p < 19; ++p) {
        const RT feb = feq_shift<RT>(p, rb - RT(1), rb, ux, uy, uz, usq);
        const RT fei = feq_shift<RT>(p, drho, rho, ux, uy, uz, usq);
        store_pop<ST, RT>(fout + (size_t)p * (size_t)kp.ld, (unsigned)n, feb + (RT(1) - om) * (f[p] - fei), kp,
                          (unsigned)p | slt);
    }
    store_vel_nt(vel_of(uout, n), ux, uy, uz);
}

// ---- spread-field probe: g and T per fluid node (same device function as the step) -------
template <typename RT>
__global__ __launch_bounds__(256) void k_spread_field(const uint32_t* __restrict__ nodeword,
                                                      const MapPlanes<RT> mp,
                                                      const Gather<RT>* __restrict__ gat,
                                                      RT* __restrict__ gout, RT* __restrict__ tout,
                                                      KParams kp)
{
    const long long n = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= kp.N) return;
    const uint32_t w = nodeword[n];
    if (!(w & NW_FLUID)) {
        gout[n] = gout[kp.ld + n] = gout[2 * kp.ld + n] = RT(0);
        tout[n] = (RT)kp.tau0;
        return;
    }
    RT g[3], th;
    spread_at<RT, -1>((unsigned)n, mp.cnt[n], mp, gat, kp, g, th);
    gout[n] = g[0];
    gout[kp.ld + n] = g[1];
    gout[2 * kp.ld + n] = g[2];
    tout[n] = (RT)kp.tau0 + (RT)kp.delta * th;
}

// ---- coverage counts: clear one set, and the count of the map pass's overflow list ----------
__global__ __launch_bounds__(256) void k_clear_counts(uint32_t* __restrict__ cnt, long long N,
                                                      int* __restrict__ ovf)
{
    const long long n = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (n == 0 && ovf) ovf[0] = 0;
    if (n < N && cnt[n]) cnt[n] = 0u;
}

// ---- FP64 reductions: mass, momentum, summed u_z (two passes, fixed order) --------------
template <typename ST, typename RT>
__global__ __launch_bounds__(256) void k_observe_partials(const ST* __restrict__ f,
                                                          const uint32_t* __restrict__ nodeword,
                                                          const void* __restrict__ u, KParams kp,
                                                          double* __restrict__ partials)
{
    double acc[6] = {0, 0, 0, 0, 0, 0};   // mass, px, py, pz, sum uz, n_fluid
    for (long long n = (long long)blockIdx.x * blockDim.x + threadIdx.x; n < kp.N;
         n += (long long)gridDim.x * blockDim.x) {
        if (!(nodeword[n] & NW_FLUID)) continue;
        double m = 0, px = 0, py = 0, pz = 0;
        for (int p = 0; p < 19; ++p) {
            const double v = (double)Store<ST, RT>::ld(f + (size_t)p * (size_t)kp.ld, (unsigned)n, kp.f16_inv);
            m += v;
            px += cx_(p) * v;
            py += cy_(p) * v;
            pz += cz_(p) * v;
        }
        acc[0] += 1.0 + m;
        acc[1] += px;
        acc[2] += py;
        acc[3] += pz;
        RT un[3];
        load_vel<RT>(u, (unsigned)n, kp, un);
        acc[4] += (double)un[2];
        acc[5] += 1.0;
    }
    __shared__ double red[6][256];
    for (int a = 0; a < 6; ++a) red[a][threadIdx.x] = acc[a];
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s)
            for (int a = 0; a < 6; ++a) red[a][threadIdx.x] += red[a][threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0)
        for (int a = 0; a < 6; ++a) partials[(long long)a * gridDim.x + blockIdx.x] = red[a][0];
}

__global__ void k_observe_final(const double* __restrict__ partials, int nblk, double* __restrict__ out)
{
    // one thread per quantity, fixed order
    const int a = threadIdx.x;
    if (a < 6) {
        double s = 0;
        for (int b = 0; b < nblk; ++b) s += partials[(long long)a * nblk + b];
        out[a] = s;
    }
}

// ---- wall shear stress at wall-adjacent nodes (FP64) ----------------------------------------
template <typename RT>
__global__ __launch_bounds__(256) void k_wss(const void* __restrict__ sig,
                                             const long long* __restrict__ wn_node,
                                             const double* __restrict__ wn_nrm, int nwn, KParams kp,
                                             double* __restrict__ wss, double* __restrict__ acc,
                                             int accumulate)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= nwn) return;
    const long long n = wn_node[k];
    double s[6];
    RT sv[6];
    load_str<RT>(sig, (unsigned)n, kp, sv);
    for (int a = 0; a < 6; ++a) s[a] = (double)sv[a];
    const double n0 = wn_nrm[3 * k], n1 = wn_nrm[3 * k + 1], n2 = wn_nrm[3 * k + 2];
    const double t0 = s[0] * n0 + s[3] * n1 + s[4] * n2;
    const double t1 = s[3] * n0 + s[1] * n1 + s[5] * n2;
    const double t2 = s[4] * n0 + s[5] * n1 + s[2] * n2;
    const double tn = t0 * n0 + t1 * n1 + t2 * n2;
    const double r0 = t0 - tn * n0, r1 = t1 - tn * n1, r2 = t2 - tn * n2;
    const double v = sqrt(r0 * r0 + r1 * r1 + r2 * r2);
    if (wss) wss[k] = v;
    if (accumulate) acc[k] += v;
}

// ---- fused multi-lattice versions of the per-node stages -------------------------------------
template <typename RT>
__device__ __forceinline__ MapPlanes<RT> map_planes_dev(const int* ids, const void* vals, uint32_t* cnt,
                                                        const KParams& kp)
{
    MapPlanes<RT> mp;
#pragma unroll
    for (int k = 0; k < CAP_MAX; ++k) mp.ids[k] = ids + (k < kp.cap ? (size_t)k * (size_t)kp.ld : 0);
    mp.vals0 = vals;
    mp.cnt = cnt;
    return mp;
}

__global__ __launch_bounds__(256) void kf_clear(const FusedArgs fa)
{
    int lb;
    const SlotDesc& d = *fa.slot[fused_slot(fa, lb)];
    const long long n = (long long)lb * 256 + threadIdx.x;
    if (n == 0) d.b.ovf[0] = 0;
    if (n < d.kp.N && d.b.cnt[n]) d.b.cnt[n] = 0u;
}

template <typename ST, typename RT>
__global__ __launch_bounds__(256) void kf_stream(const FusedArgs fa)
{
    // XCD-contiguous shares of the blocks, as in k_stream_collide (the grid is padded to 8)
    const unsigned t = xcd_tile();
    if (t >= (unsigned)fa.start[fa.n]) return;
    int lb;
    const int sl = fused_slot_at(fa, (int)t, lb);
    const SlotDesc& d = *fa.slot[sl];
    const KParams kp = d.kp;
    const bool odd = (fa.parity >> sl) & 1ull;
    using FT = typename FieldOf<ST, RT>::T;
    const PlanesLd<ST, RT> pl{(const ST*)(odd ? d.fB : d.fA), (ST*)(odd ? d.fA : d.fB), (FT*)d.b.u,
                              (FT*)d.b.sig, (unsigned long long)kp.ld};
    const MapPlanes<RT> mp = map_planes_dev<RT>(d.b.map_ids, d.b.map_vals, d.b.cnt, kp);
    const unsigned slt = step_salt<ST>(d.b.step_ctr, odd ? 1 : 0, kp, lb == 0 && threadIdx.x == 0 && threadIdx.y == 0);
    if (kp.compact) {
        // four stored segments per block, one per wavefront
        const int s = lb * 4 + (int)threadIdx.y;
        if ((long long)s * 64 < kp.N)
            stream_collide_segment<ST, RT, PlanesLd<ST, RT>, true>(pl, d.b.nodeword, mp, (const Gather<RT>*)d.b.gat,
                                                                   kp, d.b.err, d.b.tab, s, slt);
        return;
    }
    // dense layout: flat node order (no idle lanes on lattices narrower than, or not a multiple
    // of, 64)
    const unsigned n = (unsigned)lb * 256u + threadIdx.y * 64u + threadIdx.x;
    if (n >= (unsigned)kp.N) return;
    const unsigned nxy = (unsigned)kp.nx * (unsigned)kp.ny;
    const int z = (int)(n / nxy), rem = (int)(n - (unsigned)z * nxy);
    const int y = rem / kp.nx, x = rem - y * kp.nx;
    const NodeAt at{n, x, y, z, 0, slt};
    stream_collide_node<ST, RT, PlanesLd<ST, RT>, true, false>(pl, d.b.nodeword, mp, (const Gather<RT>*)d.b.gat,
                                                               kp, d.b.err, at, SegNb{});
}

// ---- launchers ---------------------------------------------------------------------------------
template <typename ST, typename RT>
void launch_stream_collide(const void* fin, void* fout, const uint32_t* nodeword, const int* ids,
                           const void* vals, uint32_t* cnt, const void* gat, void* u, void* sig,
                           const KParams& kp, unsigned* err, bool clear_counts, const SegTables& tab,
                           int nseg, unsigned* ctr, int par, hipStream_t st)
{
    if (kp.compact && nseg <= 0) return;
    Planes<ST, RT> pl;
    const size_t ld = (size_t)kp.ld;
    for (int p = 0; p < 19; ++p) {
        pl.in[p] = (const ST*)fin + p * ld;
        pl.out[p] = (ST*)fout + p * ld;
    }
    pl.u = (typename Planes<ST, RT>::FT*)u;
    pl.sig = (typename Planes<ST, RT>::FT*)sig;
    const auto mp = map_planes<RT>(ids, vals, cnt, kp);
    const Gather<RT>* g = (const Gather<RT>*)gat;
    if (kp.compact) {
        const dim3 grid(((unsigned)((nseg + 3) / 4) + 7u) / 8u * 8u);
        if (clear_counts)
            hipLaunchKernelGGL((k_stream_collide_cmp<ST, RT, true>), grid, dim3(64, 4, 1), 0, st, pl, nodeword, mp, g,
                               kp, err, tab, nseg, ctr, par);
        else
            hipLaunchKernelGGL((k_stream_collide_cmp<ST, RT, false>), grid, dim3(64, 4, 1), 0, st, pl, nodeword, mp,
                               g, kp, err, tab, nseg, ctr, par);
        return;
    }
    const unsigned nbx = (unsigned)((kp.nx + 63) / 64), nby = (unsigned)((kp.ny + 3) / 4);
    const unsigned ntiles = nbx * nby * (unsigned)kp.nz;
    const dim3 grid((ntiles + 7u) / 8u * 8u);
    if (clear_counts)
        hipLaunchKernelGGL((k_stream_collide<ST, RT, true>), grid, dim3(64, 4, 1), 0, st, pl, nodeword, mp, g, kp,
                           err, nbx, nby, ntiles, ctr, par);
    else
        hipLaunchKernelGGL((k_stream_collide<ST, RT, false>), grid, dim3(64, 4, 1), 0, st, pl, nodeword, mp, g, kp,
                           err, nbx, nby, ntiles, ctr, par);
}

template <typename ST, typename RT>
void launch_open_bc(const void* fin, void* fout, const uint32_t* nodeword, const int4* planes,
                    int nplane, const int* ids, const void* vals, uint32_t* cnt, const void* gat, void* u,
                    void* sig, const KParams& kp, const SegTables& tab, bool clear_counts, unsigned* ctr,
                    int par, hipStream_t st)
{
    if (nplane <= 0) return;
    hipLaunchKernelGGL((k_open_bc<ST, RT>), dim3((nplane + 255) / 256), dim3(256), 0, st,
                       (const ST*)fin, (ST*)fout, nodeword, planes, nplane,
                       map_planes<RT>(ids, vals, cnt, kp), (const Gather<RT>*)gat,
                       (typename FieldOf<ST, RT>::T*)u, (typename FieldOf<ST, RT>::T*)sig, kp,
                       tab, clear_counts ? 1 : 0, ctr, par);
}

template <typename RT>
void launch_spread_field(const uint32_t* nodeword, const int* ids, const void* vals, uint32_t* cnt,
                         const void* gat, void* g, void* t, const KParams& kp, hipStream_t st)
{
    const unsigned blocks = (unsigned)((kp.N + 255) / 256);
    hipLaunchKernelGGL((k_spread_field<RT>), dim3(blocks), dim3(256), 0, st, nodeword,
                       map_planes<RT>(ids, vals, cnt, kp), (const Gather<RT>*)gat, (RT*)g, (RT*)t, kp);
}

void launch_clear_counts(uint32_t* cnt, long long N, int* ovf, hipStream_t st)
{
    hipLaunchKernelGGL(k_clear_counts, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, st,
                       cnt, N, ovf);
}

template <typename ST, typename RT>
void launch_observe(const void* f, const uint32_t* nodeword, const void* u, const KParams& kp,
                    double* partials, int nblk, double* out, hipStream_t st)
{
    hipLaunchKernelGGL((k_observe_partials<ST, RT>), dim3(nblk), dim3(256), 0, st, (const ST*)f,
                       nodeword, u, kp, partials);
    hipLaunchKernelGGL(k_observe_final, dim3(1), dim3(64), 0, st, partials, nblk, out);
}

template <typename RT>
void launch_wss(const void* sig, const long long* wn_node, const double* wn_nrm, int nwn,
                const KParams& kp, double* wss, double* acc, int accumulate, hipStream_t st)
{
    if (nwn <= 0) return;
    hipLaunchKernelGGL((k_wss<RT>), dim3((nwn + 255) / 256), dim3(256), 0, st, sig,
                       wn_node, wn_nrm, nwn, kp, wss, acc, accumulate);
}

template <typename ST, typename RT>
void launch_fused_lattice(const FusedArgs& fa, int stage, hipStream_t st)
{
    const unsigned g = (unsigned)fa.start[fa.n];
    if (g == 0) return;
    if (stage == FS_CLEAR) hipLaunchKernelGGL(kf_clear, dim3(g), dim3(256), 0, st, fa);
    if (stage == FS_STREAM) hipLaunchKernelGGL((kf_stream<ST, RT>), dim3((g + 7u) / 8u * 8u), dim3(64, 4, 1), 0, st, fa);
}

#define INST_ST(ST, RT)                                                                           \
    template void launch_fused_lattice<ST, RT>(const FusedArgs&, int, hipStream_t);               \
    template void launch_stream_collide<ST, RT>(const void*, void*, const uint32_t*, const int*,  \
                                                const void*, uint32_t*, const void*, void*, void*, \
                                                const KParams&, unsigned*, bool, const SegTables&, \
                                                int, unsigned*, int, hipStream_t);                \
    template void launch_open_bc<ST, RT>(const void*, void*, const uint32_t*, const int4*,        \
                                         int, const int*, const void*, uint32_t*, const void*,    \
                                         void*, void*,                                            \
                                         const KParams&, const SegTables&, bool, unsigned*, int,  \
                                         hipStream_t);                                            \
    template void launch_observe<ST, RT>(const void*, const uint32_t*, const void*,               \
                                         const KParams&, double*, int, double*, hipStream_t);
INST_ST(double, double)
INST_ST(float, float)
INST_ST(bf16_t, float)
INST_ST(_Float16, float)
template void launch_spread_field<double>(const uint32_t*, const int*, const void*, uint32_t*,
                                          const void*, void*, void*, const KParams&, hipStream_t);
template void launch_spread_field<float>(const uint32_t*, const int*, const void*, uint32_t*,
                                         const void*, void*, void*, const KParams&, hipStream_t);
template void launch_wss<double>(const void*, const long long*, const double*, int,
                                 const KParams&, double*, double*, int, hipStream_t);
template void launch_wss<float>(const void*, const long long*, const double*, int,
                                const KParams&, double*, double*, int, hipStream_t);

}  // namespace lbrbc
