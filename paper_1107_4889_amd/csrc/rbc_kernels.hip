// rbc_kernels.hip -- per-cell kernels (gfx950): rigid-body halves, cell list, node->cell
// coverage map, interpolation onto the cells, Gay-Berne forces.
#include <climits>

#include "lbrbc_device.h"
#include "lbrbc_internal.h"

namespace lbrbc {

__device__ __forceinline__ void mat_vec(const double* M, const double* v, double* o)
{
    for (int r = 0; r < 3; ++r) o[r] = M[3 * r] * v[0] + M[3 * r + 1] * v[1] + M[3 * r + 2] * v[2];
}
__device__ __forceinline__ void matT_vec(const double* M, const double* v, double* o)
{
    for (int c = 0; c < 3; ++c) o[c] = M[c] * v[0] + M[3 + c] * v[1] + M[6 + c] * v[2];
}
__device__ __forceinline__ void cross3(const double* a, const double* b, double* o)
{
    o[0] = a[1] * b[2] - a[2] * b[1];
    o[1] = a[2] * b[0] - a[0] * b[2];
    o[2] = a[0] * b[1] - a[1] * b[0];
}

__device__ __forceinline__ double box_len(const KParams& kp, int a)
{
    return a == 0 ? (double)kp.nx : (a == 1 ? (double)kp.ny : (double)kp.nz);
}

// ---- S1: rigid-body first half (App. A, steps 1-4) ------------------------------------------
// half kick, half-step friction, drift (wrapped on periodic axes), five free sub-rotations
// n/2, t/2, g, t/2, n/2 about the body axes: Rot = Rot_k(-f h Omega_k), pi <- Rot pi,
// Q <- Q Rot^T (Q' = Q hat(Omega)).
__device__ __forceinline__ void rb1_cell(RbcState* __restrict__ st, const KParams& kp, int i)
{
    RbcState s = st[i];
    const double eT = exp(-kp.gammaT * 0.5), eR = exp(-kp.gammaR * 0.5);
    for (int a = 0; a < 3; ++a) {
        s.V[a] += 0.5 / kp.mass * s.Fc[a];
        s.Om[a] += 0.5 * s.Tc[a] / kp.inertia[a];
    }
    for (int a = 0; a < 3; ++a) {
        s.V[a] *= eT;
        s.Om[a] *= eR;
    }
    for (int a = 0; a < 3; ++a) {
        s.R[a] += s.V[a];
        if (kp.per[a]) {
            const double L = box_len(kp, a);
            if (s.R[a] >= L) s.R[a] -= L;
            else if (s.R[a] < 0.0) s.R[a] += L;
        }
    }
    const int seq[5] = {0, 1, 2, 1, 0};
    const double frac[5] = {0.5, 0.5, 1.0, 0.5, 0.5};
    for (int stp = 0; stp < 5; ++stp) {
        const int k = seq[stp];
        const double phi = frac[stp] * s.Om[k];
        double c, sn;
        sincos(-phi, &sn, &c);
        double M[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
        if (k == 0) { M[0] = 1; M[4] = c; M[5] = -sn; M[7] = sn; M[8] = c; }
        if (k == 1) { M[4] = 1; M[0] = c; M[2] = sn; M[6] = -sn; M[8] = c; }
        if (k == 2) { M[8] = 1; M[0] = c; M[1] = -sn; M[3] = sn; M[4] = c; }
        double pi[3], pn[3], Qn[9];
        for (int a = 0; a < 3; ++a) pi[a] = kp.inertia[a] * s.Om[a];
        mat_vec(M, pi, pn);
        for (int a = 0; a < 3; ++a) s.Om[a] = pn[a] / kp.inertia[a];
        for (int r = 0; r < 3; ++r)
            for (int cc = 0; cc < 3; ++cc)
                Qn[3 * r + cc] = s.Q[3 * r] * M[3 * cc] + s.Q[3 * r + 1] * M[3 * cc + 1] +
                                 s.Q[3 * r + 2] * M[3 * cc + 2];
        for (int a = 0; a < 9; ++a) s.Q[a] = Qn[a];
    }
    for (int a = 0; a < 3; ++a) {
        s.Vh[a] = s.V[a];
        s.Omh[a] = s.Om[a];
    }
    st[i] = s;
}


// ---- S2: cell list (counting sort, ids ascending per cell) --------------------------------
__device__ __forceinline__ int cell_coord(const KParams& kp, int a, double x)
{
    int c = (int)floor(x / kp.cedge[a]);
    if (c < 0) c = 0;
    if (c >= kp.ncell[a]) c = kp.ncell[a] - 1;
    return c;
}

__device__ __forceinline__ void bin_cell(const RbcState* __restrict__ st, int* cellid, int* cnt,
                                         const KParams& kp, int i)
{
    const double* R = st[i].R;
    const int c = cell_coord(kp, 0, R[0]) +
                  kp.ncell[0] * (cell_coord(kp, 1, R[1]) + kp.ncell[1] * cell_coord(kp, 2, R[2]));
    cellid[i] = c;
    atomicAdd(cnt + c, 1);
}

__global__ __launch_bounds__(256) void k_cells_bin(const RbcState* __restrict__ st, int* cellid,
                                                   int* cnt, KParams kp)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < kp.nrbc) bin_cell(st, cellid, cnt, kp, i);
}

// first half of the rigid-body step and binning of the moved centre, per cell; also clears
// the overflow count of this step's map pass
__global__ __launch_bounds__(256) void k_rb1_bin(RbcState* __restrict__ st, int* cellid, int* cnt,
                                                 int* ovf, KParams kp)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i == 0) ovf[0] = 0;
    if (i >= kp.nrbc) return;
    rb1_cell(st, kp, i);
    bin_cell(st, cellid, cnt, kp, i);
}

// Exclusive scan of the cell counts (also clears them). One round covers SCAN_CHUNK entries
// from `base` (SCAN_THREADS threads, four consecutive entries each, so the loads are
// coalesced), offset by `carry`; it writes the offsets, clears the counts and returns the
// round's total. Blocks of 256 threads find room beside the concurrent stream-collide.
constexpr int SCAN_THREADS = 256;
constexpr int SCAN_WAVES = SCAN_THREADS / 64;
constexpr int SCAN_CHUNK = 4 * SCAN_THREADS;
static_assert(SCAN_CHUNK == CELL_SCAN_CHUNK, "the arena sizes the chunk totals by CELL_SCAN_CHUNK");
constexpr int SCAN_SINGLE_BLOCK_CHUNKS = 2;

__device__ __forceinline__ int scan_round(int* cnt, int* off, int base, int n, int carry,
                                          int* wsum)
{
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    const int i0 = base + 4 * t;
    int v[4];
    if (i0 + 3 < n) {
        const int4 q = *reinterpret_cast<const int4*>(cnt + i0);
        v[0] = q.x;
        v[1] = q.y;
        v[2] = q.z;
        v[3] = q.w;
    } else {
        for (int j = 0; j < 4; ++j) v[j] = i0 + j < n ? cnt[i0 + j] : 0;
    }
    const int sum = v[0] + v[1] + v[2] + v[3];
    int incl = sum;
    for (int o = 1; o < 64; o <<= 1) {
        const int y = __shfl_up(incl, o, 64);
        if (lane >= o) incl += y;
    }
    if (lane == 63) wsum[w] = incl;
    __syncthreads();
    int before = 0, round = 0;
    for (int k = 0; k < SCAN_WAVES; ++k) {
        const int x = wsum[k];
        before += k < w ? x : 0;
        round += x;
    }
    int ex = carry + before + incl - sum;
    for (int j = 0; j < 4; ++j) {
        if (i0 + j < n) {
            off[i0 + j] = ex;
            cnt[i0 + j] = 0;
        }
        ex += v[j];
    }
    __syncthreads();   // wsum is reused by the next round
    return round;
}

// the whole scan in one block, round after round (small cell grids and the fused launches)
__device__ __forceinline__ void scan_clear_block(int* cnt, int* off, int n)
{
    __shared__ int wsum[SCAN_WAVES];
    int carry = 0;
    for (int base = 0; base < n; base += SCAN_CHUNK) carry += scan_round(cnt, off, base, n, carry, wsum);
    if (threadIdx.x == 0) off[n] = carry;
}

__global__ __launch_bounds__(SCAN_THREADS) void k_scan_clear(int* cnt, int* off, int n)
{
    scan_clear_block(cnt, off, n);
}

// Large cell grids: one block per chunk of SCAN_CHUNK counts. First the chunk totals ...
__global__ __launch_bounds__(SCAN_THREADS) void k_scan_partials(const int* __restrict__ cnt,
                                                        int* __restrict__ part, int n)
{
    __shared__ int wsum[SCAN_WAVES];
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    const int i0 = (int)blockIdx.x * SCAN_CHUNK + 4 * t;
    int v = 0;
    for (int j = 0; j < 4; ++j) v += i0 + j < n ? cnt[i0 + j] : 0;
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
    if (lane == 0) wsum[w] = v;
    __syncthreads();
    if (t == 0) {
        int tot = 0;
        for (int k = 0; k < SCAN_WAVES; ++k) tot += wsum[k];
        part[blockIdx.x] = tot;
    }
}

// ... then each chunk's scan, offset by the totals of the chunks before it (the last block
// writes off[n])
__global__ __launch_bounds__(SCAN_THREADS) void k_scan_chunks(int* cnt, int* off, const int* __restrict__ part,
                                                      int n)
{
    __shared__ int wsum[SCAN_WAVES];
    __shared__ int carry_s;
    const int b = (int)blockIdx.x, t = threadIdx.x;
    if (t < 64) {
        int c = 0;
        for (int k = t; k < b; k += 64) c += part[k];
        for (int o = 32; o > 0; o >>= 1) c += __shfl_down(c, o, 64);
        if (t == 0) carry_s = c;
    }
    __syncthreads();
    const int carry = carry_s;
    const int round = scan_round(cnt, off, b * SCAN_CHUNK, n, carry, wsum);
    if (t == 0 && b == (int)gridDim.x - 1) off[n] = carry + round;
}

__device__ __forceinline__ void scatter_cell(const int* __restrict__ cellid,
                                             const int* __restrict__ off, int* fill, int* ids, int i)
{
    const int c = cellid[i];
    ids[off[c] + atomicAdd(fill + c, 1)] = i;
}

__global__ __launch_bounds__(256) void k_cells_scatter(const int* __restrict__ cellid,
                                                       const int* __restrict__ off, int* fill,
                                                       int* ids, int nrbc)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < nrbc) scatter_cell(cellid, off, fill, ids, i);
}

// ids of grid cell c in ascending order (insertion sort of the short list); the fill
// counter of the cell is cleared for the next build
__device__ __forceinline__ void sort_cell(const int* __restrict__ off, int* ids, int* fill, int c)
{
    fill[c] = 0;
    const int b = off[c], e = off[c + 1];
    for (int k = b + 1; k < e; ++k) {
        const int v = ids[k];
        int j = k - 1;
        while (j >= b && ids[j] > v) {
            ids[j + 1] = ids[j];
            --j;
        }
        ids[j + 1] = v;
    }
}

__global__ __launch_bounds__(256) void k_cells_sort(const int* __restrict__ off, int* ids, int* fill,
                                                    int ncells)
{
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c < ncells) sort_cell(off, ids, fill, c);
}

// ---- support tile of one cell --------------------------------------------------------------
// The support |y_a| < xi_a lies within |x_a - R_a| < ext_a = sum_b |Q_ab| xi_b; the tile adds
// one node on each side (the halo of the central-difference gradient).
struct Tile {
    int lo[3], sz[3];
};

__device__ __forceinline__ void support_tile(const RbcState& s, const KParams& kp, Tile& t)
{
    for (int a = 0; a < 3; ++a) {
        const double ext = fabs(s.Q[3 * a]) * kp.xi[0] + fabs(s.Q[3 * a + 1]) * kp.xi[1] +
                           fabs(s.Q[3 * a + 2]) * kp.xi[2];
        const int lo = (int)floor(s.R[a] - ext) - 1;
        const int hi = (int)ceil(s.R[a] + ext) + 1;
        t.lo[a] = lo;
        t.sz[a] = hi - lo + 1;
    }
}

// wrap a tile coordinate into the box (a tile is never longer than a periodic axis);
// returns false outside a non-periodic face
__device__ __forceinline__ bool wrap_coord(int& X, int L, int per)
{
    const bool lo = X < 0, hi = X >= L;
    X = (per && lo) ? X + L : ((per && hi) ? X - L : X);
    return per || !(lo || hi);
}

// Nodes of tile row (ty, tz) that may lie inside the support. The body coordinates are affine
// in x along the row, y_a = Q_xa d_x + b_a, and |y_a| < xi_a cuts an open interval (xa, xb) of
// d_x. Every node that the exact FP64 test can find inside lies strictly within
// (xa - ROW_EPS, xb + ROW_EPS): ROW_EPS is far above the rounding of either computation (a few
// ulps of coordinates below 2^11). The range is [lo, hi] in tile coordinates, empty when lo > hi.
constexpr double ROW_EPS = 1e-7;
// iq[a] = 1 / Q_xa (0 where |Q_xa| <= 1e-12), computed once per cell: a product differs from the
// quotient by an ulp, far below ROW_EPS
__device__ __forceinline__ void support_row(const RbcState& s, const KParams& kp, const Tile& T, const double* iq,
                                            int ty, int tz, int& lo, int& hi)
{
    const double dy = (double)(T.lo[1] + ty) - s.R[1], dz = (double)(T.lo[2] + tz) - s.R[2];
    double xa = -1e30, xb = 1e30;
    for (int a = 0; a < 3; ++a) {
        const double qa = s.Q[a], b = s.Q[3 + a] * dy + s.Q[6 + a] * dz;
        if (fabs(qa) > 1e-12) {
            double u0 = (-kp.xi[a] - b) * iq[a], u1 = (kp.xi[a] - b) * iq[a];
            if (u0 > u1) { const double t_ = u0; u0 = u1; u1 = t_; }
            xa = fmax(xa, u0);
            xb = fmin(xb, u1);
        } else if (fabs(b) >= kp.xi[a] + 1e-9) {
            xa = 1e30;
        }
    }
    lo = T.sz[0];
    hi = -1;
    if (xa <= xb) {
        const double X0 = s.R[0] - (double)T.lo[0];
        lo = max(0, (int)floor(X0 + xa - ROW_EPS) + 1);
        hi = min(T.sz[0] - 1, (int)ceil(X0 + xb + ROW_EPS) - 1);
    }
}

// Covered x-range of tile row r from the support ranges of the rows: a node is covered when it
// or one of its six axis neighbours is inside, so the row's own range widened by one node and
// the ranges of its four neighbouring rows. Empty rows (lo > hi) add nothing.
__device__ __forceinline__ void covered_row(const short* rlo, const short* rhi, int r, int sx, int sy, int sz,
                                            int& lo, int& hi)
{
    const int ty = r % sy, tz = r / sy;
    lo = sx;
    hi = -1;
    if (rlo[r] <= rhi[r]) {
        lo = rlo[r] - 1;
        hi = rhi[r] + 1;
    }
    if (ty > 0) { lo = min(lo, (int)rlo[r - 1]); hi = max(hi, (int)rhi[r - 1]); }
    if (ty + 1 < sy) { lo = min(lo, (int)rlo[r + 1]); hi = max(hi, (int)rhi[r + 1]); }
    if (tz > 0) { lo = min(lo, (int)rlo[r - sy]); hi = max(hi, (int)rhi[r - sy]); }
    if (tz + 1 < sz) { lo = min(lo, (int)rlo[r + sy]); hi = max(hi, (int)rhi[r + sy]); }
    lo = max(lo, 0);
    hi = min(hi, sx - 1);
}

// block index -> position in the spatially sorted cell order, so that each XCD (blocks are
// dealt to the eight XCDs round-robin) works on one contiguous, spatially compact chunk and
// its L2 keeps the shared lattice lines; the grid is a multiple of 8 blocks
__device__ __forceinline__ int xcd_chunk_index(int units_per_block)
{
    const int per = gridDim.x / 8;
    const int blk = (blockIdx.x % 8) * per + blockIdx.x / 8;
    return blk * units_per_block;
}

constexpr int MC_THREADS = 256;

// F^hyd, T^hyd and the gather record of a cell from its interpolation sums (defined with S6)
template <typename RT>
__device__ __forceinline__ void hydro_cell(const RbcState& s, RbcCouple& c, const KParams& kp,
                                           Gather<RT>* __restrict__ gi);
constexpr int TILE_ROWS_MAX = 20 * 20;   // tile_max <= 20

// ---- S3 + S4: coverage map and interpolation, one block per cell ------------------------
// Pass 1 over the support tile: exact FP64 support test and the unnormalised kernel raw(x)
// on fluid nodes; S = sum raw. Pass 2: every covered node (fluid, and inside or next to an
// inside node) takes a coverage slot and stores (cell id; raw, grad raw by central
// differences), which the per-node spreading reads, and adds to the interpolation sums
// (Eqs. 16-21) with dhat = raw / S:
//   u~  = sum over inside nodes of dhat u,
//   w~  = sum over inside nodes of dhat (curl u) = sum over covered nodes of u x grad dhat
//         (summation by parts of the central-difference curl, exact with u = 0 on solid
//         nodes; it needs u only at the node itself),
//   T^S = alpha sum over inside nodes of dhat (sigma . n^) x (x - R), n^ = grad/|grad|.
template <typename RT>
__device__ void map_couple_tile(int i, unsigned char* smem, const RbcState* __restrict__ st,
                                RbcCouple* __restrict__ cp, Gather<RT>* __restrict__ gat,
                                const uint32_t* __restrict__ nodeword, const int* __restrict__ segmap,
                                uint32_t* __restrict__ cnt,
                                int* __restrict__ ids, void* __restrict__ vals,
                                const void* __restrict__ u, const void* __restrict__ sig,
                                const KParams& kp, unsigned* __restrict__ err)
{
    const int tm = kp.tile_max;
    const unsigned t3 = (unsigned)(tm * tm * tm);
    RT* raw = reinterpret_cast<RT*>(smem);
    unsigned char* flag = smem + (size_t)t3 * sizeof(RT);  // 1 inside, 2 fluid
    unsigned short* list = reinterpret_cast<unsigned short*>(smem + (((size_t)t3 * (sizeof(RT) + 1) + 1) & ~(size_t)1));
    __shared__ Tile T;
    __shared__ RT red[MC_THREADS / 64][10];
    __shared__ int wcnt[MC_THREADS / 64];
    __shared__ short rlo[TILE_ROWS_MAX], rhi[TILE_ROWS_MAX], clo[TILE_ROWS_MAX], chi[TILE_ROWS_MAX];
    const RbcState& s = st[i];
    const int tid = threadIdx.x;
    if (tid == 0) support_tile(s, kp, T);
    __syncthreads();
    if (T.sz[0] > tm || T.sz[1] > tm || T.sz[2] > tm) {
        if (tid == 0) atomicOr(err, ERR_CAPACITY);
        return;
    }
    const unsigned sx = T.sz[0], sy = T.sz[1], sz = T.sz[2], sxy = sx * sy, total = sxy * sz;
    const unsigned rows = sy * sz;
    // support range of each tile row (the exact test below decides each node; the ranges only
    // skip nodes that are certainly outside), then the covered range of each row
    double iq[3];
    for (int a = 0; a < 3; ++a) iq[a] = fabs(s.Q[a]) > 1e-12 ? 1.0 / s.Q[a] : 0.0;
    for (unsigned r = tid; r < rows; r += MC_THREADS) {
        int lo, hi;
        support_row(s, kp, T, iq, (int)(r % sy), (int)(r / sy), lo, hi);
        rlo[r] = (short)lo;
        rhi[r] = (short)hi;
    }
    __syncthreads();
    for (unsigned r = tid; r < rows; r += MC_THREADS) {
        int lo, hi;
        covered_row(rlo, rhi, (int)r, (int)sx, (int)sy, (int)sz, lo, hi);
        clo[r] = (short)lo;
        chi[r] = (short)hi;
    }
    __syncthreads();
    const RT s0 = RT(2.0 / kp.xi[0]), s1 = RT(2.0 / kp.xi[1]), s2 = RT(2.0 / kp.xi[2]);
    RT part = RT(0);
#pragma unroll 4
    for (unsigned t = tid; t < total; t += MC_THREADS) {
        const unsigned row = t / sx, tx = t - row * sx;
        const unsigned tz = row / sy, ty = row - tz * sy;
        int X = T.lo[0] + (int)tx, Y = T.lo[1] + (int)ty, Z = T.lo[2] + (int)tz;
        const bool ok = (int)tx >= clo[row] && (int)tx <= chi[row] && wrap_coord(X, kp.nx, kp.per[0]) &&
                        wrap_coord(Y, kp.ny, kp.per[1]) && wrap_coord(Z, kp.nz, kp.per[2]);
        unsigned char fl = 0;
        RT r = RT(0);
        const int kst = ok ? storage_of(segmap, kp, X, Y, Z) : -1;
        if (kst >= 0 && (nodeword[kst] & NW_FLUID)) {
            fl = 2;
            double y[3];
            const double d0 = min_img((double)X - s.R[0], (double)kp.nx, kp.per[0]);
            const double d1 = min_img((double)Y - s.R[1], (double)kp.ny, kp.per[1]);
            const double d2 = min_img((double)Z - s.R[2], (double)kp.nz, kp.per[2]);
            body_coords_exact(s.Q, d0, d1, d2, y);
            if (fabs(y[0]) < kp.xi[0] && fabs(y[1]) < kp.xi[1] && fabs(y[2]) < kp.xi[2]) {
                fl = 3;
                r = peskin((RT)y[0] * s0) * peskin((RT)y[1] * s1) * peskin((RT)y[2] * s2);
            }
        }
        raw[t] = r;
        flag[t] = fl;
        part += r;
    }
    // S: wave shuffles, then the four waves in order
    for (int o = 32; o > 0; o >>= 1) part += __shfl_down(part, o, 64);
    if ((tid & 63) == 0) red[tid >> 6][9] = part;
    __syncthreads();
    RT S = RT(0);
    for (int w = 0; w < MC_THREADS / 64; ++w) S += red[w][9];
    const RT invS = S > RT(0) ? RT(1) / S : RT(0);
    // Covered nodes (fluid, and inside or next to an inside node), compacted in position
    // order: wavefront w scans the positions [w per, (w + 1) per) sixty-four at a time and
    // appends to its own part of the list, so the order, and the sums below, are fixed.
    constexpr int NW = MC_THREADS / 64;
    const int lane = tid & 63, wv = tid >> 6;
    const unsigned per = ((total + NW - 1) / NW + 63u) & ~63u;
    {
        unsigned cnt = 0;
        const unsigned end = min(total, (unsigned)(wv + 1) * per);
        for (unsigned b = (unsigned)wv * per; b < end; b += 64) {
            const unsigned t = b + (unsigned)lane;
            bool cov = false;
            if (t < end) {
                const unsigned char fl = flag[t];
                if (fl & 2) {
                    const unsigned tz = t / sxy, rem = t - tz * sxy, ty = rem / sx, tx = rem - ty * sx;
                    cov = (fl & 1) || (tx > 0 && (flag[t - 1] & 1)) || (tx + 1 < sx && (flag[t + 1] & 1)) ||
                          (ty > 0 && (flag[t - sx] & 1)) || (ty + 1 < sy && (flag[t + sx] & 1)) ||
                          (tz > 0 && (flag[t - sxy] & 1)) || (tz + 1 < sz && (flag[t + sxy] & 1));
                }
            }
            const unsigned long long m = __ballot(cov);
            if (cov) list[(unsigned)wv * per + cnt + (unsigned)__popcll(m & ((1ull << lane) - 1ull))] = (unsigned short)t;
            cnt += (unsigned)__popcll(m);
        }
        if (lane == 0) wcnt[wv] = (int)cnt;
    }
    __syncthreads();
    int ncov = 0;
    for (int w = 0; w < NW; ++w) ncov += wcnt[w];
    RT acc[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    const size_t ld = (size_t)kp.ld;
    for (int j = tid; j < ncov; j += MC_THREADS) {
        int q = j, w = 0;
        while (w + 1 < NW && q >= wcnt[w]) q -= wcnt[w++];
        const unsigned t = list[(unsigned)w * per + (unsigned)q];
        const unsigned tz = t / sxy, rem = t - tz * sxy, ty = rem / sx, tx = rem - ty * sx;
        const bool in = flag[t] & 1;
        const bool xm = tx > 0, xp = tx + 1 < sx, ym = ty > 0, yp = ty + 1 < sy, zm = tz > 0,
                   zp = tz + 1 < sz;
        int X = T.lo[0] + (int)tx, Y = T.lo[1] + (int)ty, Z = T.lo[2] + (int)tz;
        wrap_coord(X, kp.nx, kp.per[0]);
        wrap_coord(Y, kp.ny, kp.per[1]);
        wrap_coord(Z, kp.nz, kp.per[2]);
        const unsigned n = (unsigned)storage_of(segmap, kp, X, Y, Z);   // covered nodes are fluid
        const RT r = raw[t];
        const RT gx = RT(0.5) * ((xp ? raw[t + 1] : RT(0)) - (xm ? raw[t - 1] : RT(0)));
        const RT gy = RT(0.5) * ((yp ? raw[t + sx] : RT(0)) - (ym ? raw[t - sx] : RT(0)));
        const RT gz = RT(0.5) * ((zp ? raw[t + sxy] : RT(0)) - (zm ? raw[t - sxy] : RT(0)));
        RT un[3];
        load_vel<RT>(u, n, kp, un);
        const RT ux = un[0], uy = un[1], uz = un[2];
        const uint32_t old = atomicAdd(cnt + n, 1u);
        const int slot = (int)old;
        const int e = (i << kp.ent_shift) | j;
        if (slot < kp.cap && j < (1 << kp.ent_shift)) {
            ids[(size_t)slot * ld + n] = e;
            store_entry<RT>(vals, (size_t)e, kp, r, gx, gy, gz);
        } else {
            atomicOr(err, ERR_CAPACITY);
        }
        const RT hx = gx * invS, hy = gy * invS, hz = gz * invS;
        // u x grad dhat (vorticity, summed by parts over covered nodes)
        acc[3] += uy * hz - uz * hy;
        acc[4] += uz * hx - ux * hz;
        acc[5] += ux * hy - uy * hx;
        if (!in) continue;
        const RT dh = r * invS;
        acc[0] += dh * ux;
        acc[1] += dh * uy;
        acc[2] += dh * uz;
        const RT g2 = hx * hx + hy * hy + hz * hz;
        const RT il = g2 > RT(0) ? fast_rsqrt(g2) : RT(0);
        const RT nx_ = hx * il, ny_ = hy * il, nz_ = hz * il;
        RT sn[6];
        load_str<RT>(sig, n, kp, sn);
        const RT sxx = sn[0], syy = sn[1], szz = sn[2], sxy_ = sn[3], sxz = sn[4], syz = sn[5];
        const RT t0 = sxx * nx_ + sxy_ * ny_ + sxz * nz_;
        const RT t1 = sxy_ * nx_ + syy * ny_ + syz * nz_;
        const RT t2 = sxz * nx_ + syz * ny_ + szz * nz_;
        const RT d0 = (RT)min_img((double)X - s.R[0], (double)kp.nx, kp.per[0]);
        const RT d1 = (RT)min_img((double)Y - s.R[1], (double)kp.ny, kp.per[1]);
        const RT d2 = (RT)min_img((double)Z - s.R[2], (double)kp.nz, kp.per[2]);
        const RT al = (RT)kp.alpha * dh;
        acc[6] += al * (t1 * d2 - t2 * d1);
        acc[7] += al * (t2 * d0 - t0 * d2);
        acc[8] += al * (t0 * d1 - t1 * d0);
    }
    for (int a = 0; a < 9; ++a)
        for (int o = 32; o > 0; o >>= 1) acc[a] += __shfl_down(acc[a], o, 64);
    __syncthreads();   // every wave has read red[.][9]
    if ((tid & 63) == 0)
        for (int a = 0; a < 9; ++a) red[tid >> 6][a] = acc[a];
    __syncthreads();
    if (tid == 0) {
        RT tot[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
        for (int w = 0; w < MC_THREADS / 64; ++w)
            for (int a = 0; a < 9; ++a) tot[a] += red[w][a];
        RbcCouple& c = cp[i];
        c.S = (double)S;
        for (int a = 0; a < 3; ++a) {
            c.ut[a] = (double)tot[a];
            c.wt[a] = (double)tot[3 + a];
            c.TS[a] = (double)tot[6 + a];
        }
        hydro_cell<RT>(s, c, kp, gat + i);
    }
}

// Cells whose row-compressed tile exceeds the capacity of the one-wavefront pass below take
// the full-tile pass, one block of MC_THREADS per cell, over the list the first pass left.
template <typename RT>
__global__ __launch_bounds__(MC_THREADS) void k_map_couple_tile(const RbcState* __restrict__ st,
                                                                RbcCouple* __restrict__ cp,
                                                                Gather<RT>* __restrict__ gat,
                                                                const uint32_t* __restrict__ nodeword,
                                                                const int* __restrict__ segmap,
                                                                uint32_t* __restrict__ cnt,
                                                                int* __restrict__ ids,
                                                                void* __restrict__ vals,
                                                                const int* __restrict__ ovf,
                                                                const void* __restrict__ u,
                                                                const void* __restrict__ sig,
                                                                KParams kp,
                                                                unsigned* __restrict__ err)
{
    extern __shared__ unsigned char smem[];
    const int n = ovf[0];
    for (int b = blockIdx.x; b < n; b += gridDim.x)
        map_couple_tile<RT>(ovf[1 + b], smem, st, cp, gat, nodeword, segmap, cnt, ids, vals, u, sig, kp, err);
}

// ---- S3 + S4, one wavefront per cell on the row-compressed support tile -----------------------
// The same computation as map_couple_tile, organised for occupancy: a block is one wavefront
// and one cell, and LDS holds only the candidate nodes of each tile row (the covered x-range
// of the row), row after row:
//   clo[r]   first candidate x of row r,  off[r] its first candidate index (off[rows] = total),
//   val[c]   the kernel value raw >= 0 at an inside node, -1 at a fluid node outside the
//            support, -2 at a solid node or outside a non-periodic face,
//   rowof[c] the row of candidate c as ty | tz << 8 (row r = ty + tz sy).
// Neighbours outside a row's candidate range are outside the support (raw = 0, not inside):
// the covered range of every row contains the support range of the row and of its four
// neighbouring rows. More candidates than kp.cand_cap: the cell goes to the overflow list
// ovf[1 + k] (count ovf[0]) for k_map_couple_tile.
template <typename RT, int FM>
__device__ __forceinline__ void map_couple_cell(int k, unsigned char* smem,
                                                const RbcState* __restrict__ st,
                                                RbcCouple* __restrict__ cp,
                                                Gather<RT>* __restrict__ gat,
                                                const uint32_t* __restrict__ nodeword,
                                                const int* __restrict__ segmap, uint32_t* __restrict__ cnt,
                                                int* __restrict__ ids, void* __restrict__ vals,
                                                const int* __restrict__ order,
                                                const void* __restrict__ u,
                                                const void* __restrict__ sig, const KParams& kp,
                                                unsigned* __restrict__ err, int* __restrict__ ovf)
{
    const int i = order[k];
    const RbcState& s = st[i];
    const int lane = threadIdx.x;
    const int tm = kp.tile_max, cap = kp.cand_cap;
    short* clo = reinterpret_cast<short*>(smem);
    short* off = clo + tm * tm;
    RT* val = reinterpret_cast<RT*>(smem + (((size_t)4 * tm * tm + 2 + 15) & ~(size_t)15));
    unsigned short* rowof = reinterpret_cast<unsigned short*>(val + cap);
    int* kof = reinterpret_cast<int*>(rowof + ((cap + 1) & ~1));   // storage index per candidate
    short* tlo = reinterpret_cast<short*>(val);          // support ranges (before val is used)
    short* thi = tlo + tm * tm;

    Tile T;
    support_tile(s, kp, T);
    if (T.sz[0] > tm || T.sz[1] > tm || T.sz[2] > tm) {
        if (lane == 0) atomicOr(err, ERR_CAPACITY);
        return;
    }
    const int sx = T.sz[0], sy = T.sz[1], sz = T.sz[2];
    const int rows = sy * sz;
    // support range of each row (as in map_couple_tile), then the covered range of each row
    // and its length (kept in off[] until the scan)
    double iq[3];
    for (int a = 0; a < 3; ++a) iq[a] = fabs(s.Q[a]) > 1e-12 ? 1.0 / s.Q[a] : 0.0;
    for (int r = lane; r < rows; r += 64) {
        int lo, hi;
        support_row(s, kp, T, iq, r % sy, r / sy, lo, hi);
        tlo[r] = (short)lo;
        thi[r] = (short)hi;
    }
    __syncthreads();
    for (int r = lane; r < rows; r += 64) {
        int lo, hi;
        covered_row(tlo, thi, r, sx, sy, sz, lo, hi);
        clo[r] = (short)lo;
        off[r] = (short)max(0, hi - lo + 1);
    }
    __syncthreads();
    // exclusive scan of the lengths: each lane a run of consecutive rows, then the lanes
    const int per = (rows + 63) / 64, r0 = min(rows, lane * per), r1 = min(rows, r0 + per);
    int run = 0;
    for (int r = r0; r < r1; ++r) run += off[r];
    int incl = run;
    for (int o = 1; o < 64; o <<= 1) {
        const int v = __shfl_up(incl, o, 64);
        if (lane >= o) incl += v;
    }
    const int total = __shfl(incl, 63, 64);
    int base = incl - run;
    __syncthreads();
    for (int r = r0; r < r1; ++r) {
        const int len = off[r];
        off[r] = (short)base;
        base += len;
    }
    if (lane == 63) off[rows] = (short)total;
    if (total > cap) {
        if (lane == 0) ovf[1 + atomicAdd(ovf, 1)] = i;
        return;
    }
    __syncthreads();
    for (int r = r0; r < r1; ++r)
        for (int c = off[r], e = off[r + 1]; c < e; ++c)
            rowof[c] = (unsigned short)((r % sy) | (r / sy) << 8);
    __syncthreads();

    // pass 1: exact support test and raw kernel value at every candidate; S = sum raw
    const RT s0 = RT(2.0 / kp.xi[0]), s1 = RT(2.0 / kp.xi[1]), s2 = RT(2.0 / kp.xi[2]);
    // A tile inside the box on every axis, whose nodes all lie within half a period of the
    // centre on the periodic axes, needs no coordinate wrapping, and its minimum images are
    // the plain differences (min_img is the identity there): the passes below are
    // instantiated for that case (most cells) and for the general one.
    bool interior = true;
    {
        const int Lx[3] = {kp.nx, kp.ny, kp.nz};
        for (int a = 0; a < 3; ++a) {
            interior = interior && T.lo[a] >= 0 && T.lo[a] + T.sz[a] <= Lx[a];
            if (kp.per[a])
                interior = interior && s.R[a] - (double)T.lo[a] <= 0.5 * (double)Lx[a] &&
                           (double)(T.lo[a] + T.sz[a] - 1) - s.R[a] <= 0.5 * (double)Lx[a];
        }
    }
    auto wrap3 = [&](auto inner, int& X, int& Y, int& Z) -> bool {
        if constexpr (decltype(inner)::value) return true;
        else {
            // every axis is wrapped (no short-circuit): the three coordinates are all updated
            const int in_x = wrap_coord(X, kp.nx, kp.per[0]), in_y = wrap_coord(Y, kp.ny, kp.per[1]),
                      in_z = wrap_coord(Z, kp.nz, kp.per[2]);
            return in_x && in_y && in_z;
        }
    };
    auto mimg = [&](auto inner, double d, double L, int per) -> double {
        if constexpr (decltype(inner)::value) return d;
        else return min_img(d, L, per);
    };
    RT part = RT(0);
    // the node words of P1_GROUP candidates are loaded together, then the candidates are
    // tested one after another (in the same order, so S sums identically)
    constexpr int P1_GROUP = 4;
    auto pass1 = [&](auto inner) {
        for (int c0 = lane; c0 < total; c0 += 64 * P1_GROUP) {
            int Xg[P1_GROUP], Yg[P1_GROUP], Zg[P1_GROUP], kg[P1_GROUP];
            uint32_t wg[P1_GROUP];
#pragma unroll
            for (int g = 0; g < P1_GROUP; ++g) {
                const int c = c0 + 64 * g;
                wg[g] = 0u;
                Xg[g] = Yg[g] = Zg[g] = 0;
                kg[g] = -1;
                if (c < total) {
                    const int yz = rowof[c];
                    const int ty = yz & 255, tz = yz >> 8, r = ty + tz * sy, tx = clo[r] + (c - off[r]);
                    int X = T.lo[0] + tx, Y = T.lo[1] + ty, Z = T.lo[2] + tz;
                    if (wrap3(inner, X, Y, Z)) {
                        const int kst = storage_of(segmap, kp, X, Y, Z);
                        kg[g] = kst;
                        wg[g] = kst >= 0 ? nodeword[kst] : 0u;
                    }
                    Xg[g] = X;
                    Yg[g] = Y;
                    Zg[g] = Z;
                }
            }
#pragma unroll
            for (int g = 0; g < P1_GROUP; ++g) {
                const int c = c0 + 64 * g;
                if (c >= total) break;
                const int X = Xg[g], Y = Yg[g], Z = Zg[g];
                RT v = RT(-2);
                if (wg[g] & NW_FLUID) {
                    v = RT(-1);
                    double y[3];
                    const double d0 = mimg(inner, (double)X - s.R[0], (double)kp.nx, kp.per[0]);
                    const double d1 = mimg(inner, (double)Y - s.R[1], (double)kp.ny, kp.per[1]);
                    const double d2 = mimg(inner, (double)Z - s.R[2], (double)kp.nz, kp.per[2]);
                    body_coords_exact(s.Q, d0, d1, d2, y);
                    if (fabs(y[0]) < kp.xi[0] && fabs(y[1]) < kp.xi[1] && fabs(y[2]) < kp.xi[2]) {
                        v = peskin((RT)y[0] * s0) * peskin((RT)y[1] * s1) * peskin((RT)y[2] * s2);
                        part += v;
                    }
                }
                val[c] = v;
                kof[c] = kg[g];
            }
        }
    };
    if (interior) pass1(std::true_type{});
    else pass1(std::false_type{});
    for (int o = 32; o > 0; o >>= 1) part += __shfl_down(part, o, 64);
    const RT S = __shfl(part, 0, 64);
    const RT invS = S > RT(0) ? RT(1) / S : RT(0);
    __syncthreads();

    // pass 2: covered candidates (fluid, and inside or next to an inside node). The LDS reads
    // go in three independent batches (the candidate's value and row; the row tables of its
    // row and the four neighbouring rows; the six neighbour values), and each covered node
    // issues its loads and its slot atomic together.
    // the j-th covered node in candidate order fills the cell's entry j
    RT acc[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    const size_t ld = (size_t)kp.ld;
    const unsigned long long below = (1ull << lane) - 1ull;
    int jbase = 0;
    // index of x in a row's candidates, from the row's (first x, first index, end index); -1 outside
    auto cand = [](int x, int cl, int o, int e) { const int d = x - cl; return (d >= 0 && d < e - o) ? o + d : -1; };
    auto pass2 = [&](auto inner) {
        for (int c0 = 0; c0 < total; c0 += 64) {
            const int c = c0 + lane;
            const bool live = c < total;
            const int cc = live ? c : 0;
            const RT v0 = val[cc];
            const int yz = rowof[cc];
            const int kn = kof[cc];
            const RT v = live ? v0 : RT(-2);
            const int ty = yz & 255, tz = yz >> 8, r = ty + tz * sy;
            const bool hym = ty > 0, hyp = ty + 1 < sy, hzm = tz > 0, hzp = tz + 1 < sz;
            const int rym = hym ? r - 1 : r, ryp = hyp ? r + 1 : r, rzm = hzm ? r - sy : r, rzp = hzp ? r + sy : r;
            const int cl0 = clo[r], o0 = off[r], e0 = off[r + 1];
            const int cl1 = clo[rym], o1 = off[rym], e1 = off[rym + 1];
            const int cl2 = clo[ryp], o2 = off[ryp], e2 = off[ryp + 1];
            const int cl3 = clo[rzm], o3 = off[rzm], e3 = off[rzm + 1];
            const int cl4 = clo[rzp], o4 = off[rzp], e4 = off[rzp + 1];
            const int tx = cl0 + (cc - o0);
            const int ixm = cand(tx - 1, cl0, o0, e0), ixp = cand(tx + 1, cl0, o0, e0);
            const int iym = hym ? cand(tx, cl1, o1, e1) : -1, iyp = hyp ? cand(tx, cl2, o2, e2) : -1;
            const int izm = hzm ? cand(tx, cl3, o3, e3) : -1, izp = hzp ? cand(tx, cl4, o4, e4) : -1;
            const RT m2 = RT(-2);
            const RT axm = val[max(ixm, 0)], axp = val[max(ixp, 0)], aym = val[max(iym, 0)];
            const RT ayp = val[max(iyp, 0)], azm = val[max(izm, 0)], azp = val[max(izp, 0)];
            const RT vxm = ixm >= 0 ? axm : m2, vxp = ixp >= 0 ? axp : m2, vym = iym >= 0 ? aym : m2;
            const RT vyp = iyp >= 0 ? ayp : m2, vzm = izm >= 0 ? azm : m2, vzp = izp >= 0 ? azp : m2;
            const bool cov = v > RT(-1.5) &&
                             (v >= RT(0) || vxm >= RT(0) || vxp >= RT(0) || vym >= RT(0) || vyp >= RT(0) ||
                              vzm >= RT(0) || vzp >= RT(0));
            const unsigned long long m = __ballot(cov);
            const int j = jbase + (int)__popcll(m & below);
            jbase += (int)__popcll(m);
            if (!cov) continue;
            const bool in = v >= RT(0);
            const unsigned n = (unsigned)kn;   // covered nodes are fluid: stored
            const RT z0 = RT(0);
            const RT rr = in ? v : z0;
            const RT gx = RT(0.5) * (max(vxp, z0) - max(vxm, z0));
            const RT gy = RT(0.5) * (max(vyp, z0) - max(vym, z0));
            const RT gz = RT(0.5) * (max(vzp, z0) - max(vzm, z0));
            RT un[3];
            load_vel<RT, FM>(u, n, kp, un);
            const RT ux = un[0], uy = un[1], uz = un[2];
            // the stress at inside nodes, loaded beside u before the atomic's result is needed
            RT sg[6] = {z0, z0, z0, z0, z0, z0};
            if (in) load_str<RT, FM>(sig, n, kp, sg);
            const uint32_t old = atomicAdd(cnt + n, 1u);
            const int slot = (int)old;
            const int e = (i << kp.ent_shift) | j;
            if (slot < kp.cap && j < (1 << kp.ent_shift)) {
                ids[(size_t)slot * ld + n] = e;
                store_entry<RT, FM>(vals, (size_t)e, kp, rr, gx, gy, gz);
            } else {
                atomicOr(err, ERR_CAPACITY);
            }
            const RT hx = gx * invS, hy = gy * invS, hz = gz * invS;
            acc[3] += uy * hz - uz * hy;
            acc[4] += uz * hx - ux * hz;
            acc[5] += ux * hy - uy * hx;
            if (!in) continue;
            const RT dh = rr * invS;
            acc[0] += dh * ux;
            acc[1] += dh * uy;
            acc[2] += dh * uz;
            const RT g2 = hx * hx + hy * hy + hz * hz;
            const RT il = g2 > RT(0) ? fast_rsqrt(g2) : RT(0);
            const RT nx_ = hx * il, ny_ = hy * il, nz_ = hz * il;
            const RT sxx = sg[0], syy = sg[1], szz = sg[2], sxy_ = sg[3], sxz = sg[4], syz = sg[5];
            int X = T.lo[0] + tx, Y = T.lo[1] + ty, Z = T.lo[2] + tz;
            wrap3(inner, X, Y, Z);
            const RT t0 = sxx * nx_ + sxy_ * ny_ + sxz * nz_;
            const RT t1 = sxy_ * nx_ + syy * ny_ + syz * nz_;
            const RT t2 = sxz * nx_ + syz * ny_ + szz * nz_;
            const RT d0 = (RT)mimg(inner, (double)X - s.R[0], (double)kp.nx, kp.per[0]);
            const RT d1 = (RT)mimg(inner, (double)Y - s.R[1], (double)kp.ny, kp.per[1]);
            const RT d2 = (RT)mimg(inner, (double)Z - s.R[2], (double)kp.nz, kp.per[2]);
            const RT al = (RT)kp.alpha * dh;
            acc[6] += al * (t1 * d2 - t2 * d1);
            acc[7] += al * (t2 * d0 - t0 * d2);
            acc[8] += al * (t0 * d1 - t1 * d0);
        }
    };
    if (interior) pass2(std::true_type{});
    else pass2(std::false_type{});
    for (int a = 0; a < 9; ++a)
        for (int o = 32; o > 0; o >>= 1) acc[a] += __shfl_down(acc[a], o, 64);
    if (lane == 0) {
        RbcCouple& c = cp[i];
        c.S = (double)S;
        for (int a = 0; a < 3; ++a) {
            c.ut[a] = (double)acc[a];
            c.wt[a] = (double)acc[3 + a];
            c.TS[a] = (double)acc[6 + a];
        }
        hydro_cell<RT>(s, c, kp, gat + i);
    }
}

// FM: the field mode of u and sigma (KParams::field16), fixed per instantiation
template <typename RT, int FM>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(5))) void k_map_couple(const RbcState* __restrict__ st,
                                                   RbcCouple* __restrict__ cp,
                                                   Gather<RT>* __restrict__ gat,
                                                   const uint32_t* __restrict__ nodeword,
                                                   const int* __restrict__ segmap, uint32_t* __restrict__ cnt,
                                                   int* __restrict__ ids, void* __restrict__ vals,
                                                   const int* __restrict__ order,
                                                   const void* __restrict__ u,
                                                   const void* __restrict__ sig, KParams kp,
                                                   unsigned* __restrict__ err,
                                                   int* __restrict__ ovf)
{
    extern __shared__ unsigned char smem[];
    const int k = xcd_chunk_index(1);
    if (k < kp.nrbc)
        map_couple_cell<RT, FM>(k, smem, st, cp, gat, nodeword, segmap, cnt, ids, vals, order, u, sig, kp, err, ovf);
}

// ---- S5: Gay-Berne forces and torques (Sec. II E, Eqs. 24-28; App. B) -----------------------
// F on i = -du/dR R^ - (1/R^2) du/dphi [k - (k.R^) R^], k = H^-1 R_ij, H = A_i + A_j;
// torques tau_i = (1/R) R_ci x f_k, R_ci = -A_i k, f_k = -(1/R) du/dphi k (lab frame).
// (A_i + A_j)^-1 by cofactors
__device__ __forceinline__ void gb_inverse(const double* Ai, const double* Aj, double* Hi)
{
    double H[9];
    for (int a = 0; a < 9; ++a) H[a] = Ai[a] + Aj[a];
    const double det = H[0] * (H[4] * H[8] - H[5] * H[7]) - H[1] * (H[3] * H[8] - H[5] * H[6]) +
                       H[2] * (H[3] * H[7] - H[4] * H[6]);
    const double id = 1.0 / det;
    Hi[0] = (H[4] * H[8] - H[5] * H[7]) * id;
    Hi[1] = (H[2] * H[7] - H[1] * H[8]) * id;
    Hi[2] = (H[1] * H[5] - H[2] * H[4]) * id;
    Hi[3] = (H[5] * H[6] - H[3] * H[8]) * id;
    Hi[4] = (H[0] * H[8] - H[2] * H[6]) * id;
    Hi[5] = (H[2] * H[3] - H[0] * H[5]) * id;
    Hi[6] = (H[3] * H[7] - H[4] * H[6]) * id;
    Hi[7] = (H[1] * H[6] - H[0] * H[7]) * id;
    Hi[8] = (H[0] * H[4] - H[1] * H[3]) * id;
}

// one pair given Hi = (A_i + A_j)^-1; returns 1 at rho <= 0 (or coincident centres)
__device__ int gb_pair(const KParams& kp, const double* rij, const double* Ai, const double* Hi,
                       double smin, double* F, double* ti)
{
    const double R = sqrt(rij[0] * rij[0] + rij[1] * rij[1] + rij[2] * rij[2]);
    if (!(R > 0.0)) return 1;
    double rh[3], kap[3];
    for (int k = 0; k < 3; ++k) rh[k] = rij[k] / R;
    mat_vec(Hi, rij, kap);
    const double phi = 0.5 * (rh[0] * kap[0] + rh[1] * kap[1] + rh[2] * kap[2]) / R;
    const double sigma = 1.0 / sqrt(phi);
    const double rho = (R - sigma + smin) / smin;
    if (!(rho > 0.0)) return 1;
    const double r2 = rho * rho, r6 = r2 * r2 * r2;
    if (r6 > 2.0) return 0;
    const double ir6 = 1.0 / r6, ir7 = ir6 / rho, ir13 = ir7 * ir6;
    const double core = -24.0 * kp.eps0 * (2.0 * ir13 - ir7);
    const double dudr = core / smin;
    const double dudphi = core * sigma * sigma * sigma / (2.0 * smin);
    const double kr = kap[0] * rh[0] + kap[1] * rh[1] + kap[2] * rh[2];
    for (int k = 0; k < 3; ++k) F[k] += -dudr * rh[k] - dudphi / (R * R) * (kap[k] - kr * rh[k]);
    double Aik[3], fk[3], c[3];
    mat_vec(Ai, kap, Aik);
    for (int k = 0; k < 3; ++k) {
        fk[k] = -dudphi / R * kap[k];
        Aik[k] = -Aik[k];
    }
    cross3(Aik, fk, c);
    for (int k = 0; k < 3; ++k) ti[k] += c[k] / R;
    return 0;
}

__device__ __forceinline__ void shape_matrix(const KParams& kp, const double* Q, double* A)
{
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) {
            double a = 0.0;
            for (int k = 0; k < 3; ++k) a += Q[3 * r + k] * kp.axes[k] * kp.axes[k] * Q[3 * c + k];
            A[3 * r + c] = a;
        }
}

// Neighbour cell `q` (0..26, dx fastest) of cell coordinates cc; -1 when it does not exist
// (outside a non-periodic face). An axis with fewer than three cells lists each of its
// cells once (offset index d -> cell d).
__device__ __forceinline__ int neighbour_cell(const KParams& kp, const int* ncell, const int cc[3], int q)
{
    const int d[3] = {q % 3, (q / 3) % 3, q / 9};
    int v[3];
    for (int a = 0; a < 3; ++a) {
        const int m = ncell[a];
        if (m < 3) {
            if (d[a] >= m) return -1;
            v[a] = d[a];
        } else {
            int x = cc[a] + d[a] - 1;
            if (x < 0 || x >= m) {
                if (!kp.per[a]) return -1;
                x = (x + m) % m;
            }
            v[a] = x;
        }
    }
    return v[0] + ncell[0] * (v[1] + ncell[1] * v[2]);
}

// Flattened candidates of the 27 neighbour cells: lanes 0..26 hold one cell's CSR range, an
// inclusive wave scan gives the running totals, and candidate e belongs to the first cell
// whose running total exceeds e (binary search over the 27 totals kept in LDS).
struct CandidateRanges {
    int base[27];
    int pre[27];
    int total;
};

__device__ __forceinline__ void gather_ranges(const int* __restrict__ off, int cell_of_lane, int lane,
                                              CandidateRanges& cr)
{
    int cnt = 0, base = 0;
    if (lane < 27 && cell_of_lane >= 0) {
        base = off[cell_of_lane];
        cnt = off[cell_of_lane + 1] - base;
    }
    int incl = cnt;
    for (int o = 1; o < 32; o <<= 1) {
        const int v = __shfl_up(incl, o, 64);
        if (lane >= o) incl += v;
    }
    if (lane < 27) {
        cr.base[lane] = base;
        cr.pre[lane] = incl;
    }
    cr.total = __shfl(incl, 26, 64);
}

__device__ __forceinline__ int candidate(const CandidateRanges& cr, const int* __restrict__ ids, int e)
{
    int lo = 0, hi = 26;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (cr.pre[mid] > e) hi = mid;
        else lo = mid + 1;
    }
    const int start = lo ? cr.pre[lo - 1] : 0;
    return ids[cr.base[lo] + (e - start)];
}

// one wavefront per cell: lanes stride over the flattened candidates (cells, then wall
// points), then a fixed-order shuffle reduction (bitwise repeatable)
// one wavefront per cell k of the sorted order (wavefront wv of its block); the lab force and
// body torque of cell i go to outF[stride i + a], outT[stride i + a] (the cell's coupling
// record, or caller arrays with stride 3)
__device__ __forceinline__ void gay_berne_cell(int k, const RbcState* __restrict__ st,
                                               double* __restrict__ outF, double* __restrict__ outT,
                                               int ostride,
                                               const int* __restrict__ order,
                                               const int* __restrict__ cell_off,
                                               const int* __restrict__ cell_ids,
                                               const int* __restrict__ wall_xyz,
                                               const int* __restrict__ wcell_off,
                                               const int* __restrict__ wcell_ids,
                                               const KParams& kp, unsigned* err)
{
    __shared__ CandidateRanges ranges[4][2];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int i = order[k];
    const double* Ri = st[i].R;
    const double* Qi = st[i].Q;
    int cc[3];
    for (int a = 0; a < 3; ++a) cc[a] = cell_coord(kp, a, Ri[a]);
    gather_ranges(cell_off, lane < 27 ? neighbour_cell(kp, kp.ncell, cc, lane) : -1, lane, ranges[wv][0]);
    if (kp.wall_particles) {
        // wall points are binned in their own grid, of edge at least the cell-wall cut-off
        int wc[3];
        for (int a = 0; a < 3; ++a) {
            wc[a] = (int)floor(Ri[a] / kp.wcedge[a]);
            wc[a] = wc[a] < 0 ? 0 : (wc[a] >= kp.wncell[a] ? kp.wncell[a] - 1 : wc[a]);
        }
        gather_ranges(wcell_off, lane < 27 ? neighbour_cell(kp, kp.wncell, wc, lane) : -1, lane,
                      ranges[wv][1]);
    }
    __builtin_amdgcn_wave_barrier();
    double Ai[9], Aw[9];
    shape_matrix(kp, Qi, Ai);
    for (int a = 0; a < 9; ++a) Aw[a] = (a % 4 == 0) ? kp.a_wall * kp.a_wall : 0.0;
    const double amin = fmin(kp.axes[0], fmin(kp.axes[1], kp.axes[2]));
    const double smin_cc = sqrt(4.0 * amin * amin);
    double F[3] = {0, 0, 0}, tl[3] = {0, 0, 0};
    const double rcc2 = kp.rc_pair * kp.rc_pair, rcw2 = kp.rc_wall * kp.rc_wall;
    // Pairs beyond the cut-off shell are skipped before the contact distance sigma is formed:
    // gb_pair returns nothing for them (rho^6 > 2, i.e. R - sigma > (2^(1/6) - 1) sigma_min).
    // Cell-cell: sigma^2 = 2 R^2 / (r^T H^-1 r) <= 2 r^T H r / R^2 for the symmetric positive
    // definite H = A_i + A_j (Cauchy-Schwarz), with r^T A r = sum_k s_k^2 ((Q^T r)_k)^2.
    // Cell-wall: H = A_i + a_w^2 1 is diagonal in the body frame, sigma^2 = 2 R^2 / sum_k
    // (Q_i^T r)_k^2 / (s_k^2 + a_w^2). A margin of 1e-9 (1 + R) keeps every pair the rounding
    // of either form could leave in range, so the forces and the overlap flag are unchanged.
    const double shell = exp2(1.0 / 6.0) - 1.0;
    const double dcc = shell * smin_cc, dcw = shell * kp.sigmin_wall;
    auto body_sq = [&](const double* Q, const double* r, const double* wk) {
        double q = 0.0;
        for (int k = 0; k < 3; ++k) {
            const double y = Q[0 * 3 + k] * r[0] + Q[1 * 3 + k] * r[1] + Q[2 * 3 + k] * r[2];
            q += wk[k] * y * y;
        }
        return q;
    };
    double s2[3], hw[3];
    for (int k = 0; k < 3; ++k) {
        s2[k] = kp.axes[k] * kp.axes[k];
        hw[k] = 1.0 / (s2[k] + kp.a_wall * kp.a_wall);
    }
    int bad = 0;
    const CandidateRanges& rc = ranges[wv][0];
    for (int e = lane; e < rc.total; e += 64) {
        const int j = candidate(rc, cell_ids, e);
        if (j == i) continue;
        double r[3];
        for (int a = 0; a < 3; ++a) r[a] = min_img(Ri[a] - st[j].R[a], box_len(kp, a), kp.per[a]);
        const double R2 = r[0] * r[0] + r[1] * r[1] + r[2] * r[2];
        if (R2 > rcc2) continue;
        {
            const double R = sqrt(R2);
            const double sub = sqrt(2.0 * (body_sq(Qi, r, s2) + body_sq(st[j].Q, r, s2)) / R2);
            if (R - sub > dcc + 1e-9 * (1.0 + R)) continue;
        }
        double Aj[9], Hi[9];
        shape_matrix(kp, st[j].Q, Aj);
        gb_inverse(Ai, Aj, Hi);
        bad |= gb_pair(kp, r, Ai, Hi, smin_cc, F, tl);
    }
    if (kp.wall_particles) {
        // H^-1 = (A_i + a_w^2 1)^-1 is the same for every wall point
        double Hw[9];
        gb_inverse(Ai, Aw, Hw);
        const CandidateRanges& rw = ranges[wv][1];
        for (int e = lane; e < rw.total; e += 64) {
            const int wq = candidate(rw, wcell_ids, e);
            double r[3];
            for (int a = 0; a < 3; ++a)
                r[a] = min_img(Ri[a] - (double)wall_xyz[3 * wq + a], box_len(kp, a), kp.per[a]);
            const double R2 = r[0] * r[0] + r[1] * r[1] + r[2] * r[2];
            if (R2 > rcw2) continue;
            {
                const double R = sqrt(R2);
                const double sig = sqrt(2.0 * R2 / body_sq(Qi, r, hw));
                if (R - sig > dcw + 1e-9 * (1.0 + R)) continue;
            }
            bad |= gb_pair(kp, r, Ai, Hw, kp.sigmin_wall, F, tl);
        }
    }
    for (int o = 32; o > 0; o >>= 1) {
        for (int a = 0; a < 3; ++a) {
            F[a] += __shfl_down(F[a], o, 64);
            tl[a] += __shfl_down(tl[a], o, 64);
        }
        bad |= __shfl_down(bad, o, 64);
    }
    if (lane == 0) {
        if (bad) atomicOr(err, ERR_OVERLAP);
        double tb[3];
        matT_vec(Qi, tl, tb);
        for (int a = 0; a < 3; ++a) {
            outF[(size_t)ostride * i + a] = F[a];
            outT[(size_t)ostride * i + a] = tb[a];
        }
    }
}

// blocks of one wavefront: on the side stream they fit into whatever slots the concurrent
// map pass and stream-collide leave
__global__ __launch_bounds__(64) void k_gay_berne(const RbcState* __restrict__ st,
                                                   double* __restrict__ outF,
                                                   double* __restrict__ outT, int ostride,
                                                   const int* __restrict__ order,
                                                   const int* __restrict__ cell_off,
                                                   const int* __restrict__ cell_ids,
                                                   const int* __restrict__ wall_xyz,
                                                   const int* __restrict__ wcell_off,
                                                   const int* __restrict__ wcell_ids, KParams kp,
                                                   unsigned* err)
{
    const int k = xcd_chunk_index(1);
    if (k < kp.nrbc)
        gay_berne_cell(k, st, outF, outT, ostride, order, cell_off, cell_ids, wall_xyz, wcell_off,
                       wcell_ids, kp, err);
}

// ---- S6: combined force/torque, hydrodynamic force/torque, second half --------------------
// F^comb = F^mech + F^ext + gT M u~; tau^comb = tau^mech + tau^ext + Q^T T^S + gR I (s Q^T w~)
// (F^ext lab, tau^ext body: the constant drive of the single-cell drag and spin experiments);
// F^hyd = -M gT (V - u~); T^hyd = Q [-gR I (Omega - s Q^T w~)] + T^S (lab), with the velocities
// after the first half (which equal the half-step values within a step).
// hydro_cell: F^hyd, T^hyd and the gather record of cell i from its interpolation sums in c
// (S, u~, w~, T^S, just written by the same thread); run at the end of the map pass.
template <typename RT>
__device__ __forceinline__ void hydro_cell(const RbcState& s, RbcCouple& c, const KParams& kp,
                                           Gather<RT>* __restrict__ gi)
{
    double wb[3], tb[3], tl[3], Fh[3], Th[3];
    matT_vec(s.Q, c.wt, wb);
    for (int a = 0; a < 3; ++a) {
        Fh[a] = -kp.mass * kp.gammaT * (s.V[a] - c.ut[a]);
        tb[a] = -kp.gammaR * kp.inertia[a] * (s.Om[a] - kp.vort_scale * wb[a]);
    }
    mat_vec(s.Q, tb, tl);
    for (int a = 0; a < 3; ++a) Th[a] = tl[a] + c.TS[a];
    Gather<RT> G;
    for (int a = 0; a < 3; ++a) {
        c.Fh[a] = Fh[a];
        c.Th[a] = Th[a];
        G.F[a] = (RT)Fh[a];
        G.T[a] = (RT)Th[a];
    }
    G.invS = c.S > 0.0 ? (RT)(1.0 / c.S) : RT(0);
    G.pad = RT(0);
    *gi = G;
}

// kick_cell: combined force and torque (needs the Gay-Berne forces), half-step friction and
// half kick
__device__ __forceinline__ void kick_cell(RbcState* __restrict__ st, const RbcCouple* __restrict__ cp,
                                          const KParams& kp, int i)
{
    RbcState s = st[i];
    const RbcCouple& c = cp[i];
    double wb[3], tsb[3];
    matT_vec(s.Q, c.wt, wb);
    matT_vec(s.Q, c.TS, tsb);
    const double eT = exp(-kp.gammaT * 0.5), eR = exp(-kp.gammaR * 0.5);
    for (int a = 0; a < 3; ++a) {
        s.Fc[a] = c.Fm[a] + kp.ext_force[a] + kp.gammaT * kp.mass * c.ut[a];
        s.Tc[a] = c.Tm[a] + kp.ext_torque[a] + tsb[a] + kp.gammaR * kp.inertia[a] * kp.vort_scale * wb[a];
        s.V[a] *= eT;
        s.Om[a] *= eR;
        s.V[a] += 0.5 / kp.mass * s.Fc[a];
        s.Om[a] += 0.5 * s.Tc[a] / kp.inertia[a];
    }
    st[i] = s;
}

__global__ __launch_bounds__(128) void k_rb_second_half(RbcState* __restrict__ st,
                                                        const RbcCouple* __restrict__ cp, KParams kp)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < kp.nrbc) kick_cell(st, cp, kp, i);
}

__global__ void k_init_combined(RbcState* __restrict__ st, const RbcCouple* __restrict__ cp, KParams kp)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= kp.nrbc) return;
    for (int a = 0; a < 3; ++a) {
        st[i].Fc[a] = cp[i].Fm[a] + kp.ext_force[a];
        st[i].Tc[a] = cp[i].Tm[a] + kp.ext_torque[a];
    }
}


// ---- fused multi-lattice versions of the per-cell stages (one launch for many contexts) -----
constexpr int FUSED_TILE_BLOCKS = 4;   // blocks per slot of the full-tile overflow pass

__global__ __launch_bounds__(256) void kf_cells_a(const FusedArgs fa)
{
    int lb;
    const SlotDesc& d = *fa.slot[fused_slot(fa, lb)];
    const KParams kp = d.kp;
    const int i = lb * 256 + (int)threadIdx.x;
    if (i == 0) d.b.ovf[0] = 0;   // overflow list of this step's map pass
    if (i >= kp.nrbc) return;
    rb1_cell(d.b.st, kp, i);
    bin_cell(d.b.st, d.b.cellid, d.b.cell_cnt, kp, i);
}

__global__ __launch_bounds__(SCAN_THREADS) void kf_scan(const FusedArgs fa)
{
    int lb;
    const SlotDesc& d = *fa.slot[fused_slot(fa, lb)];
    scan_clear_block(d.b.cell_cnt, d.b.cell_off, d.kp.ncell[0] * d.kp.ncell[1] * d.kp.ncell[2]);
}

__global__ __launch_bounds__(256) void kf_scatter(const FusedArgs fa)
{
    int lb;
    const SlotDesc& d = *fa.slot[fused_slot(fa, lb)];
    const int i = lb * 256 + (int)threadIdx.x;
    if (i < d.kp.nrbc) scatter_cell(d.b.cellid, d.b.cell_off, d.b.cell_cnt, d.b.cell_ids, i);
}

__global__ __launch_bounds__(256) void kf_sort(const FusedArgs fa)
{
    int lb;
    const SlotDesc& d = *fa.slot[fused_slot(fa, lb)];
    const int c = lb * 256 + (int)threadIdx.x;
    if (c < d.kp.ncell[0] * d.kp.ncell[1] * d.kp.ncell[2]) sort_cell(d.b.cell_off, d.b.cell_ids, d.b.cell_cnt, c);
}

template <typename RT, int FM>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(5))) void kf_map(const FusedArgs fa)
{
    extern __shared__ unsigned char smem[];
    int lb;
    const SlotDesc& d = *fa.slot[fused_slot(fa, lb)];
    const KParams kp = d.kp;
    if (lb < kp.nrbc)
        map_couple_cell<RT, FM>(lb, smem, d.b.st, d.b.cp, (Gather<RT>*)d.b.gat, d.b.nodeword, d.b.tab.map, d.b.cnt,
                            d.b.map_ids,
                            d.b.map_vals,
                            d.b.cell_ids, d.b.u, d.b.sig, kp, d.b.err, d.b.ovf);
}

template <typename RT>
__global__ __launch_bounds__(MC_THREADS) void kf_map_tile(const FusedArgs fa)
{
    extern __shared__ unsigned char smem[];
    int lb;
    const SlotDesc& d = *fa.slot[fused_slot(fa, lb)];
    const KParams kp = d.kp;
    const int n = d.b.ovf[0];
    for (int b = lb; b < n; b += FUSED_TILE_BLOCKS)
        map_couple_tile<RT>(d.b.ovf[1 + b], smem, d.b.st, d.b.cp, (Gather<RT>*)d.b.gat, d.b.nodeword, d.b.tab.map,
                            d.b.cnt,
                            d.b.map_ids,
                            d.b.map_vals, d.b.u, d.b.sig, kp, d.b.err);
}

// one cell per one-wavefront block, as k_gay_berne: beside the map pass and the stream-collide
// a block needing several wave slots at once waits long for them
__global__ __launch_bounds__(64) void kf_gb(const FusedArgs fa)
{
    int lb;
    const SlotDesc& d = *fa.slot[fused_slot(fa, lb)];
    const KParams kp = d.kp;
    const int k = lb;
    if (k < kp.nrbc)
        gay_berne_cell(k, d.b.st, d.b.cp[0].Fm, d.b.cp[0].Tm, COUPLE_STRIDE, d.b.cell_ids, d.b.cell_off,
                       d.b.cell_ids, d.b.wall_xyz, d.b.wcell_off, d.b.wcell_ids, kp, d.b.err);
}

__global__ __launch_bounds__(128) void kf_kick(const FusedArgs fa)
{
    int lb;
    const SlotDesc& d = *fa.slot[fused_slot(fa, lb)];
    const KParams kp = d.kp;
    const int i = lb * 128 + (int)threadIdx.x;
    if (i < kp.nrbc) kick_cell(d.b.st, d.b.cp, kp, i);
}

// ---- launchers ---------------------------------------------------------------------------------
static inline unsigned nblk(long long n, int b) { return (unsigned)((n + b - 1) / b); }

// cell offsets from the counts: one block for a few chunks, else one block per chunk
static void launch_scan_clear(const CellBuffers& b, int nc, hipStream_t st)
{
    const int nchunk = (nc + SCAN_CHUNK - 1) / SCAN_CHUNK;
    if (nchunk <= SCAN_SINGLE_BLOCK_CHUNKS) {
        hipLaunchKernelGGL(k_scan_clear, dim3(1), dim3(SCAN_THREADS), 0, st, b.cell_cnt, b.cell_off, nc);
        return;
    }
    hipLaunchKernelGGL(k_scan_partials, dim3(nchunk), dim3(SCAN_THREADS), 0, st, b.cell_cnt, b.cell_part, nc);
    hipLaunchKernelGGL(k_scan_chunks, dim3(nchunk), dim3(SCAN_THREADS), 0, st, b.cell_cnt, b.cell_off,
                       b.cell_part, nc);
}



void launch_rb1_cell_list(const CellBuffers& b, const KParams& kp, hipStream_t st)
{
    const int nc = kp.ncell[0] * kp.ncell[1] * kp.ncell[2];
    hipLaunchKernelGGL(k_rb1_bin, dim3(nblk(kp.nrbc, 64)), dim3(64), 0, st, b.st, b.cellid,
                       b.cell_cnt, b.ovf, kp);
    launch_scan_clear(b, nc, st);
    hipLaunchKernelGGL(k_cells_scatter, dim3(nblk(kp.nrbc, 64)), dim3(64), 0, st, b.cellid,
                       b.cell_off, b.cell_cnt, b.cell_ids, kp.nrbc);
    hipLaunchKernelGGL(k_cells_sort, dim3(nblk(nc, 64)), dim3(64), 0, st, b.cell_off,
                       b.cell_ids, b.cell_cnt, nc);
}

void launch_cell_list(const CellBuffers& b, const KParams& kp, hipStream_t st)
{
    const int nc = kp.ncell[0] * kp.ncell[1] * kp.ncell[2];
    // cell_cnt is all zero here: k_scan_clear leaves it so, and init clears it once
    hipLaunchKernelGGL(k_cells_bin, dim3(nblk(kp.nrbc, 256)), dim3(256), 0, st, b.st, b.cellid,
                       b.cell_cnt, kp);
    launch_scan_clear(b, nc, st);
    hipLaunchKernelGGL(k_cells_scatter, dim3(nblk(kp.nrbc, 64)), dim3(64), 0, st, b.cellid,
                       b.cell_off, b.cell_cnt, b.cell_ids, kp.nrbc);
    // the sort leaves the fill counters at zero for the next call
    hipLaunchKernelGGL(k_cells_sort, dim3(nblk(nc, 64)), dim3(64), 0, st, b.cell_off,
                       b.cell_ids, b.cell_cnt, nc);
}

static inline unsigned grid8(long long units, int per_block)
{
    const long long b = (units + per_block - 1) / per_block;
    return (unsigned)((b + 7) / 8 * 8);
}

size_t map_couple_lds(int tile_max, int cand_cap, int real_bytes)
{
    return (((size_t)4 * tile_max * tile_max + 2 + 15) & ~(size_t)15) + (size_t)cand_cap * (real_bytes + 2 + 4) + 4;
}

size_t map_couple_tile_lds(int tile_max, int real_bytes)
{
    // raw kernel values, flags, then the covered-position list (2 bytes per entry; the
    // per-wavefront parts are rounded up to 64 entries)
    const size_t t3 = (size_t)tile_max * tile_max * tile_max;
    return ((t3 * (real_bytes + 1) + 1) & ~(size_t)1) + 2 * (t3 + MC_THREADS);
}

// the map pass instantiated for the field mode of u and sigma (FP32 arithmetic: compute
// precision, BF16 or scaled FP16; FP64 arithmetic: compute precision only)
template <typename RT, typename F>
static void with_field_mode(int field16, F&& f)
{
    if constexpr (sizeof(RT) == 4) {
        if (field16 == 1) return f(std::integral_constant<int, 1>{});
        if (field16 == 2) return f(std::integral_constant<int, 2>{});
    }
    f(std::integral_constant<int, 0>{});
}

template <typename RT>
void launch_map_couple(const CellBuffers& b, const KParams& kp, hipStream_t st)
{
    auto go = [&](auto fm) {
        hipLaunchKernelGGL((k_map_couple<RT, decltype(fm)::value>), dim3(grid8(kp.nrbc, 1)), dim3(64),
                           map_couple_lds(kp.tile_max, kp.cand_cap, (int)sizeof(RT)), st, b.st, b.cp,
                           (Gather<RT>*)b.gat, b.nodeword, b.tab.map, b.cnt, b.map_ids, b.map_vals,
                           b.cell_ids, b.u, b.sig, kp, b.err, b.ovf);
    };
    with_field_mode<RT>(kp.field16, go);
    // the overflow list is short (normally empty): a small grid loops over it
    hipLaunchKernelGGL((k_map_couple_tile<RT>), dim3(64), dim3(MC_THREADS),
                       map_couple_tile_lds(kp.tile_max, (int)sizeof(RT)), st, b.st, b.cp,
                       (Gather<RT>*)b.gat, b.nodeword, b.tab.map, b.cnt, b.map_ids, b.map_vals, b.ovf,
                       b.u,
                       b.sig, kp, b.err);
}

__global__ __launch_bounds__(256) void k_zero_ints(int* __restrict__ p, long long n)
{
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0;
}

void launch_zero_ints(int* p, long long n, hipStream_t st)
{
    if (n > 0) hipLaunchKernelGGL(k_zero_ints, dim3(nblk(n, 256)), dim3(256), 0, st, p, n);
}

void launch_gay_berne_out(const CellBuffers& b, const KParams& kp, double* F, double* T, int stride,
                          hipStream_t st)
{
    hipLaunchKernelGGL(k_gay_berne, dim3(grid8(kp.nrbc, 1)), dim3(64), 0, st, b.st, F, T, stride,
                       b.cell_ids, b.cell_off, b.cell_ids, b.wall_xyz, b.wcell_off, b.wcell_ids,
                       kp, b.err);
}

void launch_gay_berne(const CellBuffers& b, const KParams& kp, hipStream_t st)
{
    launch_gay_berne_out(b, kp, b.cp[0].Fm, b.cp[0].Tm, COUPLE_STRIDE, st);
}

void launch_rb_second_half(const CellBuffers& b, const KParams& kp, hipStream_t st)
{
    hipLaunchKernelGGL(k_rb_second_half, dim3(nblk(kp.nrbc, 64)), dim3(64), 0, st, b.st, b.cp, kp);
}

void launch_init_combined(const CellBuffers& b, const KParams& kp, hipStream_t st)
{
    hipLaunchKernelGGL(k_init_combined, dim3(nblk(kp.nrbc, 128)), dim3(128), 0, st, b.st, b.cp, kp);
}

int fused_blocks(const KParams& kp, int stage)
{
    const long long nc = (long long)kp.ncell[0] * kp.ncell[1] * kp.ncell[2];
    const int cells = kp.nrbc;
    switch (stage) {
    case FS_CELLS_A: return (int)nblk(cells, 256);
    case FS_SCAN: return cells > 0 ? 1 : 0;
    case FS_SCATTER: return (int)nblk(cells, 256);
    case FS_SORT: return cells > 0 ? (int)nblk(nc, 256) : 0;
    case FS_CLEAR: return cells > 0 ? (int)nblk(kp.N, 256) : 0;
    case FS_MAP: return cells;
    case FS_MAP_TILE: return cells > 0 ? FUSED_TILE_BLOCKS : 0;
    case FS_GB: return cells;
    case FS_RB2: return (int)nblk(cells, 128);
    case FS_STREAM: return (int)nblk(kp.N, 256);
    default: return 0;
    }
}

template <typename RT>
void launch_fused_cells(const FusedArgs& fa, int stage, size_t lds, hipStream_t st)
{
    const unsigned g = (unsigned)fa.start[fa.n];
    if (g == 0) return;
    switch (stage) {
    case FS_CELLS_A: hipLaunchKernelGGL(kf_cells_a, dim3(g), dim3(256), 0, st, fa); break;
    case FS_SCAN: hipLaunchKernelGGL(kf_scan, dim3(g), dim3(SCAN_THREADS), 0, st, fa); break;
    case FS_SCATTER: hipLaunchKernelGGL(kf_scatter, dim3(g), dim3(256), 0, st, fa); break;
    case FS_SORT: hipLaunchKernelGGL(kf_sort, dim3(g), dim3(256), 0, st, fa); break;
    case FS_MAP:
        with_field_mode<RT>(fa.field16, [&](auto fm) {
            hipLaunchKernelGGL((kf_map<RT, decltype(fm)::value>), dim3(g), dim3(64), lds, st, fa);
        });
        break;
    case FS_MAP_TILE: hipLaunchKernelGGL((kf_map_tile<RT>), dim3(g), dim3(MC_THREADS), lds, st, fa); break;
    case FS_GB: hipLaunchKernelGGL(kf_gb, dim3(g), dim3(64), 0, st, fa); break;
    case FS_RB2: hipLaunchKernelGGL(kf_kick, dim3(g), dim3(128), 0, st, fa); break;
    default: break;
    }
}

template void launch_fused_cells<double>(const FusedArgs&, int, size_t, hipStream_t);
template void launch_fused_cells<float>(const FusedArgs&, int, size_t, hipStream_t);
template void launch_map_couple<double>(const CellBuffers&, const KParams&, hipStream_t);
template void launch_map_couple<float>(const CellBuffers&, const KParams&, hipStream_t);


}  // namespace lbrbc
