// lbrbc_device.h -- device-side types and helpers of the MI355X library (gfx950).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

namespace lbrbc {

// ---- D3Q19 (Sec. II A) -------------------------------------------------------------------
// 0 rest; 1-6 axis speeds; 7-18 face diagonals; opposite speeds adjacent.
__host__ __device__ constexpr int cx_(int p)
{
    constexpr int t[19] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
    return t[p];
}
__host__ __device__ constexpr int cy_(int p)
{
    constexpr int t[19] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1};
    return t[p];
}
__host__ __device__ constexpr int cz_(int p)
{
    constexpr int t[19] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1};
    return t[p];
}
__host__ __device__ constexpr int opp_(int p) { return p == 0 ? 0 : ((p & 1) ? p + 1 : p - 1); }
__host__ __device__ constexpr double w_(int p)
{
    return p == 0 ? 1.0 / 3.0 : (p < 7 ? 1.0 / 18.0 : 1.0 / 36.0);
}

// ---- node word ---------------------------------------------------------------------------
// bits 0-18: bit p set <=> the pull source x - c_p is solid or outside a wall face
// bit 19: fluid node; bit 20: has an in-box solid neighbour (wall-adjacent);
// bit 21: open-boundary plane node; bit 22: fluid node next to an open-plane node along z
// (the boundary kernel extrapolates from it). The coverage counts live in arrays of their own.
constexpr uint32_t NW_FLUID = 1u << 19;
constexpr uint32_t NW_WALLADJ = 1u << 20;
constexpr uint32_t NW_OPEN = 1u << 21;
constexpr uint32_t NW_OPEN_INNER = 1u << 22;
constexpr int CAP_MAX = 12;

// device fault bits
constexpr unsigned ERR_UNSTABLE = 1u, ERR_OVERLAP = 2u, ERR_CAPACITY = 4u;

// ---- parameters (kernel argument, by value) ----------------------------------------------
struct KParams {
    int nx, ny, nz;
    int per[3];
    long long N;      // storage slots: 64 per stored row segment (the nodes of the compact layout)
    long long ld;     // plane stride (N rounded up)
    int nbx;          // 64-node column segments per lattice row, ceil(nx / 64)
    int compact;      // 1: compact layout (only the row segments holding fluid are stored)
    int forcing;
    int cap;
    double tau0, delta, kappa;
    int kappa_int;    // kappa if it is an integer in [0, 64], else -1
    double gext[3];
    double gammaT, gammaR, alpha, mass, inertia[3], vort_scale;
    double ext_force[3], ext_torque[3];   // on every cell: lab force, body torque
    double xi[3], axes[3], eps0, a_wall, sigmin_wall;
    int wall_particles;
    int open_z;
    double rho_in, rho_out;
    float f16_scale, f16_inv;
    int nrbc;
    int ncell[3];
    double cedge[3];
    int wncell[3];    // grid of the wall points (edge >= rc_wall)
    double wcedge[3];
    double rc;        // cell-list cut-off (bounds every pair kind)
    double rc_pair;   // cell-cell Gay-Berne cut-off bound
    double rc_wall;   // cell-wall Gay-Berne cut-off bound
    int tile_max;     // LDS tile edge bound
    int cand_cap;     // candidate nodes per cell held in LDS by the one-wavefront map pass
    int ent_shift;    // log2 of the coverage entries reserved per cell
    int bf16_sr;      // BF16 storage with stochastic rounding
    int moving_walls; // wall_u_lo or wall_u_hi nonzero
    double uw_lo[3], uw_hi[3];   // velocities of the solid nodes below / from the mid-plane y = ny/2
    int field16;      // 16-bit storages: u and sigma in BF16 (1) or FP16 times 2^12 (2), coverage
                      // entries in FP16 times 2^8 (both); 0: all in the compute precision
};

// ---- compact layout -------------------------------------------------------------------------
// Only the 64-node row segments (x0 = 64 b, y, z) that hold a fluid node are stored, one after
// another: node (x, y, z) of stored segment s has storage index k = 64 s + (x - x0). Tables:
//   seg[s]           (x0, y, z, 0) of stored segment s;
//   segnb[27 s + e]  the stored segment holding the neighbouring column segment (dx, dy, dz) in
//                    {-1, 0, 1}^3, e = (dx + 1) + 3 (dy + 1) + 9 (dz + 1), where dx = -1 is the
//                    segment of x0 - 1 and dx = +1 that of the first node past the segment
//                    (wrapped on periodic axes); -1 when it is outside the box or not stored;
//   segmap[b + nbx (y + ny z)]  stored segment of column segment b of row (y, z), or -1.
struct SegTables {
    const int4* seg;
    const int* nb;
    const int* map;
};

// storage index of node (X, Y, Z): x + nx (y + ny z) in the dense layout; in the compact one
// from the segment map, -1 when the node's row segment is not stored (the node is solid)
__device__ __forceinline__ int storage_of(const int* __restrict__ segmap, const KParams& kp, int X, int Y, int Z)
{
    if (!kp.compact) return X + kp.nx * (Y + kp.ny * Z);
    const int s = segmap[(X >> 6) + kp.nbx * (Y + kp.ny * Z)];
    return s < 0 ? -1 : (s << 6) | (X & 63);
}

// ---- per-cell records ---------------------------------------------------------------------
struct RbcState {        // FP64, lab frame except Om (body) and Tc (body)
    double R[3], Q[9], V[3], Om[3];
    double Fc[3], Tc[3];     // combined force (lab) / torque (body)
    double Vh[3], Omh[3];    // after the first half
};
struct RbcCouple {       // interpolation results and forces
    double S, ut[3], wt[3], TS[3];
    double Fm[3], Tm[3];     // Gay-Berne force (lab), torque (body)
    double Fh[3], Th[3];     // hydrodynamic force / torque (lab)
};
// doubles between consecutive cells' records (the Gay-Berne pass writes Fm and Tm with it)
constexpr int COUPLE_STRIDE = (int)(sizeof(RbcCouple) / sizeof(double));
static_assert(sizeof(RbcCouple) % sizeof(double) == 0, "RbcCouple holds doubles only");

// Record read by the per-node spreading: hydrodynamic force and torque (lab) and 1/S in
// the compute precision (32 B for float, 64 B for double).
template <typename RT>
struct alignas(16) Gather {
    RT F[3];
    RT invS;
    RT T[3];
    RT pad;
};

// ---- storage conversions ------------------------------------------------------------------
// Loads and stores take a per-plane base (scalar registers) and a 32-bit element offset; the
// byte offset i * sizeof(T) is formed in 32 bits so that the access is base + zero-extended
// offset. lb_init rejects lattices whose padded planes would reach 4 GiB (more than
// 2^29 - 4096 nodes with 8-byte elements, 2^30 - 4096 otherwise), so the offset never wraps.
struct bf16_t { uint16_t v; };

template <typename T>
__device__ __forceinline__ const T* at32(const T* base, unsigned i)
{
    return reinterpret_cast<const T*>(reinterpret_cast<const char*>(base) + i * (unsigned)sizeof(T));
}
template <typename T>
__device__ __forceinline__ T* at32(T* base, unsigned i)
{
    return reinterpret_cast<T*>(reinterpret_cast<char*>(base) + i * (unsigned)sizeof(T));
}

template <typename ST, typename RT>
struct Store;
template <>
struct Store<double, double> {
    __device__ static double ld(const double* p, unsigned i, float) { return *at32(p, i); }
    __device__ static void st(double* p, unsigned i, double v, float) { __builtin_nontemporal_store(v, at32(p, i)); }
};
template <>
struct Store<float, float> {
    __device__ static float ld(const float* p, unsigned i, float) { return *at32(p, i); }
    __device__ static void st(float* p, unsigned i, float v, float) { __builtin_nontemporal_store(v, at32(p, i)); }
};
template <>
struct Store<bf16_t, float> {
    __device__ static float ld(const bf16_t* p, unsigned i, float)
    {
        uint32_t u = (uint32_t)*at32(reinterpret_cast<const uint16_t*>(p), i) << 16;
        return __uint_as_float(u);
    }
    __device__ static void st(bf16_t* p, unsigned i, float v, float)
    {
        // round to nearest even on the upper 16 bits
        uint32_t u = __float_as_uint(v);
        uint16_t r;
        if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x007fffffu)) r = 0x7fc0;
        else r = (uint16_t)((u + 0x7fffu + ((u >> 16) & 1u)) >> 16);
        __builtin_nontemporal_store(r, at32(reinterpret_cast<uint16_t*>(p), i));
    }
};
// Stochastic rounding of FP32 to BF16: add 16 random bits below the kept mantissa, then
// truncate (rounds up with probability equal to the dropped fraction: unbiased). The bits
// are the MurmurHash3 32-bit finalizer of the node, the direction and the value.
__device__ __forceinline__ uint32_t fmix32(uint32_t h)
{
    h ^= h >> 16;
    h *= 0x85ebca6bu;
    h ^= h >> 13;
    h *= 0xc2b2ae35u;
    h ^= h >> 16;
    return h;
}
__device__ __forceinline__ void store_bf16_sr(bf16_t* p, unsigned i, float v, unsigned dir)
{
    const uint32_t u = __float_as_uint(v);
    uint16_t r;
    if ((u & 0x7f800000u) == 0x7f800000u) r = (u & 0x007fffffu) ? 0x7fc0 : (uint16_t)(u >> 16);
    else r = (uint16_t)((u + (fmix32(i * 0x9e3779b1u ^ dir * 0x85ebca77u ^ u) & 0xffffu)) >> 16);
    __builtin_nontemporal_store(r, at32(reinterpret_cast<uint16_t*>(p), i));
}

// store of population `dir` at node i: the storage's own rounding, or stochastic for BF16
template <typename ST, typename RT>
__device__ __forceinline__ void store_pop(ST* p, unsigned i, RT v, const KParams& kp, unsigned dir)
{
    if constexpr (std::is_same<ST, bf16_t>::value) {
        if (kp.bf16_sr) {
            store_bf16_sr(p, i, v, dir);
            return;
        }
    }
    Store<ST, RT>::st(p, i, v, kp.f16_scale);
}

template <>
struct Store<_Float16, float> {
    __device__ static float ld(const _Float16* p, unsigned i, float inv) { return (float)*at32(p, i) * inv; }
    __device__ static void st(_Float16* p, unsigned i, float v, float scale)
    {
        __builtin_nontemporal_store((_Float16)(v * scale), at32(p, i));
    }
};

// reciprocal and square roots in the compute precision: the hardware instructions (1 ulp)
// for float, correctly rounded for double
__device__ __forceinline__ float recip(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double recip(double x) { return 1.0 / x; }
__device__ __forceinline__ float fast_sqrt(float x) { return __builtin_amdgcn_sqrtf(x); }
__device__ __forceinline__ double fast_sqrt(double x) { return sqrt(x); }
__device__ __forceinline__ float fast_rsqrt(float x) { return __builtin_amdgcn_rsqf(x); }
__device__ __forceinline__ double fast_rsqrt(double x) { return 1.0 / sqrt(x); }

// Coverage: per node, a count and up to `cap` slot planes of entry indices
// e = (cell << ent_shift) | j; entry e holds (raw, grad raw) of the j-th covered node of that
// cell, cell-major. Two such sets alternate with the step's parity, so the next step's map
// pass can fill one while the stream-collide reads the other.
template <typename RT>
struct MapPlanes {
    const int* ids[CAP_MAX];
    const void* vals0;   // entries (see store_entry)
    uint32_t* cnt;
};

// Velocity and stress are stored node-interleaved, u[3k + a] and sigma[6k + q] (q: xx yy zz xy
// xz yz): the map pass reads them at the few consecutive covered nodes of each support row, so
// one node's components share a cache line instead of sitting in 3 and 6 separate planes. The
// stream-collide writes them for consecutive nodes, which stays contiguous per wavefront.
// Their element type is the compute precision for FP64 and FP32 storage. The 16-bit storages
// keep them in 16 bits as well (KParams::field16): BF16 rounded to nearest even, or FP16
// holding the value times 2^12 (|value| < 16; the velocity is bounded by 0.3 and the stress far
// below that). A 16-bit velocity record is padded to four elements, so that a node's u is one
// aligned 8-byte word and its sigma three 4-byte words.
template <typename ST, typename RT>
struct FieldOf {
    using T = RT;
};
template <>
struct FieldOf<bf16_t, float> {
    using T = bf16_t;
};
template <>
struct FieldOf<_Float16, float> {
    using T = _Float16;
};
constexpr float FIELD16_SCALE = 4096.0f, FIELD16_INV = 1.0f / 4096.0f;
template <typename FT>
constexpr unsigned vel_stride() { return sizeof(FT) == 2 ? 4u : 3u; }

template <typename FT>
__device__ __forceinline__ FT* vel_of(FT* u, unsigned k) { return u + vel_stride<FT>() * (size_t)k; }
template <typename FT>
__device__ __forceinline__ const FT* vel_of(const FT* u, unsigned k) { return u + vel_stride<FT>() * (size_t)k; }
template <typename FT>
__device__ __forceinline__ FT* str_of(FT* s, unsigned k) { return s + 6 * (size_t)k; }
template <typename FT>
__device__ __forceinline__ const FT* str_of(const FT* s, unsigned k) { return s + 6 * (size_t)k; }

// 16-bit field codes (low 16 bits of the result)
__device__ __forceinline__ uint32_t bf16_rne_bits(float v)
{
    const uint32_t u = __float_as_uint(v);
    if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x007fffffu)) return 0x7fc0u;
    return (u + 0x7fffu + ((u >> 16) & 1u)) >> 16;
}
template <typename FT>
__device__ __forceinline__ uint32_t field_code(float v)
{
    if constexpr (std::is_same<FT, bf16_t>::value) return bf16_rne_bits(v);
    else return (uint32_t)__builtin_bit_cast(uint16_t, (_Float16)(v * FIELD16_SCALE));
}
__device__ __forceinline__ float field_value(uint32_t h, int mode)
{
    h &= 0xffffu;
    return mode == 1 ? __uint_as_float(h << 16)
                     : (float)__builtin_bit_cast(_Float16, (uint16_t)h) * FIELD16_INV;
}

// streaming (non-temporal) stores of one node's u and sigma as a few vector stores
template <typename FT, typename RT>
__device__ __forceinline__ void store_vel_nt(FT* p, RT a, RT b, RT c)
{
    if constexpr (sizeof(FT) == 2) {
        // the padded record: one 8-byte store
        typedef uint32_t V2 __attribute__((ext_vector_type(2)));
        const V2 v = {field_code<FT>(a) | field_code<FT>(b) << 16, field_code<FT>(c)};
        __builtin_nontemporal_store(v, reinterpret_cast<V2*>(p));
    } else if constexpr (sizeof(FT) == 4) {
        // one 12-byte store (the 3-vector's store size; its 16-byte allocation size is not used)
        typedef FT V3 __attribute__((ext_vector_type(3), aligned(4)));
        const V3 v = {a, b, c};
        __builtin_nontemporal_store(v, reinterpret_cast<V3*>(p));
    } else {
        // a 3-vector of doubles is stored as 32 bytes: element stores instead
        __builtin_nontemporal_store(a, p);
        __builtin_nontemporal_store(b, p + 1);
        __builtin_nontemporal_store(c, p + 2);
    }
}
template <typename FT, typename RT>
__device__ __forceinline__ void store_str_nt(FT* p, RT s0, RT s1, RT s2, RT s3, RT s4, RT s5)
{
    if constexpr (sizeof(FT) == 2) {
        // 12 bytes at 12k: one 3-word store
        typedef uint32_t V3 __attribute__((ext_vector_type(3), aligned(4)));
        const V3 v = {field_code<FT>(s0) | field_code<FT>(s1) << 16, field_code<FT>(s2) | field_code<FT>(s3) << 16,
                      field_code<FT>(s4) | field_code<FT>(s5) << 16};
        __builtin_nontemporal_store(v, reinterpret_cast<V3*>(p));
    } else {
        typedef FT V2 __attribute__((ext_vector_type(2)));   // 6k elements: aligned to 2 elements
        const V2 a = {s0, s1}, b = {s2, s3}, c = {s4, s5};
        __builtin_nontemporal_store(a, reinterpret_cast<V2*>(p));
        __builtin_nontemporal_store(b, reinterpret_cast<V2*>(p + 2));
        __builtin_nontemporal_store(c, reinterpret_cast<V2*>(p + 4));
    }
}

// one node's u and sigma in the compute precision, from fields of either element type (the
// per-cell and reduction kernels serve every storage of a compute precision). FM: the field mode
// (KParams::field16) when the caller's instantiation fixes it, or -1 to read it from kp.
template <typename RT, int FM = -1>
__device__ __forceinline__ void load_vel(const void* u, unsigned k, const KParams& kp, RT out[3])
{
    if constexpr (sizeof(RT) == 4 && FM != 0) {
        const int m = FM > 0 ? FM : kp.field16;
        if (m) {
            typedef uint32_t V2 __attribute__((ext_vector_type(2)));
            const V2 w = *(reinterpret_cast<const V2*>(u) + k);
            out[0] = field_value(w.x, m);
            out[1] = field_value(w.x >> 16, m);
            out[2] = field_value(w.y, m);
            return;
        }
    }
    const RT* p = static_cast<const RT*>(u) + 3 * (size_t)k;
    out[0] = p[0];
    out[1] = p[1];
    out[2] = p[2];
}
template <typename RT, int FM = -1>
__device__ __forceinline__ void load_str(const void* s, unsigned k, const KParams& kp, RT out[6])
{
    if constexpr (sizeof(RT) == 4 && FM != 0) {
        const int m = FM > 0 ? FM : kp.field16;
        if (m) {
            const uint32_t* p = static_cast<const uint32_t*>(s) + 3 * (size_t)k;
            const uint32_t w0 = p[0], w1 = p[1], w2 = p[2];
            out[0] = field_value(w0, m);
            out[1] = field_value(w0 >> 16, m);
            out[2] = field_value(w1, m);
            out[3] = field_value(w1 >> 16, m);
            out[4] = field_value(w2, m);
            out[5] = field_value(w2 >> 16, m);
            return;
        }
    }
    const RT* p = static_cast<const RT*>(s) + 6 * (size_t)k;
#pragma unroll
    for (int q = 0; q < 6; ++q) out[q] = p[q];
}

// field mode of a storage (KParams::field16) at compile time
template <typename ST>
constexpr int field_mode_of()
{
    return std::is_same<ST, bf16_t>::value ? 1 : (std::is_same<ST, _Float16>::value ? 2 : 0);
}

// Coverage entry e: (raw kernel, grad raw) of one (cell, covered node) pair, written by the map
// pass and read by the spreading. Four values in the compute precision; for the 16-bit storages
// four FP16 values holding 2^8 times the value (raw <= 1/8 and |grad raw| <= 1/8 for the Peskin
// kernel), one 8-byte word. FM as for load_vel.
constexpr float ENTRY16_SCALE = 256.0f, ENTRY16_INV = 1.0f / 256.0f;
__device__ __forceinline__ uint32_t entry_code(float v)
{
    return (uint32_t)__builtin_bit_cast(uint16_t, (_Float16)(v * ENTRY16_SCALE));
}
__device__ __forceinline__ float entry_value(uint32_t h)
{
    return (float)__builtin_bit_cast(_Float16, (uint16_t)(h & 0xffffu)) * ENTRY16_INV;
}
template <typename RT, int FM = -1>
__device__ __forceinline__ void store_entry(void* vals, size_t e, const KParams& kp, RT r, RT gx, RT gy, RT gz)
{
    if constexpr (sizeof(RT) == 4 && FM != 0) {
        if (FM > 0 || kp.field16) {
            typedef uint32_t V2 __attribute__((ext_vector_type(2)));
            const V2 w = {entry_code(r) | entry_code(gx) << 16, entry_code(gy) | entry_code(gz) << 16};
            *(reinterpret_cast<V2*>(vals) + e) = w;
            return;
        }
    }
    RT* v = static_cast<RT*>(vals) + 4 * e;
    v[0] = r;
    v[1] = gx;
    v[2] = gy;
    v[3] = gz;
}
template <typename RT, int FM = -1>
__device__ __forceinline__ void load_entry(const void* vals, size_t e, const KParams& kp, RT& r, RT& gx, RT& gy,
                                           RT& gz)
{
    if constexpr (sizeof(RT) == 4 && FM != 0) {
        if (FM > 0 || kp.field16) {
            typedef uint32_t V2 __attribute__((ext_vector_type(2)));
            const V2 w = *(reinterpret_cast<const V2*>(vals) + e);
            r = entry_value(w.x);
            gx = entry_value(w.x >> 16);
            gy = entry_value(w.y);
            gz = entry_value(w.y >> 16);
            return;
        }
    }
    const RT* v = static_cast<const RT*>(vals) + 4 * e;
    r = v[0];
    gx = v[1];
    gy = v[2];
    gz = v[3];
}

// per-plane pointers of one stream-collide launch (kernel argument)
template <typename ST, typename RT>
struct Planes {
    using FT = typename FieldOf<ST, RT>::T;
    const ST* in[19];
    ST* out[19];
    FT* u;
    FT* sig;
    __device__ const ST* src(int p) const { return in[p]; }
    __device__ ST* dst(int p) const { return out[p]; }
};
// the same planes from the buffer bases and the plane stride (fused multi-lattice launches)
template <typename ST, typename RT>
struct PlanesLd {
    using FT = typename FieldOf<ST, RT>::T;
    const ST* fin;
    ST* fout;
    FT* u;
    FT* sig;
    unsigned long long ld;
    __device__ const ST* src(int p) const { return fin + (unsigned long long)p * ld; }
    __device__ ST* dst(int p) const { return fout + (unsigned long long)p * ld; }
};

// ---- Peskin four-point kernel at r = 2|y|/xi (the normalised 1-D profile) ----------------
template <typename RT>
__device__ __forceinline__ RT peskin(RT r)
{
    // both pieces with one square root (selects): (3 - 2r + sqrt(1 + 4r - 4r^2)) / 8 on
    // [0, 1], (5 - 2r - sqrt(-7 + 12r - 4r^2)) / 8 on (1, 2), 0 beyond. The second piece
    // falls to exactly 0 at r = 2, where the rounded square root can exceed 5 - 2r by an ulp:
    // the kernel is clamped at its true lower bound 0, so a value is never negative (the map
    // pass reads a negative value as "outside the support")
    r = fabs(r);
    const bool in1 = r <= RT(1);
    const RT q = in1 ? RT(1) + RT(4) * r - RT(4) * r * r : RT(-7) + RT(12) * r - RT(4) * r * r;
    const RT sq = fast_sqrt(q > RT(0) ? q : RT(0));
    const RT v = (in1 ? RT(3) - RT(2) * r + sq : RT(5) - RT(2) * r - sq) * RT(0.125);
    return r < RT(2) && v > RT(0) ? v : RT(0);
}

__device__ __forceinline__ double min_img(double d, double L, int per)
{
    // one period at most (selects, no branches)
    d = (per && d > 0.5 * L) ? d - L : d;
    d = (per && d < -0.5 * L) ? d + L : d;
    return d;
}

// body coordinates y = Q^T d, each component summed left to right with no contraction, so
// that the support test |y_a| < xi_a is reproducible bit for bit
__device__ __forceinline__ void body_coords_exact(const double* Q, double d0, double d1, double d2,
                                                  double y[3])
{
#pragma clang fp contract(off)
    for (int a = 0; a < 3; ++a) {
        double t0 = Q[0 * 3 + a] * d0;
        double t1 = Q[1 * 3 + a] * d1;
        double t2 = Q[2 * 3 + a] * d2;
        y[a] = (t0 + t1) + t2;
    }
}

template <typename RT>
__device__ __forceinline__ RT ipow_or_pow(RT b, double kappa, int kint)
{
    if (kint >= 0) {
        RT r = RT(1), x = b;
        int k = kint;
        while (k) {
            if (k & 1) r *= x;
            x *= x;
            k >>= 1;
        }
        return r;
    }
    return pow(b, (RT)kappa);
}

}  // namespace lbrbc
