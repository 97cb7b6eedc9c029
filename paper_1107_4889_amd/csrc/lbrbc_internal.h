// lbrbc_internal.h -- launchers shared between the kernel and API translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <utility>

#include "lbrbc_device.h"

namespace lbrbc {

// per-node kernels (lb_kernels.hip)
// clear_counts: also clear the coverage counts for the next step (no open planes)
template <typename ST, typename RT>
void launch_stream_collide(const void* fin, void* fout, const uint32_t* nodeword, const int* ids,
                           const void* vals, uint32_t* cnt, const void* gat, void* u, void* sig,
                           const KParams& kp, unsigned* err, bool clear_counts, const SegTables& tab,
                           int nseg, unsigned* ctr, int par, hipStream_t st);
// planes: per open-plane node (k, k of its inner neighbour, x | y << 16, z)
template <typename ST, typename RT>
void launch_open_bc(const void* fin, void* fout, const uint32_t* nodeword, const int4* planes,
                    int nplane, const int* ids, const void* vals, uint32_t* cnt, const void* gat, void* u,
                    void* sig, const KParams& kp, const SegTables& tab, bool clear_counts, unsigned* ctr,
                    int par, hipStream_t st);
template <typename RT>
void launch_spread_field(const uint32_t* nodeword, const int* ids, const void* vals, uint32_t* cnt,
                         const void* gat, void* g, void* t, const KParams& kp, hipStream_t st);
void launch_clear_counts(uint32_t* cnt, long long N, int* ovf, hipStream_t st);
template <typename ST, typename RT>
void launch_observe(const void* f, const uint32_t* nodeword, const void* u, const KParams& kp,
                    double* partials, int nblk, double* out, hipStream_t st);
template <typename RT>
void launch_wss(const void* sig, const long long* wn_node, const double* wn_nrm, int nwn,
                const KParams& kp, double* wss, double* acc, int accumulate, hipStream_t st);

// per-cell kernels (rbc_kernels.hip)
// cell counts per block of the multi-block cell-list scan (256 threads, four counts each)
constexpr int CELL_SCAN_CHUNK = 1024;

struct CellBuffers {
    RbcState* st;
    RbcCouple* cp;
    void* gat;            // Gather<RT>[nrbc]
    int* cellid;          // [nrbc]
    int* cell_cnt;        // [ncells]
    int* cell_off;        // [ncells + 1]
    int* cell_part;       // [ceil(ncells / CELL_SCAN_CHUNK)] chunk totals of the multi-block scan
    int* cell_ids;        // [nrbc]
    const int* wall_xyz;  // [3 * nwall]
    const int* wcell_off; // [ncells + 1]
    const int* wcell_ids; // [nwall]
    uint32_t* nodeword;   // static bits per node (fluid, bounce-back, wall, open planes)
    SegTables tab;        // compact layout: stored segments, their neighbours, the segment map
    unsigned* step_ctr;   // [2] step counter, read and advanced by the stream-collide
    // one of the two coverage sets (chosen by the step's parity)
    int* map_ids;         // [cap * ld] entry index per coverage slot
    void* map_vals;       // [entries * 4] RT: raw kernel and its gradient per entry
    uint32_t* cnt;        // [ld] coverage count per node
    const void* u;        // [3 * ld] RT
    const void* sig;      // [6 * ld] RT
    unsigned* err;
    int* ovf;             // [1 + nrbc] overflow count, then cells for the full-tile map pass
};

// ---- fused multi-lattice launches -----------------------------------------------------------
// Everything a fused launch needs about one context; kept in the context's arena.
struct SlotDesc {
    KParams kp;
    CellBuffers b;
    void* fA;            // population buffers A and B of the arena
    void* fB;
};
// Kernel argument of a fused launch over up to FUSE_MAX contexts: block b belongs to the slot
// s with start[s] <= b < start[s + 1]; parity bit s: slot s reads B and writes A this step.
constexpr int FUSE_MAX = 64;
struct FusedArgs {
    const SlotDesc* slot[FUSE_MAX];
    int start[FUSE_MAX + 1];
    int n;
    int field16;          // KParams::field16 of the slots (host side: selects the map pass)
    unsigned long long parity;
};
// one step of every slot; every slot has the same storage type ST/RT, no open boundary and
// no WSS accumulation
enum FusedStage { FS_CELLS_A, FS_SCAN, FS_SCATTER, FS_SORT, FS_CLEAR, FS_MAP, FS_MAP_TILE, FS_GB,
                  FS_RB2, FS_STREAM, FS_NSTAGES };
int fused_blocks(const KParams& kp, int stage);    // blocks of one slot in a stage
// per-cell stages (FS_CELLS_A .. FS_RB2 except FS_CLEAR); lds: dynamic LDS of FS_MAP and
// FS_MAP_TILE (the largest over the slots)
template <typename RT>
void launch_fused_cells(const FusedArgs& fa, int stage, size_t lds, hipStream_t st);
// per-node stages (FS_CLEAR, FS_STREAM)
template <typename ST, typename RT>
void launch_fused_lattice(const FusedArgs& fa, int stage, hipStream_t st);

// slot of block b of a fused launch, and the block's index within the slot
__device__ __forceinline__ int fused_slot_at(const FusedArgs& fa, int b, int& lb)
{
    int lo = 0, hi = fa.n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (fa.start[mid] <= b) lo = mid;
        else hi = mid - 1;
    }
    lb = b - fa.start[lo];
    return lo;
}
__device__ __forceinline__ int fused_slot(const FusedArgs& fa, int& lb)
{
    return fused_slot_at(fa, (int)blockIdx.x, lb);
}

void launch_cell_list(const CellBuffers& b, const KParams& kp, hipStream_t st);
// first rigid-body half fused with the binning, then the rest of the cell list
void launch_rb1_cell_list(const CellBuffers& b, const KParams& kp, hipStream_t st);
template <typename RT>
void launch_map_couple(const CellBuffers& b, const KParams& kp, hipStream_t st);
size_t map_couple_lds(int tile_max, int cand_cap, int real_bytes);   // dynamic LDS, bytes
size_t map_couple_tile_lds(int tile_max, int real_bytes);
void launch_gay_berne(const CellBuffers& b, const KParams& kp, hipStream_t st);
// the same forces and torques into F[stride i + a] (lab) and T[stride i + a] (body)
void launch_gay_berne_out(const CellBuffers& b, const KParams& kp, double* F, double* T, int stride,
                          hipStream_t st);
// zero n ints (a kernel, so it can be captured into a graph)
void launch_zero_ints(int* p, long long n, hipStream_t st);
// combined force and torque, friction and half kick (the map pass has written F^hyd, T^hyd
// and the gather records)
void launch_rb_second_half(const CellBuffers& b, const KParams& kp, hipStream_t st);
void launch_init_combined(const CellBuffers& b, const KParams& kp, hipStream_t st);

}  // namespace lbrbc
