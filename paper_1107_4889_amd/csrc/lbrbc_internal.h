// lbrbc_internal.h -- launchers shared between the kernel and API translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <utility>

#include "lbrbc_device.h"

namespace lbrbc {

// per-node kernels (lb_kernels.hip)
template <typename ST, typename RT>
void launch_stream_collide(const void* fin, void* fout, const uint32_t* nodeword, const int* ids,
                           const void* vals, const void* gat, void* u, void* sig,
                           const KParams& kp, unsigned* err, hipStream_t st);
template <typename ST, typename RT>
void launch_open_bc(const void* fin, void* fout, const uint32_t* nodeword, const long long* planes,
                    int nplane, const int* ids, const void* vals, const void* gat, void* u,
                    void* sig, const KParams& kp, hipStream_t st);
template <typename RT>
void launch_spread_field(const uint32_t* nodeword, const int* ids, const void* vals,
                         const void* gat, void* g, void* t, const KParams& kp, hipStream_t st);
void launch_clear_counts(uint32_t* nodeword, long long N, int* ovf, hipStream_t st);
template <typename ST, typename RT>
void launch_observe(const void* f, const uint32_t* nodeword, const void* u, const KParams& kp,
                    double* partials, int nblk, double* out, hipStream_t st);
template <typename RT>
void launch_wss(const void* sig, const long long* wn_node, const double* wn_nrm, int nwn,
                const KParams& kp, double* wss, double* acc, int accumulate, hipStream_t st);

// per-cell kernels (rbc_kernels.hip)
struct CellBuffers {
    RbcState* st;
    RbcCouple* cp;
    void* gat;            // Gather<RT>[nrbc]
    int* cellid;          // [nrbc]
    int* cell_cnt;        // [ncells]
    int* cell_off;        // [ncells + 1]
    int* cell_ids;        // [nrbc]
    const int* wall_xyz;  // [3 * nwall]
    const int* wcell_off; // [ncells + 1]
    const int* wcell_ids; // [nwall]
    uint32_t* nodeword;
    int* map_ids;         // [cap * ld] cell id per coverage slot
    void* map_vals;       // [cap * ld * 4] RT: raw kernel and its gradient per slot
    const void* u;        // [3 * ld] RT
    const void* sig;      // [6 * ld] RT
    unsigned* err;
    int* ovf;             // [1 + nrbc] overflow count, then cells for the full-tile map pass
};

void launch_rb_first_half(const CellBuffers& b, const KParams& kp, hipStream_t st);
void launch_cell_list(const CellBuffers& b, const KParams& kp, hipStream_t st);
template <typename RT>
void launch_map_couple(const CellBuffers& b, const KParams& kp, hipStream_t st);
size_t map_couple_lds(int tile_max, int cand_cap, int real_bytes);   // dynamic LDS, bytes
size_t map_couple_tile_lds(int tile_max, int real_bytes);
void launch_gay_berne(const CellBuffers& b, const KParams& kp, hipStream_t st);
enum { RB2_NOW = 0, RB2_ALL = 1, RB2_HYDRO = 2, RB2_KICK = 3 };
template <typename RT>
void launch_rb_second_half(const CellBuffers& b, const KParams& kp, int mode, hipStream_t st);
void launch_init_combined(const CellBuffers& b, const KParams& kp, hipStream_t st);
void launch_fill_u32(uint32_t* p, uint32_t v, long long n, hipStream_t st);

}  // namespace lbrbc
