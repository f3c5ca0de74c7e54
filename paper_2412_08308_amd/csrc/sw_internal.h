// Internal declarations shared by the gfx950 kernels and the host runtime.
//
// Terminology (query Q of m residues along rows i, subject D of n residues
// along columns j, as in the paper's Section 2.2 recurrence):
//   R      query rows a lane keeps in registers (a "row block")
//   K      lanes that cooperate on one subject (a pipelined group)
//   pass   one sweep over all columns of a subject covering K row blocks
//   item   the work of one wavefront: 64/K subjects (int32 path) or 128/K
//          subjects (packed 16-bit path), all of one query
//   slot   per-wavefront scratch in the workspace that carries the bottom row
//          (H - Go, F) of one pass to the first row of the next pass
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

namespace swdb {

constexpr int kAlpha = 32;           // residue codes 0..31 accepted at the ABI
constexpr int kCodes = 33;           // + internal pad code
constexpr uint8_t kPad = 32;         // pad code: subject tails and chunk fill
constexpr int kWave = 64;
constexpr int kXcds = 8;             // accelerator dies of the device, an L2 each; workgroups go to them in turn
constexpr int kRescoreMaxWaves = 8; // wavefronts of a rescore workgroup, at most
constexpr int kFlagSortCap = 4096;   // overflow lists up to this length are sorted by cost
constexpr int kI16Rows = 24;       // query rows per lane of the packed 16-bit variant

// Bytes between the profile entries of consecutive residue codes in one row
// block: R entries of ES bytes plus at least 8 spare bytes, in 16-byte units
// (aligned loads).  For the database search's 8-bit row blocks (24 or 32
// rows), whose profile is staged in LDS, an odd number of units, so that the
// reads of lanes with different codes start on different LDS bank groups for
// every code difference below 16 (an even number aliased codes 8 apart).
// 16-bit row blocks keep the narrower stride: the wider one pushed the
// 567-residue query's packed profile past the 64 KiB a workgroup stages in
// LDS by default, and measured 4% slower.  The single-pair kernel's short row
// blocks read their profile through the cache hierarchy, where a wider stride
// would only grow the footprint.
__host__ __device__ constexpr int code_stride(int R, int ES)
{
    return (ES == 1 && R >= 24 ? ((R + 8 + 15) / 16 | 1) : (R * ES + 8 + 15) / 16) * 16;
}

// Work item (one wavefront).  meta = nsub | K << 16 | critical << 24 (K =
// lanes per subject, 1..64, floor(64 / K) lane groups per wavefront; critical
// marks items whose per-lane work is far above the planner's target).
struct Item {
    int32_t s0;      // first sorted subject index
    int32_t ncols;   // columns to sweep: longest subject of the item, rounded up to 4
    int32_t q;       // query index in the batch
    int32_t meta;
};

// Per-query descriptor, built on the host, uploaded with the items.
struct QueryDesc {
    int64_t prof_off;   // byte offset of this query's profile in the profile area
    int32_t m;          // query length
    int32_t nbr;        // row blocks: ceil(m / R)
    int32_t prof_bytes; // (nbr + 1) * 33 * code_stride(R, entry bytes)
    int32_t lds;        // 1: profile staged in LDS; 0: read from global memory
    int32_t item_begin; // first work item of this query in the item array
    int32_t item_count; // number of work items of this query
    int32_t out_row;    // row of the score matrix this query writes
    int32_t pad;
};

// Status words at the start of a search workspace, cleared by the first
// launch group of every search call and accumulated over its groups (int32
// each): a query residue code >= 32 was seen; subjects the exact rescore gave
// up on (their score is stored as -1); subjects sent to the rescore; work
// items the search kernel skipped as inconsistent with its launch.
constexpr int kStatusBytes = 256;
constexpr int kStatusBadQuery = 0;
constexpr int kStatusRescoreFailed = 1;
constexpr int kStatusFlagged = 2;
constexpr int kStatusBadItems = 3;

struct Matrix8 {
    int8_t v[kAlpha * kAlpha];   // [query residue][subject residue]
};

struct SearchArgs {
    // prepared database
    const uint8_t* res;          // lane-interleaved residues (16 per lane per block)
    const int64_t* chunk_off;    // byte offset of each 64-subject chunk
    const int32_t* perm;         // sorted index -> caller's index
    const int32_t* slen;         // sorted index -> length
    int32_t nseq;
    // plan
    const Item* items;           // every query's items, queries in queue order
    const QueryDesc* qd;         // queue order (largest query first)
    int32_t nq;
    int32_t* heads;              // [nq] per-query queue heads
    int64_t n_items;             // entries of items
    const uint8_t* prof;         // profile area (global)
    // outputs and scratch
    int32_t* scores;             // [nq][out_stride]
    int64_t out_stride;
    int32_t* counters;           // [1] overflow-flag count, [2] rescore queue head (per launch group)
    int32_t* status;             // status words (kStatus*)
    int2* bnd;                   // slots
    int64_t slot_elems;          // int2 entries per slot
    int2* flags;                 // (q, sorted subject) of 16-bit overflows
    int32_t flag_cap;
    int32_t go, ge;
};

struct ProfileArgs {
    const uint8_t* queries;      // concatenated query residues (device)
    const int64_t* q_off;        // device copy of offsets
    const QueryDesc* qd;
    uint8_t* prof;
    int32_t* bad;                // set to 1 if a query residue code is >= 32 (null: read codes modulo 32)
    int32_t nq;
    int32_t go;
    int32_t pad;                 // entry of pad codes and pad rows
    Matrix8 sm;
};

// One anti-diagonal of tiles of a single long pair (query rows x subject
// columns).  Band b holds rows [b*K*R, (b+1)*K*R), lane g of its group rows
// [(b*K + g)*R, +R); chunk c holds columns [c*wc, (c+1)*wc).  Tiles (b, c)
// with b + c = d run in one launch; boundaries pass between launches through
// three buffers updated in place (each is read by a tile before that tile
// overwrites it, and no two tiles of a launch share an entry):
//   rowbuf[col]  (H - Go, F) of the bottom row of the band above, per column
//   colbuf[row]  (H - Go, E) of the last column of the chunk to the left, per row
//   corner[b*3 + c%3]  H - Go of the bottom-right cell of tile (b-1, c-1)
struct PairArgs {
    const uint8_t* subj;         // subject codes padded with the pad code to nc*wc (16-byte aligned)
    const uint8_t* prof;         // query profile (nbr + 1 row blocks)
    int2* rowbuf;                // [nc * wc]
    int2* colbuf;                // [nb * K * R]
    int32_t* corner;             // [(nb + 1) * 3]
    int32_t* score;              // [1] running maximum (atomicMax)
    int32_t nbr;                 // query row blocks: ceil(m / R)
    int32_t nb, nc;              // bands, column chunks
    int32_t K, wc;               // lanes per band, columns per chunk (multiple of 16)
    int32_t go, ge;
    int32_t d;                   // anti-diagonal: b + c
    int32_t b_lo, ntiles;        // first band on the diagonal, tiles on it
    // traceback pass only (8 rows per lane): per cell a 4-bit code, bits 0-1
    // the source of H (0: H = 0, 1: diagonal, 2: E, 3: F), bit 2 E opened
    // (from H) rather than extended, bit 3 the same for F; column-major, one
    // 32-bit word per 8 rows: dir[col * dir_stride + row / 8]
    // dir may be null (end key only).  A block run writes the codes of the
    // block alone: dir[(col - dir_col0) * dir_stride + row / 8 - dir_rb0].
    uint32_t* dir;
    int64_t dir_stride;          // words per column: nb * K (a block: its bands * K)
    int64_t m, n;                // real lengths (cells past them are padding)
    unsigned long long* end_key; // min over cells with H = *score of col << 32 | row
    int64_t dir_col0;
    int32_t dir_rb0;
    // Checkpointed alignment.  The checkpointing score pass stores, below
    // every ckpt_gb-th band, its bottom row (H - Go, F) per column:
    // ckpt_row[k * ckpt_row_stride + col], k = (b + 1) / ckpt_gb - 1; right of
    // every ckpt_gc-th chunk, its last column (H - Go, E) per row:
    // ckpt_col[k * ckpt_col_stride + row], k = (c + 1) / ckpt_gc - 1; and the
    // largest H of every chunk (chunk_max[c], atomicMax).  A block run (the
    // direction pass over bands from b_org, chunks from a checkpoint column)
    // starts from buffers filled from those checkpoints; the corners of its
    // first band come from top_ckpt (the checkpoint row above b_org, by
    // absolute column), null when b_org = 0.
    int2* ckpt_row;
    int2* ckpt_col;
    int64_t ckpt_row_stride, ckpt_col_stride;
    int32_t ckpt_gb, ckpt_gc;
    int32_t* chunk_max;
    int32_t b_org;
    const int2* top_ckpt;
    // Skewed score pass: lane g of band b covers, in chunk c, columns
    // [c*wc - b*kr - g, +wc) (kr: K rounded up to 16); carry[row block] holds
    // (H - Go, F) of the lane's bottom row at its last column and the H - Go
    // above that column, for the lane's next tile.  n_pad: bytes of subj.
    int32_t kr;
    int4* carry;                 // [nb * K]
    int64_t n_pad;
    // 64 bytes per wavefront of a launch: where lanes of no tile store their
    // direction words (skewed trace pass)
    uint8_t* sink;
};

// Pipelined pass over one long pair (sw_pair_flow.hip): one-wave workgroups
// take bands of 64 lanes x R rows (bands w, w + waves, ...), stage the band's
// profile in LDS and sweep all columns; a band hands its bottom row to the band
// below through tagged 64-bit words.
struct FlowArgs {
    const uint8_t* subj;         // subject codes padded with the pad code (n_pad bytes, multiple of 16)
    const uint8_t* prof;         // query profile, R-row blocks (nbr + 1 of them)
    unsigned long long* rows;    // [n + 16] handoff words (cleared by the launch)
    int32_t* score;              // [1] running maximum (atomicMax); -1 if a wait timed out
    int32_t* status;             // [1] nonzero once a wait timed out
    int32_t n, n_pad;            // subject length, bytes of subj
    int32_t nbr, nb;             // query row blocks, bands (64 row blocks each)
    int32_t waves;               // wavefronts of the launch
    int32_t go, ge;
    uint64_t timeout;            // s_memrealtime ticks a wait may last
    // direction-code pass (null dir: the score pass)
    uint32_t* dir;               // [column * dir_stride + row block] 4-bit codes of 8 rows
    unsigned long long* end_key; // first cell holding the score, (column << 32) | row (atomic minimum)
    int64_t dir_stride;          // row blocks per column
    int64_t m;                   // query length (rows past it hold no end cell)
};
// Bytes per (code, lane) entry group of a band's profile staged in LDS by the
// flow pass: the lane's R entries rounded up to a power of two (aligned reads).
__host__ __device__ constexpr int flow_lds_stride(int R, int ES)
{
    return R * ES <= 4 ? 4 : (R * ES <= 8 ? 8 : (R * ES <= 16 ? 16 : 32));
}
// Rows per lane the flow pass is built for (the planner keeps the band count
// at or below the device's SIMDs where it can).
constexpr int kFlowRowChoices[6] = {4, 6, 8, 10, 12, 16};
// From this many rows per lane the flow pass checks the handoff words' tags
// once per 16-step block; below, once per step.
constexpr int kFlowBlockwiseRows = 8;
// The flow pass on `grid` workgroups of `wpg` waves (a.waves = grid * wpg),
// each asking for `lds` bytes of LDS (at least wpg band profiles).
hipError_t launch_pair_flow(const FlowArgs& a, int rows, int elem, int wpg, int grid, int lds, hipStream_t st);
// resident workgroups per CU (0 on error); trace: the direction-code pass
int flow_occupancy(int rows, int elem, int wpg, int lds, bool trace = false);
__host__ __device__ constexpr int flow_lds_bytes(int rows, int elem)   // LDS of one wave's band profile
{
    return kCodes * kWave * flow_lds_stride(rows, elem);
}
// LDS a workgroup of wpg waves needs: one band profile per wave.
__host__ __device__ constexpr int flow_group_lds(int rows, int elem, int wpg)
{
    return wpg * flow_lds_bytes(rows, elem);
}

// Alignment found by the traceback pass (device memory, written by the
// traceback kernel): 1-based inclusive positions, operation count.
struct AlignOut {
    int32_t score, q_begin, s_begin, q_end, s_end, n_ops;
};

// State of the traceback walk between blocks (device memory): the current
// 1-based cell and state (0: H, 1: in a gap of the query (E), 2: in a gap of
// the subject (F)), whether the last step was a diagonal one, operations so
// far, and, once done, the begin cell and whether the codes were consistent.
struct WalkState {
    int64_t i, j, n_ops, bi, bj;
    int32_t st, prev_m, done, ok;
    int32_t q_end, s_end;
};

// Kernel variants the runtime may launch.
enum Variant : int {
    kI32_R32_P8 = 0,   // int32 lanes, 32 rows, 8-bit profile
    kI32_R32_P16 = 1,  // int32 lanes, 32 rows, 16-bit profile
    kI16 = 2,          // packed 16-bit lanes, kI16Rows rows, 16-bit profile
    kI16_P8 = 3,       // packed 16-bit lanes, kI16Rows rows, 8-bit profile with
                       // every entry s + Go in [0, 127] (zero-extended)
};

struct LaunchInfo {
    int rows;            // R
    int prof_elem;       // bytes per profile entry
    int subjects_per_lane;
};
LaunchInfo variant_info(Variant v);

// Host-side launchers (defined with the kernels).
hipError_t launch_profile(const ProfileArgs& a, int rows, int elem, int max_entries, hipStream_t st);
hipError_t launch_search(Variant v, const SearchArgs& a, int grid, int waves, int lds_bytes, hipStream_t st);
hipError_t launch_flag_sort(const SearchArgs& a, hipStream_t st);
hipError_t launch_rescore(Variant v, const SearchArgs& a, int grid, int waves, hipStream_t st);
hipError_t launch_interleave(const uint8_t* src, const int64_t* src_off, const int32_t* perm,
                             const int32_t* slen, const int64_t* chunk_off, int32_t nseq,
                             int64_t nthreads_total, const int64_t* block_prefix, int32_t nchunks,
                             uint8_t* dst, int32_t* bad, hipStream_t st);
int search_occupancy(Variant v, int waves, int lds_bytes);   // workgroups per CU
// Single long pair: the padded subject (codes modulo 32), the cleared score and
// the query's profile descriptor; then one launch per anti-diagonal.
// Query rows per lane of the pair kernel (int32 lanes): fewer rows give more
// lanes on each anti-diagonal (short pairs), more rows fewer instructions per
// cell (long pairs).
constexpr int kPairRowChoices[2] = {8, 16};
hipError_t launch_pair_prep(const uint8_t* subj, int64_t n, int64_t n_pad, uint8_t* dst, int32_t* score,
                            const QueryDesc& qd, QueryDesc* qd_out, int64_t* qoff_out, hipStream_t st);
// The plain score pass over skewed tiles (one anti-diagonal of them), and the
// direction-code pass of an alignment with whole-matrix codes (8 rows per lane).
hipError_t launch_pair_skew(const PairArgs& a, int rows, int elem, hipStream_t st);
hipError_t launch_trace_skew(const PairArgs& a, int elem, hipStream_t st);
// Traceback: the direction pass over one anti-diagonal (8 rows per lane, K =
// 64), the end-key reset, and the single-lane walk that writes the alignment.
hipError_t launch_trace_diag(const PairArgs& a, int elem, hipStream_t st);
hipError_t launch_trace_reset(unsigned long long* end_key, hipStream_t st);
// Checkpointing score pass (8 rows per lane, K = 64) and the fill of the
// boundary buffers of a block run from the checkpoints.
hipError_t launch_pair_diag_ckpt(const PairArgs& a, int elem, hipStream_t st);
hipError_t launch_block_init(const PairArgs& a, int64_t kb, int64_t kc, int64_t b_hi, int64_t c_org,
                             int64_t c_hi, hipStream_t st);
// Walk: start from the end key, continue inside a block of codes (rows
// [r_lo, r_hi), columns [c_lo, c_hi), 0-based) until it leaves the block or
// ends, finish (reverse the operations, write the result).
hipError_t launch_walk_init(const unsigned long long* end_key, const int32_t* score, WalkState* w,
                            hipStream_t st);
hipError_t launch_walk(const uint32_t* dir, int64_t dir_stride, int64_t r_lo, int64_t c_lo, int64_t r_hi,
                       int64_t c_hi, WalkState* w, char* ops, int64_t cap, hipStream_t st);
hipError_t launch_walk_finish(const WalkState* w, const int32_t* score, char* ops, AlignOut* out,
                              hipStream_t st);

}  // namespace swdb
