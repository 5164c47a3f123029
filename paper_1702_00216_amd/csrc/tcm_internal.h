// Internal declarations shared by the HIP kernels and the host runtime of
// libtcm.so.  Nothing here is part of the public C-ABI (include/tcm.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace tcmk {

// A block ("cell" of the paper) is 8^3 nodes.  Its pool slot holds three
// planes of 512 floats, x fastest inside a plane: phi level 0, phi level 1
// and C2 = (c dt / dx)^2.  Level (n & 1) holds phi^n; the other holds
// phi^{n-1} and is overwritten by phi^{n+1} (two-array overwrite).  The pool
// stores each kind of plane in an array of its own (all slots' level-0
// planes, then all level-1 planes, then all C2 planes), so that blocks in
// consecutive slots stream as one contiguous run per array: measured on the
// stencil's access pattern (one wave per slot, consecutive slots per
// workgroup), 5.88 TB/s against 5.52 TB/s with a slot's three planes side
// by side.
constexpr int BE = 8;
constexpr int BV = BE * BE * BE;
constexpr int SLOT = 3 * BV;                 // floats of pool per slot
constexpr int PLANE_C2 = 2;                  // plane kinds: 0, 1 (phi levels), 2 (C2)
constexpr int EMPTY = -1;
constexpr int CLAIMED = -2;
constexpr int ERR_POOL = -3;       // sticky device errors (TCM_E_POOL, TCM_E_NONFINITE)
constexpr int ERR_NONFINITE = -8;
constexpr int KEEP_BIT = 64;
constexpr int HOT_BIT = 128;       // any |phi| of either level above the trigger

// Blocks are numbered per shot in 4x4x4 tiles: key = tile * 64 + local with
// local = (lz * 4 + ly) * 4 + lx, tiles in x-fastest order.  One 64-bit word
// of the activity bitmap covers one tile.  A shot owns the global key range
// [key_base, key_base + 64 * ntiles); key_base is a multiple of 64.
struct Shot {
    int nx, ny, nz;
    int bx, by, bz;          // blocks per axis
    int tx, ty, tz;          // tiles per axis
    int media_kind;
    long long key_base;
    long long word_base;     // key_base / 64
    long long nwords;        // tx * ty * tz
    const float* c;          // DENSE media (device, nx*ny*nz)
    const int* z_top;        // LAYERED media (device)
    const float* c_layer;
    int nlayers;
    int lx, ly, lz, log2s;   // LATTICE media
    const double* lattice;
};

// Device-side counters.  step/n_act/free_cnt describe the state between
// steps; n_new/n_ret are per-step scratch; emit tells the list writer
// whether the step committed.
struct DevState {
    int step, n_act, n_new, n_ret;
    int free_cnt, error, err_step, emit;
    int peak_act, add_error, n_dec;
    unsigned long long scan_acc;     // k_pool_count: scanning workgroups arrived (high 32 bits) and
                                     // their range totals (low 32 bits); 0 between steps
    unsigned long long cells_cur;    // in-domain nodes of the current active list
    unsigned long long updates;      // in-domain nodes stepped so far
    unsigned long long cells_cur_u;  // ... of those, nodes of blocks with a uniform C2
    unsigned long long updates_u;
    unsigned long long cells_cur_l;  // ... of those, nodes of blocks with a lattice record (STEP_LAT)
    unsigned long long updates_l;
    unsigned long long decays;       // block-steps of the shutdown decay
    unsigned maxbits;                // adaptive levels: max |phi^{n+1}| of this step (float bits)
    float trig_cur, ret_cur;         // levels used by the last plan
    int n_ne;                        // per step: chunks of the bitmap with a set bit
    unsigned long long activations, retirements;
    int free_next;                   // free slots after this step's allocation: installed, and the
                                     // step's n_new / n_ret / n_dec cleared, by the compaction
    int fast_par;                    // two-launch update: parity of the next active set (k_fast_plan)
    int n_gblocks;                   // adjoint: gradient blocks handed out (first gradient term of a key)
    int grad_error;                  // adjoint: a gradient block or lap-store entry was out of range
    int nf_step;                     // n + 1 for the first step n that wrote a non-finite value, else 0
    int adv_tk[8], adv_top;          // stencil advancing the step itself: workgroups done per class
                                     // (blockIdx % 8), then classes done (0 between launches)
};

struct Src {
    long long key;     // global block key
    int local;         // node inside the block, (z * 8 + y) * 8 + x
    int t0, ns;        // first step and sample count
    int pad;
    long long w_off;   // offset of the samples in the sample array
};

struct Rec {
    long long key;
    int local, pad;
};

struct Tables {
    DevState* st;
    const Shot* shots;
    int nshots;
    const int* word_shot;           // per bitmap word: its shot (nullptr with one shot)
    int cap;                        // pool slots
    long long nkeys;                // global block keys (all shots)
    float* pool;
    int* cell2box;                  // per global key: slot, EMPTY or CLAIMED
    unsigned long long* bitmap;     // next active set, one bit per global key (two-launch update:
                                    // the active set of even steps)
    unsigned long long* bitmap2;    // two-launch update: the active set of odd steps
    int fast;                       // 1: the two-launch activation update (launch_fast_update)
    int nfchunks;                   // two-launch update: groups of FAST_WORDS bitmap words
    int* fc_cnt;                    // per group: blocks of the next set
    // up to FAST_DIRECT_CHUNKS groups, per group:
    int* fc_new;                    //   activations,
    int* fc_ret;                    //   releases,
    unsigned long long* fc_cells;   //   in-domain nodes of the next set (all, scalar-C2 blocks,
                                    //   lattice-record blocks);
    // beyond, per run of FAST_BLK groups:
    int nfblk;                      // runs (0: up to FAST_DIRECT_CHUNKS groups)
    unsigned long long* fc_blk;     // [2][nfblk][3] per run, summed by the plan of an even / odd
                                    // step: {blocks of the next set, activations, releases} (21 bits
                                    // each), {its in-domain nodes, of scalar-C2 blocks} (32 bits
                                    // each), its nodes of lattice-record blocks
    long long nwords;
    int* act_slot;                  // active list (length n_act)
    int* act_shot;
    unsigned* act_key;              // key inside the shot
    int* rows;                      // per list entry: slot, 6 neighbour slots (or EMPTY), global key
    unsigned char* flags;           // per slot: face bits 0..5 and KEEP_BIT
    int* pin_until;                 // per slot two ints: [2 slot] active while step < it (sources);
                                    // [2 slot + 1] the block's sources in the (key-ordered) source
                                    // table, count << 24 | first, or -1
    float* slot_c2u;                // per slot: the block's C2 if uniform over the block, else NaN
                                    // (LAT_C2_BITS when the slot holds a lattice record)
    double* slot_lat;               // per slot, lattice media with spacing >= 8 (the block inside one
                                    // lattice cell, all of it in the domain): the cell's 8 corner
                                    // speeds, [h * 4 + dy * 2 + dx] at (iz + h, iy + dy, ix + dx)
    int4* slot_latm;                //   and {x, y, z offset of the block in the cell, log2 spacing}
    int lat_c2;                     // 1: the stencil computes those blocks' C2 (STEP_LAT variants)
    int self_advance;               // this stencil launch ends a step without an activation update
                                    // and without receivers: its last workgroup advances the step
                                    // (instead of a k_advance launch; constant levels only)
    int dx_pow2;                    // dx is a power of two: (c dt) / dx == (c dt) * (1 / dx)
    double rdx;                     // 1 / dx
    unsigned char* sdlog;           // per slot: shutdown steps left (0: not shutting down)
    int* dec_slot;                  // per step: slots whose levels are multiplied by alpha
    int shutdown_steps;             // eq.(6) n (0: release at once)
    float shutdown_alpha;           // eq.(6) alpha
    int interval;                   // activation update after every interval-th step (1..8)
    int adaptive;                   // levels relative to the domain maximum (Table 1 Trig_level)
    float trigger_rel, retire_rel;
    float* bmax;                    // adaptive: per slot 6 face maxima, max |phi^{n+1}|, max |phi^n|
    int uniform_c2;                 // 1: blocks with a uniform C2 read it as a scalar
    int c2_ready;                   // 1: a slot is always its key's (a pool of one slot per key), and
                                    // every slot's C2 plane and slot_c2u were filled at creation
    long long* slot_key;            // per slot: global key, or -1 when the slot is free
    long long* new_key;             // per step: claimed keys
    int* new_shot;
    int* ret_slot;                  // per step: released slots ...
    long long* ret_key;             //   ... and the global keys they held
    unsigned* partial;              // per 16-word chunk: set bits, then offset inside its range
    int nchunks;                    // ceil(nwords / 16); the bitmap is padded to whole chunks
    unsigned* wg_total;             // per k_pool_count workgroup: set bits of its chunk range
                                    // (k_emit scans them into the ranges' offsets)
    int chunks_per_wg;              // chunks per scanning k_pool_count workgroup (contiguous)
    int scan_wgs;                   // the first scan_wgs workgroups of k_pool_count scan
    int* ne_chunks;                 // per step: the chunks with a set bit (any order)
    const Src* src;
    int nsrc;
    const float* srcw;
    const Rec* rec;
    int nrec;
    float* traces;                  // [trace_cap][nrec]
    int trace_step0, trace_cap;
    double dt, dx;
    float trigger, retire;
    // Recomputation of a forward segment for the adjoint (null otherwise):
    // the block stencil also stores L u^n of list entry i at rec_lap + i * 512
    // (entries below rec_lapcap) and i at rec_fidx[global key].
    float* rec_lap;
    int* rec_fidx;
    int rec_lapcap;
    // Adjoint field with the gradient (null otherwise): the stencil of the
    // adjoint field that forms mu^m also adds mu^m (L u^{m-1}) to the FP32
    // gradient block of each entry's key, where g_lap / g_fidx are the store
    // of forward step m - 1.  Gradient blocks (512 FP32 partials in g_gs, 512
    // FP64 sums in g_acc) are handed out on a key's first term:
    // g_slot[global key] (-1: none yet), at most g_cap.
    const float* g_lap;
    const int* g_fidx;
    float* g_gs;
    double* g_acc;
    int* g_slot;
    int g_cap;
    unsigned long long* g_terms_wg;   // per stencil workgroup: nodes whose gradient term it formed
};

// The compaction works on chunks of 16 bitmap words (1024 blocks), one
// workgroup per chunk.
constexpr int CHUNK_WORDS = 16;
// Upper bound on the scanning workgroups of k_pool_count; each takes
// chunks_per_wg consecutive chunks (scan_wgs * chunks_per_wg >= nchunks).
constexpr int POOL_COUNT_MAX_WG = 1024;

// ---- launch wrappers (tcm_kernels.hip) -----------------------------------
hipError_t launch_init_tables(const Tables& t, long long nkeys, hipStream_t s);
// w: blocks per workgroup (2, 4 or 8; 64 * w threads).  e0 / e1 (optional):
// events stamped by the dispatch itself at the kernel's start and end.
hipError_t launch_block_step(const Tables& t, int grid, int w, int pb, hipStream_t s,
                             hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr);
// Variants of the block stencil: a plain step, a recomputed forward step of
// the adjoint (also stores L u per entry, Tables::rec_lap), or a step of the
// adjoint field (also adds the gradient term, Tables::g_lap).
// launch_block_step picks the variant from the Tables.
constexpr int STEP_PLAIN = 0, STEP_RECORD = 1, STEP_GRAD = 2;
// Flag on top of those (constant levels only): blocks whose slot holds a
// lattice record (Tables::slot_lat) take their C2 from it, computed as the
// media evaluation does, instead of reading the slot's C2 plane.
constexpr int STEP_LAT = 4;
// slot_c2u of such a block: a quiet NaN (non-uniform C2) with this payload
constexpr unsigned LAT_C2_BITS = 0x7fc0004cu;
// resident workgroups per CU of a variant (w waves per workgroup, pb blocks per wave;
// mode: STEP_PLAIN / STEP_RECORD / STEP_GRAD, with STEP_LAT for the lattice-record variants)
int block_step_occupancy(bool adaptive, int w, int pb, int mode = STEP_PLAIN);
bool block_step_shape_ok(int w, int pb);
hipError_t launch_plan(const Tables& t, int grid, hipStream_t s);
hipError_t launch_advance(const Tables& t, hipStream_t s);   // step without an activation update
hipError_t launch_pool_count(const Tables& t, int grid, hipStream_t s);   // grid >= scan_wgs
hipError_t launch_emit(const Tables& t, int grid, hipStream_t s);
// The activation update in two launches for constant levels, an update every
// step, no shutdown and one slot per key (Tables::fast): k_fast_plan then
// k_fast_emit (tcm_kernels.hip).  FAST_WORDS bitmap words per workgroup.
// Up to FAST_DIRECT_CHUNKS groups each compaction workgroup sums the counts
// of the groups before its own; beyond, the plan also sums the counts of
// each run of FAST_BLK groups (device atomics), so that a compaction
// workgroup finds its offset from at most FAST_MAX_CHUNKS / FAST_BLK run
// sums and FAST_BLK - 1 group counts.
constexpr int FAST_WORDS = 4;
constexpr int FAST_DIRECT_CHUNKS = 4096;
constexpr int FAST_BLK = 16;
constexpr int FAST_MAX_CHUNKS = FAST_BLK * 4096;
hipError_t launch_fast_update(const Tables& t, int grid, hipStream_t s);
// Activate n blocks (distinct global keys; shot and key inside the shot per
// entry), pin each while step < pins[i] and, where heads[i] >= 0, give it
// that source range; one wave per block.  Blocks that are active already
// only raise their pin (and take the range).  pins[i] == -1: only refresh the
// range of an active block; -2: clear pin and range of an active block.  No
// free slot: add_error = -3.
hipError_t launch_activate_list(const Tables& t, const long long* keys, const int* shots,
                                const unsigned* local_keys, const int* pins, const int* heads, int n,
                                hipStream_t s);
hipError_t launch_refresh_rows(const Tables& t, hipStream_t s);
// C2 plane and slot_c2u of every slot from its key's block (c2_ready pools)
hipError_t launch_prefill_c2(const Tables& t, long long nkeys, hipStream_t s);
// table invariants between steps: mark = cap zeroed ints, bad = two zeroed
// counters (violations, keys with a slot)
hipError_t launch_check(const Tables& t, int* mark, unsigned long long* bad, hipStream_t s);
hipError_t launch_read(const Tables& t, int shot, int which, int x0, int y0, int z0, int sx,
                       int sy, int sz, float* out, hipStream_t s);
hipError_t launch_media_c2(const Shot& shot, const Shot* dshot, double dt, double dx, float* c2,
                           hipStream_t s);

// dense engine (every node every step; the same arithmetic)
struct DenseArgs {
    int nx, ny, nz;
    const float* cur;
    float* nxt;                      // holds phi^{n-1} on entry, phi^{n+1} on exit
    const float* c2;
};
hipError_t launch_dense_step(const DenseArgs& a, hipStream_t s, hipEvent_t e0 = nullptr,
                             hipEvent_t e1 = nullptr);
hipError_t launch_dense_inject(float* nxt, int n, const Src* src, int nsrc, const float* srcw,
                               const Rec* rec, int nrec, float* traces, int trace_row,
                               hipStream_t s);
hipError_t launch_read_dense(const float* f, int nx, int ny, int x0, int y0, int z0, int sx, int sy,
                             int sz, float* out, hipStream_t s);

// adjoint support
hipError_t launch_receiver_c2(const Shot* shots, const int* xyz, const int* rshot, int nrec,
                              double dt, double dx, float* out, hipStream_t s);
// adjoint steps whose FP32 partial gradient is summed before it is folded
// into the FP64 gradient (groups of absolute step numbers, so the result does
// not depend on the checkpoint interval)
constexpr int GRAD_GROUP = 32;
// the adjoint field's stencil, which also forms the gradient terms, runs on
// at most GRAD_ACCUM_MAX_WG workgroups (one node-count slot each)
constexpr int GRAD_ACCUM_MAX_WG = 4096;
// g_acc += g_gs, g_gs = 0 over the gradient blocks handed out so far
hipError_t launch_grad_flush(const Tables& mu, hipStream_t s);
// out[node] = (2 / c) * gradient sum of shot 0 (0 where c = 0 or no term)
hipError_t launch_grad_finish(const Tables& mu, const Shot& shot, const Shot* dshot, float* out,
                              hipStream_t s);
// fill n ints with v
hipError_t launch_fill_int(int* p, long long n, int v, hipStream_t s);
// Sparse state copy of a block-engine handle: the active list (n entries)
// with its slots' three planes and per-slot tables, to / from buf (layout in
// tcm_kernels.hip, ck_layout); restore expects freshly initialised tables.
size_t ck_sparse_bytes(long long n);
hipError_t launch_ck_gather(const Tables& t, long long n, char* buf, hipStream_t s);
hipError_t launch_ck_scatter(const Tables& t, long long n, const char* buf, hipStream_t s);
// HBM ceiling probe (n floats per source, n a multiple of hbm_probe_chunk())
long long hbm_probe_chunk();
hipError_t launch_hbm_probe(const float* src, float* dst, long long n, int nread, int grid, hipStream_t s,
                            hipEvent_t e0, hipEvent_t e1);

// staging of tcm_read_noalloc (tcm_noalloc.hip): a static device array of
// NOALLOC_FLOATS floats per GPU; its device address for the current device
constexpr long long NOALLOC_FLOATS = 8LL << 20;
hipError_t noalloc_staging(float** out);

}  // namespace tcmk
