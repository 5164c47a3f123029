// HIP kernels of the Triggered Cells Method hot path for gfx950 (MI355X).
//
// One step n (phi^n -> phi^{n+1}) is four launches, all sized from device
// counters so that a sequence of steps can be replayed as a hipGraph:
//
//   k_block_step  eq.(3) on every active 8^3 block: a 64-lane wave per block
//                 (or per two consecutive blocks), lane = (x, y) column with
//                 the 8 z values in registers, the neighbour face planes
//                 staged in LDS (x faces shared between the blocks of a
//                 workgroup, which takes x-adjacent blocks); a wave raises
//                 its issue priority while it issues a block's loads;
//                 additive source insertion; wave-ballot face/keep
//                 predicates -> one flag byte per slot.
//   k_plan        keep / release each active block, claim empty face neighbours
//                 with a compare-and-swap on the block table, mark the next
//                 active set in a bitmap; receivers are recorded here.
//   k_pool_count  lock-free slot allocator: a new block claims the first free
//                 slot at or after its preferred slot (the key itself with one
//                 slot per key, else a hashed 64-slot group of its tile) with a
//                 compare-and-swap, so the pool keeps the spatial order of the
//                 active list; zero-fill + C2 of new blocks; a two-level scan
//                 of the bitmap (chunk ranges per scanning workgroup, then the
//                 range totals in the last one), which also lists the
//                 non-empty chunks and commits the step counters.
//   k_emit        compaction of the bitmap into the next active list and its
//                 neighbour rows (spatial tile order), clearing the bitmap for
//                 the next step; it also installs the allocator's free count
//                 and clears the step's claim / release / decay counters,
//                 which every allocating workgroup reads at its start.
//
// A step without an activation update (update interval > 1) is k_block_step
// and k_advance (receivers, step counter).
//
// Arithmetic of the node update (eq.(3)), fixed for bit-exact comparisons:
//   s = ((x+ + x-) + (y+ + y-)) + (z+ + z-);  lap = s - 6 phi;
//   next = (2 phi - prev) + C2 lap;  compiled with -ffp-contract=off.
#include "tcm_internal.h"

#include <hip/hip_ext.h>

namespace tcmk {

// plane k (0, 1: phi levels; 2: C2) of a slot
__device__ __forceinline__ float* plane_of(const Tables& t, long long slot, int k) {
    return t.pool + ((size_t)k * (size_t)t.cap + (size_t)slot) * BV;
}

// --------------------------------------------------------------------------
// small helpers
// --------------------------------------------------------------------------
// First error of the run and the step it happened in (sticky; the step's
// phi^{n+1} is kept).
__device__ __forceinline__ void report_error(DevState* st, int code, int step) {
    if (atomicCAS(&st->error, 0, code) == 0) st->err_step = step;
}
// A non-finite value written by the stencil of step n sets nf_step = n + 1
// (only the stencil writes it, so every other workgroup of that launch still
// runs).  The step completes with its old active set, like a pool failure;
// later steps do nothing.
__device__ __forceinline__ bool halted_before(const DevState* st, int n) {
    return st->error || (st->nf_step && st->nf_step != n + 1);
}
__device__ __forceinline__ int lane_id() { return __lane_id(); }

// A list row's last field is the global key, with bit 31 set when the slot
// has sources in the source table or a pin (keys are below 2^31): the
// stencil loads a block's pin and source range only then, instead of for
// every block, and folds a pin that still holds into the block's keep flag.
constexpr int ROW_SRC_BIT = (int)0x80000000u;
__device__ __forceinline__ bool slot_has_pin_or_src(const Tables& t, long long slot) {
    const unsigned long long ph = ((const unsigned long long*)t.pin_until)[slot];   // {pin, first source}
    return (int)(unsigned)ph > 0 || (int)(unsigned)(ph >> 32) >= 0;
}
__device__ __forceinline__ int row_key_field(const Tables& t, long long slot, long long G) {
    return (int)G | (slot_has_pin_or_src(t, slot) ? ROW_SRC_BIT : 0);
}
__device__ __forceinline__ int row_key(int v) { return v & 0x7fffffff; }

// Read-only (for the reading kernel) tables addressed uniformly by a wave are
// read through the scalar data cache: constant address space loads.
template <class T>
using scalar_ptr = const __attribute__((address_space(4))) T*;
template <class T>
__device__ __forceinline__ scalar_ptr<T> as_scalar(const T* p) {
    return (scalar_ptr<T>)(p);
}

__device__ __forceinline__ void key_to_block(const Shot& S, unsigned key, int& bx, int& by,
                                             int& bz) {
    const unsigned tile = key >> 6, l = key & 63u;
    const unsigned tx = tile % (unsigned)S.tx;
    const unsigned r = tile / (unsigned)S.tx;
    const unsigned ty = r % (unsigned)S.ty;
    const unsigned tz = r / (unsigned)S.ty;
    bx = (int)(tx * 4 + (l & 3u));
    by = (int)(ty * 4 + ((l >> 2) & 3u));
    bz = (int)(tz * 4 + (l >> 4));
}

__device__ __forceinline__ unsigned block_to_key(const Shot& S, int bx, int by, int bz) {
    const unsigned tile = ((unsigned)(bz >> 2) * (unsigned)S.ty + (unsigned)(by >> 2)) *
                              (unsigned)S.tx + (unsigned)(bx >> 2);
    return tile * 64u + ((unsigned)(bz & 3) << 4) + ((unsigned)(by & 3) << 2) + (unsigned)(bx & 3);
}

// global key of the block across face d (0:-x 1:+x 2:-y 3:+y 4:-z 5:+z), or -1
__device__ __forceinline__ long long neighbour_key(const Shot& S, int bx, int by, int bz, int d) {
    int x = bx, y = by, z = bz;
    switch (d) {
        case 0: x--; break;
        case 1: x++; break;
        case 2: y--; break;
        case 3: y++; break;
        case 4: z--; break;
        default: z++; break;
    }
    if (x < 0 || y < 0 || z < 0 || x >= S.bx || y >= S.by || z >= S.bz) return -1;
    return S.key_base + (long long)block_to_key(S, x, y, z);
}

__device__ __forceinline__ int block_cells(const Shot& S, int bx, int by, int bz) {
    const int ex = min(BE, S.nx - bx * BE), ey = min(BE, S.ny - by * BE), ez = min(BE, S.nz - bz * BE);
    return ex * ey * ez;
}

// Append for every lane with pred; returns the lane's index or -1.
// Must be reached by all lanes of the wave.
__device__ __forceinline__ int wave_append(int* counter, bool pred) {
    const unsigned long long m = __ballot(pred);
    if (m == 0ull) return -1;
    const int lane = lane_id();
    const int leader = __ffsll((long long)m) - 1;
    int base = 0;
    if (lane == leader) base = atomicAdd(counter, __popcll(m));
    base = __shfl(base, leader);
    const int rank = __popcll(m & ((1ull << lane) - 1ull));
    return pred ? base + rank : -1;
}

// wave speed at global node (gx, gy, gz) of shot S ("Media": array or rules)
__device__ float media_speed(const Shot& S, int gx, int gy, int gz) {
    if (S.media_kind == 0) {
        return S.c[(size_t)gx + (size_t)S.nx * ((size_t)gy + (size_t)S.ny * (size_t)gz)];
    }
    if (S.media_kind == 1) {
        float v = S.c_layer[0];
        for (int k = 1; k < S.nlayers; k++)
            if (gz >= S.z_top[k]) v = S.c_layer[k];
        return v;
    }
    // LATTICE: trilinear interpolation in FP64, x then y then z, one rounding
    const int s = S.log2s;
    const int ix = gx >> s, iy = gy >> s, iz = gz >> s;
    const double inv = 1.0 / (double)(1 << s);
    const double fx = (double)(gx - (ix << s)) * inv;
    const double fy = (double)(gy - (iy << s)) * inv;
    const double fz = (double)(gz - (iz << s)) * inv;
    const double gx0 = 1.0 - fx, gy0 = 1.0 - fy, gz0 = 1.0 - fz;
    const size_t LX = (size_t)S.lx, LXY = (size_t)S.lx * (size_t)S.ly;
    double cy[2];
    for (int h = 0; h < 2; h++) {
        const double* L = S.lattice + (size_t)(iz + h) * LXY + (size_t)iy * LX + (size_t)ix;
        const double cx0 = L[0] * gx0 + L[1] * fx;
        const double cx1 = L[LX] * gx0 + L[LX + 1] * fx;
        cy[h] = cx0 * gy0 + cx1 * fy;
    }
    return (float)(cy[0] * gz0 + cy[1] * fz);
}

__device__ __forceinline__ float coeff_c2(float c, double dt, double dx) {
    const double t = (double)c * dt / dx;
    return (float)(t * t);
}

// Fill the C2 plane of a slot from the media (one wave, lane = (x, y)
// column).  Returns (to every lane) the block's C2 if all 512 nodes are in
// the domain and share it ("homogenic" cell of Table 1), else NaN.
__device__ float fill_c2(const Tables& t, const Shot& S, long long slot, int bx, int by, int bz) {
    float* __restrict__ pc = plane_of(t, slot, PLANE_C2);
    const int lane = lane_id();
    const int x = lane & 7, y = lane >> 3;
    float first = 0.f;
    bool same = true;
#pragma unroll
    for (int z = 0; z < 8; z++) {
        const int gx = bx * BE + x, gy = by * BE + y, gz = bz * BE + z;
        float c2 = 0.f;   // nodes outside the domain keep C2 = 0 and stay zero
        const bool in = gx < S.nx && gy < S.ny && gz < S.nz;
        if (in) c2 = coeff_c2(media_speed(S, gx, gy, gz), t.dt, t.dx);
        pc[z * 64 + lane] = c2;
        if (z == 0) first = c2;
        same = same && in && c2 == first;
    }
    const float ref = __shfl(first, 0);
    same = same && first == ref;
    const bool uniform = t.uniform_c2 && __ballot(!same) == 0ull;
    if (uniform) return ref;
    // lattice media with spacing >= 8: the block lies inside one lattice cell,
    // whose 8 corners (and the block's offset in it) give every node's C2 as
    // above; the stencil's STEP_LAT variants compute it from this record
    // instead of reading the plane (blocks that reach outside the domain,
    // whose outer nodes have C2 = 0, keep the plane)
    const bool whole = (bx + 1) * BE <= S.nx && (by + 1) * BE <= S.ny && (bz + 1) * BE <= S.nz;
    if (t.slot_lat && S.media_kind == 2 && S.log2s >= 3 && whole) {
        const int sh = S.log2s;
        const int ix = (bx * BE) >> sh, iy = (by * BE) >> sh, iz = (bz * BE) >> sh;
        const size_t LX = (size_t)S.lx, LXY = (size_t)S.lx * (size_t)S.ly;
        if (lane < 8) {
            const int h = lane >> 2, dy = (lane >> 1) & 1, dx = lane & 1;
            t.slot_lat[8 * (size_t)slot + lane] =
                S.lattice[(size_t)(iz + h) * LXY + (size_t)(iy + dy) * LX + (size_t)(ix + dx)];
        }
        if (lane == 0) t.slot_latm[slot] = make_int4(bx * BE - (ix << sh), by * BE - (iy << sh), bz * BE - (iz << sh), sh);
        return __uint_as_float(LAT_C2_BITS);
    }
    return __builtin_nanf("");
}

// 64-bit value of lane l (l uniform)
__device__ __forceinline__ double readlane_f64(double v, int l) {
    const unsigned long long b = (unsigned long long)__double_as_longlong(v);
    const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)b, l);
    const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(b >> 32), l);
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// C2 of the 8 nodes of lane (x, y) of a block with a lattice record (its
// corners in lanes 0-7 of lv, its offsets m): the trilinear interpolation of
// media_speed and the coefficient of coeff_c2, operation for operation, so
// the values equal the C2 plane bit for bit
__device__ __forceinline__ void lattice_c2(const Tables& t, double lv, int4 m, int x, int y, float* k2) {
    double L[8];
#pragma unroll
    for (int k = 0; k < 8; k++) L[k] = readlane_f64(lv, k);
    const int sh = __builtin_amdgcn_readfirstlane(m.w);
    const int ox = __builtin_amdgcn_readfirstlane(m.x), oy = __builtin_amdgcn_readfirstlane(m.y),
              oz = __builtin_amdgcn_readfirstlane(m.z);
    // 1 / 2^sh, exactly (as the division it stands for)
    const double inv = __longlong_as_double((long long)(1023 - sh) << 52);
    const double fx = (double)(ox + x) * inv;
    const double fy = (double)(oy + y) * inv;
    const double gx0 = 1.0 - fx, gy0 = 1.0 - fy;
    double cy[2];
#pragma unroll
    for (int h = 0; h < 2; h++) {
        const double cx0 = L[h * 4 + 0] * gx0 + L[h * 4 + 1] * fx;
        const double cx1 = L[h * 4 + 2] * gx0 + L[h * 4 + 3] * fx;
        cy[h] = cx0 * gy0 + cx1 * fy;
    }
    double cd[8];
#pragma unroll
    for (int z = 0; z < 8; z++) {
        const double fz = (double)(oz + z) * inv;
        const double gz0 = 1.0 - fz;
        const float c = (float)(cy[0] * gz0 + cy[1] * fz);
        cd[z] = (double)c * t.dt;
    }
    // (c dt) / dx: nothing to do for dx = 1, a product where 1 / dx is exact
    // (the branches are uniform)
    if (t.dx == 1.0) {
#pragma unroll
        for (int z = 0; z < 8; z++) k2[z] = (float)(cd[z] * cd[z]);
    } else if (t.dx_pow2) {
        const double r = t.rdx;
#pragma unroll
        for (int z = 0; z < 8; z++) {
            const double tt = cd[z] * r;
            k2[z] = (float)(tt * tt);
        }
    } else {
        const double d = t.dx;
#pragma unroll
        for (int z = 0; z < 8; z++) {
            const double tt = cd[z] / d;
            k2[z] = (float)(tt * tt);
        }
    }
}

// Zero both phi levels of a new slot and fill its C2 plane (fill_c2), unless
// the pool's C2 planes were filled at creation (then the slot's scalar C2
// is returned as stored).
__device__ __forceinline__ void zero_levels(const Tables& t, long long slot) {
    float* __restrict__ p0 = plane_of(t, slot, 0);
    float* __restrict__ p1 = plane_of(t, slot, 1);
    const int lane = lane_id();
#pragma unroll
    for (int z = 0; z < 8; z++) {
        p0[z * 64 + lane] = 0.f;
        p1[z * 64 + lane] = 0.f;
    }
}

__device__ float fill_slot(const Tables& t, const Shot& S, long long slot, int bx, int by, int bz) {
    zero_levels(t, slot);
    if (t.c2_ready) return t.slot_c2u[slot];
    return fill_c2(t, S, slot, bx, by, bz);
}

// --------------------------------------------------------------------------
// table initialisation
// --------------------------------------------------------------------------
// shot owning bitmap word w (shots own consecutive key ranges): the word's
// entry of the table, or a search over the shots
__device__ __forceinline__ int shot_of_word(const Tables& t, long long w) {
    if (t.word_shot) return t.word_shot[w];
    int lo = 0, hi = t.nshots - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (t.shots[mid].word_base <= w) lo = mid; else hi = mid - 1;
    }
    return lo;
}

__global__ void k_init_tables(Tables t, long long nkeys) {
    const long long gs = (long long)gridDim.x * blockDim.x;
    const long long g0 = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    for (long long i = g0; i < nkeys; i += gs) t.cell2box[i] = EMPTY;
    for (long long i = g0; i < (long long)t.nchunks * CHUNK_WORDS; i += gs) {
        t.bitmap[i] = 0ull;
        if (t.fast) t.bitmap2[i] = 0ull;
    }
    if (t.fast)
        for (long long i = g0; i < 6ll * t.nfblk; i += gs) t.fc_blk[i] = 0ull;
    for (long long i = g0; i < t.cap; i += gs) {
        t.slot_key[i] = -1;
        t.pin_until[2 * (size_t)(i)] = 0;
        t.pin_until[2 * (size_t)(i) + 1] = -1;
        t.flags[i] = 0;
        if (!t.c2_ready) t.slot_c2u[i] = __builtin_nanf("");
        t.sdlog[i] = 0;
    }
    if (g0 == 0) {
        DevState* st = t.st;
        st->step = 0; st->n_act = 0; st->n_new = 0; st->n_ret = 0;
        st->free_cnt = t.cap; st->error = 0; st->err_step = -1; st->emit = 0; st->nf_step = 0;
        for (int g = 0; g < 8; g++) st->adv_tk[g] = 0;
        st->adv_top = 0;
        st->peak_act = 0; st->scan_acc = 0; st->add_error = 0; st->n_dec = 0;
        st->cells_cur = 0; st->updates = 0; st->activations = 0; st->retirements = 0;
        st->cells_cur_u = 0; st->updates_u = 0; st->decays = 0;
        st->cells_cur_l = 0; st->updates_l = 0;
        st->maxbits = 0u; st->trig_cur = t.trigger; st->ret_cur = t.retire; st->n_ne = 0;
        st->free_next = t.cap;
        st->n_gblocks = 0; st->grad_error = 0;
    }
}

// One wave per key: with a pool of one slot per key a block's C2 plane
// depends only on its key, so it is computed once, when the pool is made
// (the activation of a block then only zeroes its two phi levels).
__global__ __launch_bounds__(256) void k_prefill_c2(Tables t, long long nkeys) {
    const long long G = ((long long)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    if (G >= nkeys) return;
    const int shot = shot_of_word(t, G >> 6);
    const Shot& S = t.shots[shot];
    int bx, by, bz;
    key_to_block(S, (unsigned)(G - S.key_base), bx, by, bz);
    const float u = fill_c2(t, S, G, bx, by, bz);
    if (lane_id() == 0) t.slot_c2u[G] = u;
}

hipError_t launch_prefill_c2(const Tables& t, long long nkeys, hipStream_t s) {
    if (!t.c2_ready || t.cap < nkeys) return hipErrorInvalidValue;
    const long long grid = (nkeys + 3) / 4;
    if (grid > 0x7fffffffLL) return hipErrorInvalidValue;
    if (grid > 0) hipLaunchKernelGGL(k_prefill_c2, dim3((unsigned)grid), dim3(256), 0, s, t, nkeys);
    return hipGetLastError();
}

hipError_t launch_init_tables(const Tables& t, long long nkeys, hipStream_t s) {
    long long n = nkeys > t.nwords ? nkeys : t.nwords;
    if ((long long)t.cap > n) n = t.cap;
    long long grid = (n + 255) / 256;
    if (grid > 65536) grid = 65536;
    if (grid < 1) grid = 1;
    hipLaunchKernelGGL(k_init_tables, dim3((unsigned)grid), dim3(256), 0, s, t, nkeys);
    return hipGetLastError();
}

// --------------------------------------------------------------------------
// Block stencil + source insertion + face/keep ballots
// --------------------------------------------------------------------------
// LDS tile per wave: columns (xx, yy) in [0,10)^2 (node x = xx - 1,
// y = yy - 1) of 8 z values each; interior 8x8 from the block, the four x/y
// side faces from the neighbours, corners unused.
typedef int row8 __attribute__((ext_vector_type(8)));
constexpr int TILE_COLS = 10;
constexpr int TILE_FLOATS = TILE_COLS * TILE_COLS * BE;

// W: waves per workgroup; P: blocks per wave (1 or 2).  A workgroup pass
// takes B = W * P consecutive list entries, which in a full tile are
// x-adjacent blocks; wave w takes entries w * P .. w * P + P - 1 of the pass
// and issues the loads of its P blocks together (with P = 2 the two blocks
// sit in consecutive slots, so each plane array is read as one 4 KiB run per
// wave: on the stencil's access pattern 6.06 TB/s against 5.67 TB/s with one
// block per wave at the same occupancy).
// MODE: STEP_PLAIN, or STEP_RECORD (a recomputed forward step of the adjoint:
// also store L u^n of every entry and its list index per key).
template <bool ADAPT, int W, int P, int MODE>
__global__ __launch_bounds__(64 * W) void k_block_step(Tables t) {
    constexpr int BASE = MODE & 3;
    constexpr bool LAT = (MODE & STEP_LAT) != 0;
    static_assert(BASE == STEP_PLAIN || BASE == STEP_RECORD || BASE == STEP_GRAD, "stencil variants");
    static_assert(BASE != STEP_GRAD || (!ADAPT && P == 1), "the adjoint field: constant levels, a block per wave");
    static_assert(!LAT || !ADAPT, "lattice records: constant levels");
    constexpr int B = W * P;
    static_assert(B <= 8, "a pass of the workgroup stays inside one group of 8 entries");
    // two sets of per-block tiles: iteration k writes set k & 1, so one
    // workgroup barrier per iteration separates writes from every read
    __shared__ __align__(16) float lds[2][B][TILE_FLOATS];
    const DevState* st = t.st;
    const int n = st->step;
    if (halted_before(st, n)) return;
    const int nact = st->n_act;
    const int p = n & 1;
    const int lane = lane_id();
    const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int x = lane & 7, y = lane >> 3;
    // face loaders: lane -> (a, zz) on a side face
    const int a = lane & 7, zz = lane >> 3;

    // XCD-aware split: workgroup b runs on XCD b % 8.  The (spatially
    // ordered) list is cut into groups of 2^lg entries dealt round-robin to
    // the XCDs, so neighbouring blocks of a group share one XCD's L2 while all
    // XCDs sweep one common window of the pool (one front in HBM rather than
    // eight).  Entry j of XCD x is list entry gidx(j).  Groups are 128 entries
    // (two 4^3 tiles; where a row of tiles is 16 tiles, each XCD then takes
    // the same two tiles of every row of a full set, with their y and z
    // neighbours), 256 for the adjoint field (each measured faster for its
    // variant), fewer for short lists so that every XCD has work.
    const int per = gridDim.x >> 3;
    const int xcd = blockIdx.x & 7, jw = blockIdx.x >> 3;
    int lg = BASE == STEP_GRAD ? 8 : 7;
    while (lg > 3 && (nact >> 3) < (1 << lg)) lg--;          // B <= 8 divides every group
    const int grp = 1 << lg;
    const int ng = (nact + grp - 1) >> lg;
    const int nfull = nact >> lg, rem = nact - (nfull << lg);
    int end = ng > xcd ? (((ng - 1 - xcd) >> 3) + 1) << lg : 0;
    if (rem && (nfull & 7) == xcd) end -= grp - rem;          // the partial group is this XCD's last
    auto gidx = [&](int j) { return ((((j >> lg) << 3) + xcd) << lg) + (j & (grp - 1)); };
    const float trig = t.trigger, ret = t.retire;
    float wave_max = 0.f;
    unsigned long long nonfinite = 0ull;       // lanes that wrote a NaN or infinity
    // adjoint field: nodes whose gradient term this workgroup formed
    __shared__ unsigned long long wg_terms;
    unsigned long long terms = 0;
    if constexpr (BASE == STEP_GRAD) {
        if (threadIdx.x == 0) wg_terms = 0;
        __syncthreads();
    }

    // Each list entry has a row {slot, 6 neighbour slots, global key} written by
    // the compaction; the next rows are fetched while the current blocks are
    // processed, so only the data loads sit on the critical path.
    const scalar_ptr<int> rows = as_scalar((const int*)t.rows);
    // per slot {pin, first source}: one 8-byte scalar load for both, made
    // only for blocks whose row says they have sources.  (Scalar loads share
    // their wait counter with the LDS, so one that misses the scalar cache
    // delays the block's LDS waits: loading it for every block cost 3.7 %
    // of the stencil's time on the 64-shot batch, 1468 against 1415 us per
    // launch, whose per-slot table is 21 MB; a second scalar load per block
    // cost 2 % on the 512^3 workload.)
    const scalar_ptr<unsigned long long> pin_head = as_scalar((const unsigned long long*)t.pin_until);
    const scalar_ptr<float> slot_c2u = as_scalar((const float*)t.slot_c2u);
    const int stride = per * B;
    // The loop count is uniform over the workgroup (barriers below).  Entry
    // j = wid * P + q of the pass takes the x face it shares with entry j - 1
    // or j + 1 of the same pass from that entry's tile.
    int r[P][8], sl_prev[P], sl_next[P];
    auto fetch = [&](int ib0) {
#pragma unroll
        for (int q = 0; q < P; q++) {
            const int j = wid * P + q;
            const int i = ib0 + j;
#pragma unroll
            for (int k = 0; k < 8; k++) r[q][k] = 0;
            sl_prev[q] = EMPTY;
            sl_next[q] = EMPTY;
            if (i < end) {
                // the whole 32-byte row in one scalar load, whichever fields
                // the variant uses (split loads measured 2 % slower)
                const row8 v = *(const __attribute__((address_space(4))) row8*)(rows + 8 * (size_t)gidx(i));
#pragma unroll
                for (int k = 0; k < 8; k++) r[q][k] = v[k];
                if (j > 0) sl_prev[q] = rows[8 * (size_t)gidx(i - 1)];
                if (j < B - 1 && i + 1 < end) sl_next[q] = rows[8 * (size_t)gidx(i + 1)];
            }
        }
    };
    int ib = jw * B;
    fetch(ib);
    int buf = 0;
    for (; ib < end; ib += stride, buf ^= 1) {
        bool have[P], share_m[P], share_p[P];
        int slot[P], nb[P][6], G[P], pinned[P], shead[P], li[P];
        bool has_src[P];
        float cur[P][8], prv[P][8], k2[P][8], zlo[P], zhi[P];
        float* out_p[P];
        // adjoint field: L u^{m-1} of the forward block (fi: its entry in the
        // store of forward step m - 1, -1 if it was inactive), the key's
        // FP32 partial gradient (gb: its gradient block, -1 if none yet)
        float lu[P][8], ga[P][8];
        int fi[P], gb[P];
        // lattice records (STEP_LAT)
        bool islat[P];
        double latv[P];
        int4 latm[P];
#pragma unroll
        for (int q = 0; q < P; q++) {
            const int j = wid * P + q;
            have[q] = ib + j < end;
            li[q] = gidx(ib + j);
            slot[q] = r[q][0];
#pragma unroll
            for (int d = 0; d < 6; d++) nb[q][d] = r[q][1 + d];
            G[q] = row_key(r[q][7]);
            has_src[q] = r[q][7] < 0;
            share_m[q] = have[q] && j > 0 && nb[q][0] >= 0 && nb[q][0] == sl_prev[q];
            share_p[q] = have[q] && j < B - 1 && nb[q][1] >= 0 && nb[q][1] == sl_next[q];
        }
        fetch(ib + stride);
        // all loads of the wave's blocks, then their tiles.  The wave raises
        // its own issue priority while it issues the loads, so that a wave
        // starting its blocks gets its loads out ahead of waves busy with
        // their arithmetic and LDS work (on the 512^3 two-layer workload 138.2
        // against 140.5 us per launch with one block per wave at 16 waves per
        // CU, 140.5 against 147.1 us with two blocks per wave).
        float fmx[P], fpx[P], fmy[P], fpy[P];
        __builtin_amdgcn_s_setprio(1);
#pragma unroll
        for (int q = 0; q < P; q++) {
            zlo[q] = 0.f; zhi[q] = 0.f; pinned[q] = 0; shead[q] = -1; out_p[q] = nullptr;
            fmx[q] = 0.f; fpx[q] = 0.f; fmy[q] = 0.f; fpy[q] = 0.f;
            fi[q] = -1; gb[q] = -1;
            if (!have[q]) continue;
            if constexpr (BASE == STEP_GRAD) {
                fi[q] = as_scalar(t.g_fidx)[G[q]];
                if (fi[q] >= 0) {
                    gb[q] = as_scalar((const int*)t.g_slot)[G[q]];
                    const float* __restrict__ lp = t.g_lap + (size_t)fi[q] * BV;
#pragma unroll
                    for (int z = 0; z < 8; z++) lu[q][z] = __builtin_nontemporal_load(&lp[z * 64 + lane]);
                    if (gb[q] >= 0) {
                        const float* __restrict__ gp = t.g_gs + (size_t)gb[q] * BV;
#pragma unroll
                        for (int z = 0; z < 8; z++) ga[q][z] = __builtin_nontemporal_load(&gp[z * 64 + lane]);
                    }
                }
            }
            if (has_src[q]) {
                const unsigned long long ph = pin_head[slot[q]];    // {pin, first source}
                pinned[q] = (int)(unsigned)ph;
                shead[q] = (int)(unsigned)(ph >> 32);
            }
            const float c2u = slot_c2u[slot[q]];
            if constexpr (LAT) {
                // the slot's lattice record (80 B instead of the 2 KiB plane:
                // corners in lanes 0-7, offsets in every lane) before the data,
                // and whether or not the slot holds one (no wait on c2u here),
                // so that its C2 is formed while the data loads are in flight
                latv[q] = t.slot_lat[8 * (size_t)slot[q] + (lane & 7)];
                latm[q] = t.slot_latm[slot[q]];
            }
            const float* __restrict__ cur_p = plane_of(t, slot[q], p);
            out_p[q] = plane_of(t, slot[q], 1 - p);
            const float* __restrict__ c2_p = plane_of(t, slot[q], PLANE_C2);
#pragma unroll
            for (int z = 0; z < 8; z++) {
                cur[q][z] = cur_p[z * 64 + lane];
                prv[q][z] = __builtin_nontemporal_load(&out_p[q][z * 64 + lane]);
            }
            islat[q] = LAT && __float_as_uint(c2u) == LAT_C2_BITS;
            if (c2u == c2u) {
#pragma unroll
                for (int z = 0; z < 8; z++) k2[q][z] = c2u;
            } else if (!islat[q]) {
#pragma unroll
                for (int z = 0; z < 8; z++) k2[q][z] = __builtin_nontemporal_load(&c2_p[z * 64 + lane]);
            }
            if (nb[q][4] >= 0) zlo[q] = plane_of(t, nb[q][4], p)[7 * 64 + lane];
            if (nb[q][5] >= 0) zhi[q] = plane_of(t, nb[q][5], p)[0 * 64 + lane];
            if (nb[q][0] >= 0 && !share_m[q]) fmx[q] = plane_of(t, nb[q][0], p)[zz * 64 + a * 8 + 7];
            if (nb[q][1] >= 0 && !share_p[q]) fpx[q] = plane_of(t, nb[q][1], p)[zz * 64 + a * 8 + 0];
            if (nb[q][2] >= 0) fmy[q] = plane_of(t, nb[q][2], p)[zz * 64 + 7 * 8 + a];
            if (nb[q][3] >= 0) fpy[q] = plane_of(t, nb[q][3], p)[zz * 64 + 0 * 8 + a];
        }
        __builtin_amdgcn_s_setprio(0);
        if constexpr (LAT) {
            // C2 from the lattice records, while the blocks' data are in flight
#pragma unroll
            for (int q = 0; q < P; q++)
                if (have[q] && islat[q]) lattice_c2(t, latv[q], latm[q], x, y, k2[q]);
        }
#pragma unroll
        for (int q = 0; q < P; q++) {
            if (!have[q]) continue;
            float* T = lds[buf][wid * P + q];
            float4* own = (float4*)(T + ((y + 1) * TILE_COLS + (x + 1)) * BE);
            own[0] = make_float4(cur[q][0], cur[q][1], cur[q][2], cur[q][3]);
            own[1] = make_float4(cur[q][4], cur[q][5], cur[q][6], cur[q][7]);
            T[((a + 1) * TILE_COLS + 0) * BE + zz] = fmx[q];
            T[((a + 1) * TILE_COLS + 9) * BE + zz] = fpx[q];
            T[(0 * TILE_COLS + (a + 1)) * BE + zz] = fmy[q];
            T[(9 * TILE_COLS + (a + 1)) * BE + zz] = fpy[q];
        }
        __syncthreads();   // every tile of this set is written
#pragma unroll
        for (int q = 0; q < P; q++) {
            if (!have[q]) continue;
            const int j = wid * P + q;
            const float* T = lds[buf][j];
            float xm[8], xp[8], ym[8], yp[8];
            {
                const float* Tm = lds[buf][j > 0 ? j - 1 : 0];
                const float* Tp = lds[buf][j < B - 1 ? j + 1 : B - 1];
                const float4* c_xm = (const float4*)(x == 0 && share_m[q] ? Tm + ((y + 1) * TILE_COLS + 8) * BE
                                                                          : T + ((y + 1) * TILE_COLS + x) * BE);
                const float4* c_xp = (const float4*)(x == 7 && share_p[q] ? Tp + ((y + 1) * TILE_COLS + 1) * BE
                                                                          : T + ((y + 1) * TILE_COLS + x + 2) * BE);
                const float4* c_ym = (const float4*)(T + (y * TILE_COLS + x + 1) * BE);
                const float4* c_yp = (const float4*)(T + ((y + 2) * TILE_COLS + x + 1) * BE);
                float4 v0 = c_xm[0], v1 = c_xm[1];
                xm[0] = v0.x; xm[1] = v0.y; xm[2] = v0.z; xm[3] = v0.w;
                xm[4] = v1.x; xm[5] = v1.y; xm[6] = v1.z; xm[7] = v1.w;
                v0 = c_xp[0]; v1 = c_xp[1];
                xp[0] = v0.x; xp[1] = v0.y; xp[2] = v0.z; xp[3] = v0.w;
                xp[4] = v1.x; xp[5] = v1.y; xp[6] = v1.z; xp[7] = v1.w;
                v0 = c_ym[0]; v1 = c_ym[1];
                ym[0] = v0.x; ym[1] = v0.y; ym[2] = v0.z; ym[3] = v0.w;
                ym[4] = v1.x; ym[5] = v1.y; ym[6] = v1.z; ym[7] = v1.w;
                v0 = c_yp[0]; v1 = c_yp[1];
                yp[0] = v0.x; yp[1] = v0.y; yp[2] = v0.z; yp[3] = v0.w;
                yp[4] = v1.x; yp[5] = v1.y; yp[6] = v1.z; yp[7] = v1.w;
            }
            float nv[8], lapv[8];
#pragma unroll
            for (int z = 0; z < 8; z++) {
                const float zd = z > 0 ? cur[q][z - 1] : zlo[q];
                const float zu = z < 7 ? cur[q][z + 1] : zhi[q];
                const float s = ((xp[z] + xm[z]) + (yp[z] + ym[z])) + (zu + zd);
                lapv[z] = s - 6.0f * cur[q][z];
                nv[z] = (2.0f * cur[q][z] - prv[q][z]) + k2[q][z] * lapv[z];
            }
            if constexpr (BASE == STEP_RECORD) {
                // L u^n of this entry, for the gradient terms of adjoint step n + 1
                if (li[q] < t.rec_lapcap) {
                    float* __restrict__ lp = t.rec_lap + (size_t)li[q] * BV;
#pragma unroll
                    for (int z = 0; z < 8; z++) __builtin_nontemporal_store(lapv[z], &lp[z * 64 + lane]);
                    if (lane == 0) t.rec_fidx[G[q]] = li[q];
                } else if (lane == 0) {
                    t.st->grad_error = 1;
                }
            }
            // additive source insertion (before the predicates): the block's
            // own sources, a range of the key-ordered table, in the order they
            // were added (a counted loop: walking a chain of indices cost 2 %
            // of the stencil's time, even for blocks without sources)
            if (pinned[q] > n && shead[q] >= 0) {
                const int first = shead[q] & 0xFFFFFF, cnt = shead[q] >> 24;
                for (int s = first; s < first + cnt; s++) {
                    const Src e = t.src[s];
                    const int k = n - e.t0;
                    if (k < 0 || k >= e.ns) continue;
                    const float w = t.srcw[e.w_off + k];
                    if (lane == (e.local & 63)) {
                        const int ez = e.local >> 6;
#pragma unroll
                        for (int z = 0; z < 8; z++)
                            if (z == ez) nv[z] = nv[z] + w;
                    }
                }
            }
#pragma unroll
            for (int z = 0; z < 8; z++) __builtin_nontemporal_store(nv[z], &out_p[q][z * 64 + lane]);
            if constexpr (BASE == STEP_GRAD) {
                // gradient term mu^m (L u^{m-1}) of the key, FP32 product and
                // sum; a key's first term hands out its gradient block and
                // clears the block's FP64 sum
                if (fi[q] >= 0) {
                    int g = gb[q];
                    if (g < 0) {
                        if (lane == 0) {
                            g = atomicAdd(&t.st->n_gblocks, 1);
                            if (g < t.g_cap) t.g_slot[G[q]] = g;
                            else t.st->grad_error = 1;
                        }
                        g = __shfl(g, 0);
                        if (g < t.g_cap) {
                            double* __restrict__ ap = t.g_acc + (size_t)g * BV;
#pragma unroll
                            for (int z = 0; z < 8; z++) {
                                ap[z * 64 + lane] = 0.0;
                                ga[q][z] = 0.f;
                            }
                        }
                    }
                    if (g < t.g_cap) {
                        float* __restrict__ gp = t.g_gs + (size_t)g * BV;
#pragma unroll
                        for (int z = 0; z < 8; z++) __builtin_nontemporal_store(ga[q][z] + nv[z] * lu[q][z], &gp[z * 64 + lane]);
                        const Shot& S0 = t.shots[0];
                        int bx, by, bz;
                        key_to_block(S0, (unsigned)((long long)G[q] - S0.key_base), bx, by, bz);
                        terms += (unsigned long long)block_cells(S0, bx, by, bz);
                    }
                }
            }
            // column maxima of |phi^{n+1}| and |phi^n|
            float colmax = fabsf(nv[0]), curmax = fabsf(cur[q][0]);
#pragma unroll
            for (int z = 1; z < 8; z++) {
                colmax = fmaxf(colmax, fabsf(nv[z]));
                curmax = fmaxf(curmax, fabsf(cur[q][z]));
            }
            // a value that is not finite fails every level comparison, so its
            // block would just be released and the value lost: the run stops
            // after this step instead (recorded once per wave, after its
            // loop).  An infinity makes the column maximum infinite; a NaN,
            // which the maximum skips, makes the column's sum NaN (an
            // overflowing sum of finite values is infinite, not NaN).  Both
            // cost no more time than the maximum alone; a NaN-propagating
            // maximum cost 1.8 % of the stencil's time on 16-byte nodes.
            {
                const float sum = ((nv[0] + nv[1]) + (nv[2] + nv[3])) + ((nv[4] + nv[5]) + (nv[6] + nv[7]));
                nonfinite |= __ballot(sum != sum || !(colmax <= 3.402823466e38f));
            }

            if constexpr (ADAPT) {
                // per-block maxima (Table 1 Max_cell_val, per face and whole block);
                // the plan compares them with this step's levels
                float v[8] = {x == 0 ? colmax : 0.f, x == 7 ? colmax : 0.f, y == 0 ? colmax : 0.f,
                              y == 7 ? colmax : 0.f, fabsf(nv[0]), fabsf(nv[7]), colmax, curmax};
                for (int o = 32; o > 0; o >>= 1) {
#pragma unroll
                    for (int k = 0; k < 8; k++) v[k] = fmaxf(v[k], __shfl_xor(v[k], o));
                }
                if (lane == 0) {
                    float4* bm = (float4*)(t.bmax + 8 * (size_t)slot[q]);
                    bm[0] = make_float4(v[0], v[1], v[2], v[3]);
                    bm[1] = make_float4(v[4], v[5], v[6], v[7]);
                }
                wave_max = fmaxf(wave_max, v[6]);
            } else {
                const bool keep = colmax > ret || curmax > ret;
                const bool col = colmax > trig, hot = curmax > trig;
                const unsigned long long bk = __ballot(keep);
                const unsigned long long bc = __ballot(col);
                const unsigned long long bh = __ballot(hot);
                const unsigned long long bz0 = __ballot(fabsf(nv[0]) > trig);
                const unsigned long long bz7 = __ballot(fabsf(nv[7]) > trig);
                if (lane == 0) {
                    unsigned f = 0;
                    if (bc & 0x0101010101010101ull) f |= 1u;    // x = 0 column
                    if (bc & 0x8080808080808080ull) f |= 2u;    // x = 7
                    if (bc & 0x00000000000000FFull) f |= 4u;    // y = 0
                    if (bc & 0xFF00000000000000ull) f |= 8u;    // y = 7
                    if (bz0) f |= 16u;
                    if (bz7) f |= 32u;
                    // a source pin that holds past this step also keeps the
                    // block and makes it hot for the 26-neighbour rule (only
                    // rows with the source bit load the pin)
                    const bool pin_holds = pinned[q] > n + 1;
                    if (bk || pin_holds) f |= (unsigned)KEEP_BIT;
                    if ((bc | bh) || pin_holds) f |= (unsigned)HOT_BIT;
                    t.flags[slot[q]] = (unsigned char)f;
                }
            }
        }
    }
    if (ADAPT && lane == 0 && wave_max > 0.f)
        atomicMax((unsigned*)&t.st->maxbits, __float_as_uint(wave_max));   // non-negative floats order as integers
    if (nonfinite && lane == 0) atomicCAS(&t.st->nf_step, 0, n + 1);
    if constexpr (BASE == STEP_GRAD) {
        // one slot per workgroup (a global atomic from every wave would
        // serialise on one address at the kernel's end)
        if (lane == 0 && terms) atomicAdd(&wg_terms, terms);
        __syncthreads();
        if (threadIdx.x == 0 && wg_terms && blockIdx.x < GRAD_ACCUM_MAX_WG) t.g_terms_wg[blockIdx.x] += wg_terms;
    }
    if constexpr (!ADAPT) {
        // a step without an activation update and without receivers: the
        // last workgroup to finish advances the step, as k_advance would.
        // Every workgroup read the step counter at its start, before taking
        // its ticket, and the last one reads nothing that another wrote in
        // this launch, so the tickets alone order it.  Tickets per class of
        // workgroups (blockIdx % 8), then one per class: no counter takes
        // more than a few hundred same-address atomics (one counter for all
        // 1024 workgroups of the adjoint field cost about 4 us per launch).
        bool last = false;
        if (t.self_advance && threadIdx.x == 0) {
            const int g = blockIdx.x & 7;
            const int in_g = ((int)gridDim.x - g + 7) >> 3;            // workgroups of class g
            const int ng = gridDim.x < 8 ? (int)gridDim.x : 8;         // classes
            if (atomicAdd(&t.st->adv_tk[g], 1) == in_g - 1) last = atomicAdd(&t.st->adv_top, 1) == ng - 1;
        }
        if (last) {
            DevState* sw = t.st;
            for (int g = 0; g < 8; g++) sw->adv_tk[g] = 0;
            sw->adv_top = 0;
            sw->updates += sw->cells_cur;
            sw->updates_u += sw->cells_cur_u;
            sw->updates_l += sw->cells_cur_l;
            sw->step = n + 1;
            sw->maxbits = 0u;
        }
    }
}

template <bool ADAPT, int W, int P, int MODE>
static int occupancy_wpm() {
    int nb = 0;
    const hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_block_step<ADAPT, W, P, MODE>,
                                                                      64 * W, 0);
    return e == hipSuccess ? nb : 0;
}

// the adjoint field's variant: constant levels, a block per wave, tiles of 4 or 8
template <bool ADAPT, int W, int P>
constexpr bool grad_variant() { return !ADAPT && P == 1 && (W == 4 || W == 8); }

template <bool ADAPT, int W, int P>
static int occupancy_wp(int mode) {
    if constexpr (!ADAPT) {
        if (mode & STEP_LAT) {
            const int base = mode & 3;
            if (base == STEP_GRAD) {
                if constexpr (grad_variant<ADAPT, W, P>()) return occupancy_wpm<ADAPT, W, P, STEP_GRAD | STEP_LAT>();
                return 0;
            }
            return base == STEP_RECORD ? occupancy_wpm<ADAPT, W, P, STEP_RECORD | STEP_LAT>()
                                       : occupancy_wpm<ADAPT, W, P, STEP_PLAIN | STEP_LAT>();
        }
    }
    mode &= 3;
    if (mode == STEP_GRAD) {
        if constexpr (grad_variant<ADAPT, W, P>()) return occupancy_wpm<ADAPT, W, P, STEP_GRAD>();
        return 0;
    }
    return mode == STEP_RECORD ? occupancy_wpm<ADAPT, W, P, STEP_RECORD>() : occupancy_wpm<ADAPT, W, P, STEP_PLAIN>();
}

template <bool ADAPT>
static int occupancy_w(int w, int pb, int mode) {
    if (pb == 1) {
        if (w == 2) return occupancy_wp<ADAPT, 2, 1>(mode);
        if (w == 4) return occupancy_wp<ADAPT, 4, 1>(mode);
        if (w == 8) return occupancy_wp<ADAPT, 8, 1>(mode);
    } else if (pb == 2) {
        if (w == 2) return occupancy_wp<ADAPT, 2, 2>(mode);
        if (w == 4) return occupancy_wp<ADAPT, 4, 2>(mode);
    }
    return 0;
}

int block_step_occupancy(bool adaptive, int w, int pb, int mode) {
    return adaptive ? occupancy_w<true>(w, pb, mode) : occupancy_w<false>(w, pb, mode);
}

bool block_step_shape_ok(int w, int pb) {
    return (pb == 1 && (w == 2 || w == 4 || w == 8)) || (pb == 2 && (w == 2 || w == 4));
}

template <bool ADAPT, int W, int P, int MODE>
static void launch_wpm(const Tables& t, int grid, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
    void (*kern)(Tables) = k_block_step<ADAPT, W, P, MODE>;
    if (e0 || e1)                   // timed launch (never inside a graph capture)
        hipExtLaunchKernelGGL(kern, dim3(grid), dim3(64 * W), 0, s, e0, e1, 0, t);
    else
        hipLaunchKernelGGL(kern, dim3(grid), dim3(64 * W), 0, s, t);
}

template <bool ADAPT, int W, int P>
static void launch_wp(const Tables& t, int grid, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
    if constexpr (!ADAPT) {
        if (t.lat_c2) {
            if (t.g_lap) {
                if constexpr (grad_variant<ADAPT, W, P>()) launch_wpm<ADAPT, W, P, STEP_GRAD | STEP_LAT>(t, grid, s, e0, e1);
            } else if (t.rec_lap) {
                launch_wpm<ADAPT, W, P, STEP_RECORD | STEP_LAT>(t, grid, s, e0, e1);
            } else {
                launch_wpm<ADAPT, W, P, STEP_PLAIN | STEP_LAT>(t, grid, s, e0, e1);
            }
            return;
        }
    }
    if (t.g_lap) {
        if constexpr (grad_variant<ADAPT, W, P>()) launch_wpm<ADAPT, W, P, STEP_GRAD>(t, grid, s, e0, e1);
    } else if (t.rec_lap) {
        launch_wpm<ADAPT, W, P, STEP_RECORD>(t, grid, s, e0, e1);
    } else {
        launch_wpm<ADAPT, W, P, STEP_PLAIN>(t, grid, s, e0, e1);
    }
}

template <bool ADAPT>
static void launch_adapt(const Tables& t, int grid, int w, int pb, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
    if (pb == 1) {
        if (w == 2) launch_wp<ADAPT, 2, 1>(t, grid, s, e0, e1);
        if (w == 4) launch_wp<ADAPT, 4, 1>(t, grid, s, e0, e1);
        if (w == 8) launch_wp<ADAPT, 8, 1>(t, grid, s, e0, e1);
    } else {
        if (w == 2) launch_wp<ADAPT, 2, 2>(t, grid, s, e0, e1);
        if (w == 4) launch_wp<ADAPT, 4, 2>(t, grid, s, e0, e1);
    }
}

hipError_t launch_block_step(const Tables& t, int grid, int w, int pb, hipStream_t s, hipEvent_t e0,
                             hipEvent_t e1) {
    if (!block_step_shape_ok(w, pb)) return hipErrorInvalidValue;
    // the adjoint field's variant exists for constant levels and tiles of 4 or
    // 8 blocks, one per wave; its grid stays within GRAD_ACCUM_MAX_WG
    if (t.g_lap && (t.adaptive || pb != 1 || (w != 4 && w != 8) || grid > GRAD_ACCUM_MAX_WG))
        return hipErrorInvalidValue;
    if (t.adaptive) launch_adapt<true>(t, grid, w, pb, s, e0, e1);
    else launch_adapt<false>(t, grid, w, pb, s, e0, e1);
    return hipGetLastError();
}

// --------------------------------------------------------------------------
// slot placement (whole wave): claim the first free slot at or after the
// preferred slot, 64 slots per probe, with a compare-and-swap on slot_key.
// With a pool of at least one slot per key the preferred slot is the key, so
// the pool is laid out in the order of the active list and the stencil
// streams it.  A smaller pool places whole tiles (64 consecutive keys) at a
// hashed group of 64 slots: an active region that is compact in space (and
// so spans a few ranges of keys) spreads evenly over the pool, and each
// tile's blocks stay contiguous.  Returns -1 only if no slot was free in a
// full pass.
// --------------------------------------------------------------------------
__device__ __forceinline__ long long preferred_slot(const Tables& t, long long G) {
    const long long cap = t.cap;
    if (cap >= t.nkeys) return G;
    const long long groups = cap >> 6;
    if (groups < 1) return G % cap;
    // Fibonacci hashing of the tile number
    const unsigned long long h = (unsigned long long)(G >> 6) * 0x9E3779B97F4A7C15ull;
    return (long long)((h >> 32) % (unsigned long long)groups) * 64 + (G & 63);
}

__device__ int place_slot(const Tables& t, long long G) {
    const int lane = lane_id();
    const long long cap = t.cap;
    const long long start = preferred_slot(t, G);
    const long long passes = cap / 64 + 2;
    for (long long it = 0; it < passes; it++) {
        long long s = start + it * 64 + lane;
        s %= cap;
        unsigned long long* p = (unsigned long long*)&t.slot_key[s];
        const unsigned long long v = __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        unsigned long long m = __ballot(v == ~0ull);
        while (m) {
            const int l = __ffsll((long long)m) - 1;
            bool won = false;
            if (lane == l) {
                unsigned long long expected = ~0ull;
                won = __hip_atomic_compare_exchange_strong(p, &expected, (unsigned long long)G,
                                                           __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                                           __HIP_MEMORY_SCOPE_AGENT);
            }
            if (__ballot(won)) return __shfl((int)s, l);
            m &= m - 1;
        }
    }
    return -1;
}

// --------------------------------------------------------------------------
// Keep / release / claim ("Updating active cells", items 1-4, 6)
// --------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_plan(Tables t) {
    DevState* st = t.st;
    const int n = st->step;
    if (halted_before(st, n)) return;
    const int nact = st->n_act;
    const int p = n & 1;
    const int gsz = gridDim.x * blockDim.x;
    const int g0 = blockIdx.x * blockDim.x + threadIdx.x;

    if (g0 == 0) st->n_ne = 0;   // filled by the allocator's scan, read by the compaction
    // receivers: traces[n - trace_step0][r] = phi^{n+1}
    // levels of this step: constant, or relative to the domain maximum
    float trig = t.trigger, ret = t.retire;
    if (t.adaptive) {
        const float M = __uint_as_float(st->maxbits);
        trig = fmaxf(trig, t.trigger_rel * M);
        ret = fmaxf(ret, t.retire_rel * M);
        if (g0 == 0) {
            st->trig_cur = trig;
            st->ret_cur = ret;
        }
    }
    const int row = n - t.trace_step0;
    if (row >= 0 && row < t.trace_cap) {
        for (int r = g0; r < t.nrec; r += gsz) {
            const Rec e = t.rec[r];
            const int s = t.cell2box[e.key];
            t.traces[(size_t)row * t.nrec + r] =
                s >= 0 ? plane_of(t, s, 1 - p)[e.local] : 0.f;
        }
    }
    // a step that wrote a non-finite value keeps its list: the allocator
    // and the compaction see that and only advance the step
    if (st->nf_step) return;

    for (int base = blockIdx.x * blockDim.x; base < nact; base += gsz) {
        const int i = base + threadIdx.x;
        const bool valid = i < nact;
        int slot = 0, shot = 0;
        unsigned key = 0, f = 0;
        int bx = 0, by = 0, bz = 0;
        bool survive = false;
        // the entry's list row: slot, the 6 face neighbours' slots (as in
        // cell2box when the list was written; only this kernel, the
        // allocator and source activation, which rewrites the rows, change
        // cell2box between two plans), global key
        int nbs[6] = {EMPTY, EMPTY, EMPTY, EMPTY, EMPTY, EMPTY};
        if (valid) {
            const int4* rp = (const int4*)(t.rows + 8 * (size_t)i);
            const int4 r0 = rp[0], r1 = rp[1];
            slot = r0.x;
            nbs[0] = r0.y; nbs[1] = r0.z; nbs[2] = r0.w;
            nbs[3] = r1.x; nbs[4] = r1.y; nbs[5] = r1.z;
            shot = t.act_shot[i];
            key = (unsigned)((long long)row_key(r1.w) - t.shots[shot].key_base);
            if (t.adaptive) {
                const float* bm = t.bmax + 8 * (size_t)slot;
                f = 0;
                for (int d = 0; d < 6; d++)
                    if (bm[d] > trig) f |= 1u << d;
                if (bm[6] > ret || bm[7] > ret) f |= (unsigned)KEEP_BIT;
                if (bm[6] > trig || bm[7] > trig) f |= (unsigned)HOT_BIT;
            } else {
                f = t.flags[slot];
            }
            key_to_block(t.shots[shot], key, bx, by, bz);
            // (the stencil folds a holding source pin into the flags; the
            // levels of an adaptive run come from bmax, so it reads the pin)
            survive = (f & KEEP_BIT) != 0 || (t.adaptive && t.pin_until[2 * (size_t)(slot)] > n + 1);
        }
        if (t.interval <= 1) {
            // an active neighbour whose face toward us is above trigger keeps
            // us (a missing neighbour loads the entry's own slot, ignored:
            // conditional loads compile to a wait after each)
#pragma unroll
            for (int d = 0; d < 6; d++) {
                const int s2 = nbs[d] >= 0 ? nbs[d] : slot;
                const bool face = t.adaptive ? t.bmax[8 * (size_t)s2 + (d ^ 1)] > trig
                                             : ((t.flags[s2] >> (d ^ 1)) & 1u) != 0;
                if (nbs[d] >= 0 && face) survive = true;
            }
            for (int d = 0; d < 6; d++) {
                bool claim = false;
                long long nk = -1;
                if (valid && nbs[d] == EMPTY && ((f >> d) & 1u)) {
                    nk = neighbour_key(t.shots[shot], bx, by, bz, d);
                    if (nk >= 0) claim = atomicCAS(&t.cell2box[nk], EMPTY, CLAIMED) == EMPTY;
                }
                const int k = wave_append(&st->n_new, claim);
                if (claim) {
                    if (k < t.cap) {
                        t.new_key[k] = nk;
                        t.new_shot[k] = shot;
                    }
                    atomicOr(&t.bitmap[nk >> 6], 1ull << (nk & 63));
                }
            }
        } else {
            // update every `interval` (<= 8) steps: values move at most one node
            // per step, so a block that is hot (or still inserting a source)
            // must have all 26 nearest and diagonal neighbours active
            const bool hot = valid && (((f & HOT_BIT) != 0) || (t.adaptive && t.pin_until[2 * (size_t)(slot)] > n + 1));
            // the 26 neighbours, a layer of nine at a time: their keys and
            // slots, then their flags (and pins, in an adaptive run), each set
            // of loads issued together (a missing neighbour loads the entry's
            // own key and slot, ignored; loads under a condition compile to a
            // wait after each)
            const Shot& S = t.shots[shot];
            const int own = (int)(S.key_base + (long long)key);
            int nk26[27], s26[27];
#pragma unroll
            for (int zl = 0; zl < 3; zl++) {
#pragma unroll
                for (int j = 0; j < 9; j++) {
                    const int d = zl * 9 + j;
                    const int x2 = bx + d % 3 - 1, y2 = by + (d / 3) % 3 - 1, z2 = bz + d / 9 - 1;
                    const bool in = valid && d != 13 && x2 >= 0 && y2 >= 0 && z2 >= 0 && x2 < S.bx &&
                                    y2 < S.by && z2 < S.bz;
                    nk26[d] = in ? (int)(S.key_base + (long long)block_to_key(S, x2, y2, z2)) : -1;
                }
                int sl[9];
#pragma unroll
                for (int j = 0; j < 9; j++) sl[j] = t.cell2box[nk26[zl * 9 + j] >= 0 ? nk26[zl * 9 + j] : own];
                bool nh[9];
                if (t.adaptive) {
#pragma unroll
                    for (int j = 0; j < 9; j++) {
                        const int s2 = sl[j] >= 0 ? sl[j] : slot;
                        nh[j] = t.bmax[8 * (size_t)s2 + 6] > trig || t.bmax[8 * (size_t)s2 + 7] > trig ||
                                t.pin_until[2 * (size_t)s2] > n + 1;
                    }
                } else {
#pragma unroll
                    for (int j = 0; j < 9; j++) nh[j] = (t.flags[sl[j] >= 0 ? sl[j] : slot] & HOT_BIT) != 0;
                }
#pragma unroll
                for (int j = 0; j < 9; j++) {
                    s26[zl * 9 + j] = sl[j];
                    if (nk26[zl * 9 + j] >= 0 && sl[j] >= 0 && nh[j]) survive = true;
                }
            }
            for (int d = 0; d < 27; d++) {
                if (d == 13) continue;
                bool claim = false;
                const long long nk = nk26[d];
                if (nk >= 0 && hot && s26[d] == EMPTY) claim = atomicCAS(&t.cell2box[nk], EMPTY, CLAIMED) == EMPTY;
                const int k = wave_append(&st->n_new, claim);
                if (claim) {
                    if (k < t.cap) {
                        t.new_key[k] = nk;
                        t.new_shot[k] = shot;
                    }
                    atomicOr(&t.bitmap[nk >> 6], 1ull << (nk & 63));
                }
            }
        }
        // shutdown process (eq.(6)): a block that no longer qualifies keeps
        // running for shutdown_steps more steps with both levels scaled by
        // alpha after each, then is released; qualifying again cancels it
        bool release = valid && !survive, decay = false;
        if (valid && t.shutdown_steps > 0) {
            const int sd = t.sdlog[slot];
            if (survive) {
                if (sd) t.sdlog[slot] = 0;
            } else if (sd == 0) {
                t.sdlog[slot] = (unsigned char)t.shutdown_steps;
                release = false;
                decay = true;
            } else if (sd > 1) {
                t.sdlog[slot] = (unsigned char)(sd - 1);
                release = false;
                decay = true;
            }
        }
        // survivors: the list is in key order, so a wave's keys fall in one or
        // two bitmap words; OR the bits within each run of equal words and let
        // the first lane of the run do the atomic
        {
            const long long G = valid ? t.shots[shot].key_base + (long long)key : -1;
            const bool stays = valid && !release;
            const long long word = stays ? (G >> 6) : -1;
            unsigned long long bits = stays ? (1ull << (G & 63)) : 0ull;
            const int lane = lane_id();
            for (int o = 1; o < 64; o <<= 1) {
                const unsigned long long ob = __shfl_down(bits, o);
                const long long ow = __shfl_down(word, o);
                if (lane + o < 64 && ow == word) bits |= ob;
            }
            const long long prev_word = __shfl_up(word, 1);
            if (word >= 0 && (lane == 0 || prev_word != word)) atomicOr(&t.bitmap[word], bits);
        }
        const int kd = wave_append(&st->n_dec, decay);
        if (kd >= 0) t.dec_slot[kd] = slot;
        const int kr = wave_append(&st->n_ret, release);
        if (kr >= 0) {
            t.ret_slot[kr] = slot;
            t.ret_key[kr] = t.shots[shot].key_base + (long long)key;
        }
    }
}

hipError_t launch_plan(const Tables& t, int grid, hipStream_t s) {
    hipLaunchKernelGGL(k_plan, dim3(grid), dim3(256), 0, s, t);
    return hipGetLastError();
}

// A step without an activation update (update interval > 1): record the
// receivers of phi^{n+1}, then advance the step counter.  One workgroup.
__global__ __launch_bounds__(256) void k_advance(Tables t) {
    DevState* st = t.st;
    const int n = st->step;                 // read by every thread before thread 0 writes it
    if (halted_before(st, n)) return;
    const int p = n & 1;
    const int row = n - t.trace_step0;
    if (row >= 0 && row < t.trace_cap) {
        for (int r = threadIdx.x; r < t.nrec; r += blockDim.x) {
            const Rec e = t.rec[r];
            const int s = t.cell2box[e.key];
            t.traces[(size_t)row * t.nrec + r] =
                s >= 0 ? plane_of(t, s, 1 - p)[e.local] : 0.f;
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        st->updates += st->cells_cur;
        st->updates_u += st->cells_cur_u;
        st->updates_l += st->cells_cur_l;
        st->step = n + 1;
        st->maxbits = 0u;
    }
}

hipError_t launch_advance(const Tables& t, hipStream_t s) {
    hipLaunchKernelGGL(k_advance, dim3(1), dim3(256), 0, s, t);
    return hipGetLastError();
}

// --------------------------------------------------------------------------
// Pool allocator and bitmap popcounts; the last workgroup scans the
// counts and commits the step ("Boxes": vacant boxes are reused).
// --------------------------------------------------------------------------
// End of the activation update (one thread): the step's counters, the next
// list's length, and whether the compaction emits it (0: the step failed).
// The counters that every allocating workgroup reads at its start (n_new,
// n_ret, n_dec, free_cnt) are left alone here, since some of those
// workgroups may not have started yet: the compaction, the next launch,
// installs free_next and clears the others.
constexpr int SCAN1_MAX = 4;          // chunks per thread of the one-workgroup scan
__device__ void commit_step(const Tables& t, DevState* st, int nn, int nr, int nfree, unsigned total) {
    const int err = st->error || st->nf_step;
    if (!err || (st->error ? st->err_step == st->step : st->nf_step == st->step + 1)) {
        // the step's phi^{n+1} is complete
        st->updates += st->cells_cur;
        st->updates_u += st->cells_cur_u;
        st->updates_l += st->cells_cur_l;
        st->step += 1;
    }
    st->free_next = err ? nfree : nfree + nr - nn;
    if (!err) {
        st->activations += (unsigned long long)nn;
        st->retirements += (unsigned long long)nr;
        st->decays += (unsigned long long)st->n_dec;
        st->n_act = (int)total;
        if ((int)total > st->peak_act) st->peak_act = (int)total;
        st->cells_cur = 0;
        st->cells_cur_u = 0;
        st->cells_cur_l = 0;
        st->emit = 1;
    } else {
        st->emit = 0;
    }
    st->maxbits = 0u;
    __threadfence();
}

__global__ __launch_bounds__(256) void k_pool_count(Tables t) {
    DevState* st = t.st;
    __shared__ unsigned red[4];
    const int lane = lane_id();
    const int wid = threadIdx.x >> 6;
    const int err0 = st->error || st->nf_step;
    const int nn = st->n_new, nr = st->n_ret, nfree = st->free_cnt;
    const int n0 = st->step;
    // When the grid has workgroups beyond the scanning ones, those allocate
    // and the scan starts at once (it reads only the bitmap); otherwise every
    // workgroup allocates.  aw: this workgroup's index among the allocating
    // ones (-1: none), nalloc: their number.
    const int a0 = (int)gridDim.x > t.scan_wgs ? t.scan_wgs : 0;
    const int aw = (int)blockIdx.x - a0, nalloc = (int)gridDim.x - a0;

    if (!err0) {
        if (nn > nfree + nr) {
            if (blockIdx.x == 0 && threadIdx.x == 0) report_error(st, ERR_POOL, n0);
        } else {
            // Only when the free slots alone cannot hold the new blocks are
            // released slots handed over directly: new block k < handoff takes
            // released slot k.  Every other released slot is freed, and every
            // other new block claims a slot by placement.  At least as many
            // slots are free as there are placing blocks, so every placement
            // succeeds (slots freed here may be taken as well).
            const int handoff = nn > nfree ? nn - nfree : 0;
            const int gsz = nalloc * blockDim.x;
            for (int r = aw * blockDim.x + threadIdx.x; aw >= 0 && r < nr; r += gsz) {
                t.cell2box[t.ret_key[r]] = EMPTY;
                if (r >= handoff)
                    __hip_atomic_store(&t.slot_key[t.ret_slot[r]], -1LL, __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_AGENT);
            }
            // new blocks (wave per entry): slot, zero phi levels, C2 from media
            const int nwaves = nalloc * (blockDim.x >> 6);
            for (int k = aw * (blockDim.x >> 6) + wid; aw >= 0 && k < nn; k += nwaves) {
                const long long G = t.new_key[k];
                // one slot per key: slot G is only ever key G's (and no slot is
                // handed over, the free slots always outnumber the new blocks)
                const int slot = t.cap >= t.nkeys ? (int)G : k < handoff ? t.ret_slot[k] : place_slot(t, G);
                if (slot < 0) {                      // unreachable (see above): fail the step
                    if (lane == 0) report_error(st, -6, n0);
                    continue;
                }
                const int shot = t.new_shot[k];
                const Shot& S = t.shots[shot];
                int bx, by, bz;
                key_to_block(S, (unsigned)(G - S.key_base), bx, by, bz);
                const float c2u = fill_slot(t, S, slot, bx, by, bz);
                if (lane == 0) {
                    t.slot_c2u[slot] = c2u;
                    t.sdlog[slot] = 0;
                    t.cell2box[G] = slot;
                    t.slot_key[slot] = G;
                    t.pin_until[2 * (size_t)(slot)] = 0;
                    t.pin_until[2 * (size_t)(slot) + 1] = -1;
                }
            }
        }
    }

    // shutdown decay (eq.(6)): both stored levels of the listed blocks times alpha
    if (!err0 && nn <= nfree + nr) {
        const int nd = st->n_dec;
        const float alpha = t.shutdown_alpha;
        const int nwaves = nalloc * (blockDim.x >> 6);
        for (int k = aw * (blockDim.x >> 6) + wid; aw >= 0 && k < nd; k += nwaves) {
            float* b0 = plane_of(t, t.dec_slot[k], 0);
            float* b1 = plane_of(t, t.dec_slot[k], 1);
#pragma unroll
            for (int j = 0; j < 8; j++) {
                b0[j * 64 + lane] = b0[j * 64 + lane] * alpha;
                b1[j * 64 + lane] = b1[j * 64 + lane] * alpha;
            }
        }
    }

    // Two-level scan of the bitmap by the first scan_wgs workgroups (the
    // rest only allocate).  Workgroup g owns chunks [g * C, g * C + C): each
    // thread counts a contiguous run of them, the workgroup scans the runs
    // and stores every chunk's offset inside the range and the range total;
    // the last scanning workgroup to finish commits the step, and the
    // compaction turns the range totals into range offsets.
    const int nw = blockDim.x >> 6;
    do {
        if ((int)blockIdx.x >= t.scan_wgs) break;
        if (t.scan_wgs == 1 && t.nchunks <= SCAN1_MAX * (int)blockDim.x) {
            // one scanning workgroup (small tables): counts stay in registers,
            // the chunk offsets are the final ones, and no range pass is needed
            const int K1 = (t.nchunks + (int)blockDim.x - 1) / (int)blockDim.x;
            const int c0 = (int)threadIdx.x * K1;
            unsigned cnt1[SCAN1_MAX];
            unsigned tsum = 0;
#pragma unroll
            for (int k = 0; k < SCAN1_MAX; k++) {
                const int c = c0 + k;
                unsigned cnt = 0;
                if (k < K1 && c < t.nchunks) {
                    const ulonglong2* bw = (const ulonglong2*)(t.bitmap + (long long)c * CHUNK_WORDS);
#pragma unroll
                    for (int j = 0; j < CHUNK_WORDS / 2; j++) {
                        const ulonglong2 v = bw[j];
                        cnt += (unsigned)__popcll(v.x) + (unsigned)__popcll(v.y);
                    }
                }
                cnt1[k] = cnt;
                tsum += cnt;
                const int q = wave_append(&st->n_ne, cnt > 0u);
                if (q >= 0) t.ne_chunks[q] = c;
            }
            unsigned incl = tsum;
            for (int o = 1; o < 64; o <<= 1) {
                const unsigned u = __shfl_up(incl, o);
                if (lane >= o) incl += u;
            }
            if (lane == 63) red[wid] = incl;
            __syncthreads();
            unsigned run = incl - tsum, total = 0;
            for (int w = 0; w < nw; w++) {
                if (w < wid) run += red[w];
                total += red[w];
            }
#pragma unroll
            for (int k = 0; k < SCAN1_MAX; k++) {
                const int c = c0 + k;
                if (k < K1 && c < t.nchunks) t.partial[c] = run;
                run += cnt1[k];
            }
            if (threadIdx.x == 0) {
                t.wg_total[0] = 0u;            // offsets are global: one range
                commit_step(t, st, nn, nr, nfree, total);
            }
            break;
        }
        const int C = t.chunks_per_wg;
        const long long c0 = (long long)blockIdx.x * C;
        const long long c1 = min((long long)t.nchunks, c0 + C);
        const int K = (C + (int)blockDim.x - 1) / (int)blockDim.x;
        const long long tc0 = c0 + (long long)threadIdx.x * K;
        unsigned tsum = 0;
        for (int k = 0; k < K; k++) {                // K is uniform: every lane runs the ballots
            const long long c = tc0 + k;
            unsigned cnt = 0;
            if (c < c1) {
                const ulonglong2* bw = (const ulonglong2*)(t.bitmap + c * CHUNK_WORDS);
#pragma unroll
                for (int j = 0; j < CHUNK_WORDS / 2; j++) {
                    const ulonglong2 v = bw[j];
                    cnt += (unsigned)__popcll(v.x) + (unsigned)__popcll(v.y);
                }
                t.partial[c] = cnt;
                tsum += cnt;
            }
            // the compaction visits only the chunks listed here
            const int q = wave_append(&st->n_ne, cnt > 0u);
            if (q >= 0) t.ne_chunks[q] = (int)c;
        }
        unsigned incl = tsum;
        for (int o = 1; o < 64; o <<= 1) {
            const unsigned u = __shfl_up(incl, o);
            if (lane >= o) incl += u;
        }
        if (lane == 63) red[wid] = incl;
        __syncthreads();
        unsigned run = incl - tsum, wg_sum = 0;
        for (int w = 0; w < nw; w++) {
            if (w < wid) run += red[w];
            wg_sum += red[w];
        }
        for (int k = 0; k < K; k++) {
            const long long c = tc0 + k;
            if (c >= c1) break;
            const unsigned v = t.partial[c];
            t.partial[c] = run;
            run += v;
        }
        if (threadIdx.x == 0) {
            t.wg_total[blockIdx.x] = wg_sum;
            // arrival and range total in one atomic: the last scanning
            // workgroup reads the list's length from its own return value, so
            // no workgroup needs a device-scope release (an L2 write-back per
            // workgroup on gfx950); the compaction scans the range totals
            const unsigned long long old = atomicAdd(&st->scan_acc, (1ull << 32) | (unsigned long long)wg_sum);
            if ((int)(old >> 32) == t.scan_wgs - 1) {
                st->scan_acc = 0ull;
                commit_step(t, st, nn, nr, nfree, (unsigned)old + wg_sum);
            }
        }
    } while (false);
}

hipError_t launch_pool_count(const Tables& t, int grid, hipStream_t s) {
    if (t.scan_wgs < 1 || t.scan_wgs > POOL_COUNT_MAX_WG || grid < t.scan_wgs ||
        (long long)t.scan_wgs * t.chunks_per_wg < t.nchunks)
        return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_pool_count, dim3(grid), dim3(256), 0, s, t);
    return hipGetLastError();
}

// --------------------------------------------------------------------------
// Compaction of the bitmap into the next active list
// --------------------------------------------------------------------------

// Workgroups of 16 waves take the chunks with a set bit (listed by the
// allocator's scan; all chunks when the grid covers them) in turn.  Every wave loads the chunk (lane = word) and
// forms the exclusive prefix of the word popcounts; wave v then emits word v
// with lane = bit, so each word's blocks are written as one contiguous run in
// key order.
constexpr int EMIT_WAVES = CHUNK_WORDS;
__global__ __launch_bounds__(64 * EMIT_WAVES) void k_emit(Tables t) {
    DevState* st = t.st;
    __shared__ unsigned long long csum[EMIT_WAVES], usum[EMIT_WAVES], lsum[EMIT_WAVES];
    __shared__ unsigned s_rng[POOL_COUNT_MAX_WG], s_wsum[EMIT_WAVES];
    static_assert(POOL_COUNT_MAX_WG <= 64 * EMIT_WAVES, "one range total per thread");
    const int lane = lane_id();
    const int wid = threadIdx.x >> 6;
    const int emit = st->emit;
    {
        // offsets of the allocator's chunk ranges: exclusive scan of their totals
        const int g = threadIdx.x;
        const unsigned v = g < t.scan_wgs ? t.wg_total[g] : 0u;
        unsigned incl = v;
        for (int o = 1; o < 64; o <<= 1) {
            const unsigned u = __shfl_up(incl, o);
            if (lane >= o) incl += u;
        }
        if (lane == 63) s_wsum[wid] = incl;
        __syncthreads();
        unsigned off = 0;
        for (int w = 0; w < wid; w++) off += s_wsum[w];
        if (g < t.scan_wgs) s_rng[g] = off + incl - v;
        __syncthreads();
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        // the allocator has finished: its free count and cleared step counters
        st->free_cnt = st->free_next;
        st->n_new = 0;
        st->n_ret = 0;
        st->n_dec = 0;
    }
    // a grid that covers every chunk takes them directly (empty ones cost a
    // load); otherwise it walks the list of non-empty chunks
    const bool direct = t.nchunks <= (int)gridDim.x;
    const int nq = direct ? t.nchunks : st->n_ne;
    unsigned long long cells = 0, ucells = 0, lcells = 0;
    for (int q = blockIdx.x; q < nq; q += gridDim.x) {      // uniform over the workgroup
        const long long chunk = direct ? q : t.ne_chunks[q];
        const long long w_lane = chunk * CHUNK_WORDS + lane;
        const bool word_lane = lane < CHUNK_WORDS && w_lane < t.nwords;
        const unsigned long long myword = word_lane ? t.bitmap[w_lane] : 0ull;
        const unsigned cnt = (unsigned)__popcll(myword);
        unsigned incl = cnt;
        for (int o = 1; o < 64; o <<= 1) {
            const unsigned u = __shfl_up(incl, o);
            if (lane >= o) incl += u;
        }
        const unsigned base = emit ? s_rng[chunk / t.chunks_per_wg] + t.partial[chunk] : 0u;
        const int j = wid;                      // the wave's own word
        do {
            const unsigned long long m = __shfl(myword, j);
            if (m == 0ull) break;
            const long long w = chunk * CHUNK_WORDS + j;
            const bool mine = (m >> lane) & 1ull;
            const long long G = w * 64 + lane;
            if (!emit) {
                // the step failed: undo its claims, keep the current list
                if (mine && t.cell2box[G] == CLAIMED) t.cell2box[G] = EMPTY;
                break;
            }
            const unsigned off = base + __shfl(incl - cnt, j) +
                                 (unsigned)__popcll(m & ((1ull << lane) - 1ull));
            const int shot = shot_of_word(t, w);
            const Shot& S = t.shots[shot];
            if (mine) {
                const unsigned key = (unsigned)(G - S.key_base);
                const int slot = t.cell2box[G];
                t.act_slot[off] = slot;
                t.act_shot[off] = shot;
                t.act_key[off] = key;
                int bx, by, bz;
                key_to_block(S, key, bx, by, bz);
                const unsigned long long bc = (unsigned long long)block_cells(S, bx, by, bz);
                cells += bc;
                const float u = t.slot_c2u[slot];
                if (u == u) ucells += bc;
                if (__float_as_uint(u) == LAT_C2_BITS) lcells += bc;
                long long nk[6];
                int nb[6];
#pragma unroll
                for (int d = 0; d < 6; d++) nk[d] = neighbour_key(S, bx, by, bz, d);
#pragma unroll
                for (int d = 0; d < 6; d++) nb[d] = t.cell2box[nk[d] >= 0 ? nk[d] : G];   // all loads at once
#pragma unroll
                for (int d = 0; d < 6; d++) if (nk[d] < 0) nb[d] = EMPTY;
                int4* rp = (int4*)(t.rows + 8 * (size_t)off);
                rp[0] = make_int4(slot, nb[0], nb[1], nb[2]);
                rp[1] = make_int4(nb[3], nb[4], nb[5], row_key_field(t, slot, G));
            }
        } while (false);
        __syncthreads();                       // every wave has read the chunk
        if (wid == 0 && word_lane && myword) t.bitmap[w_lane] = 0ull;
    }
    for (int o = 32; o > 0; o >>= 1) {
        cells += __shfl_xor(cells, o);
        ucells += __shfl_xor(ucells, o);
        lcells += __shfl_xor(lcells, o);
    }
    if (lane == 0) {
        csum[wid] = cells;
        usum[wid] = ucells;
        lsum[wid] = lcells;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long c = 0, u = 0, l = 0;
        for (int w = 0; w < EMIT_WAVES; w++) {
            c += csum[w];
            u += usum[w];
            l += lsum[w];
        }
        if (c) atomicAdd(&st->cells_cur, c);
        if (u) atomicAdd(&st->cells_cur_u, u);
        if (l) atomicAdd(&st->cells_cur_l, l);
    }
}

hipError_t launch_emit(const Tables& t, int grid, hipStream_t s) {
    hipLaunchKernelGGL(k_emit, dim3(grid), dim3(64 * EMIT_WAVES), 0, s, t);
    return hipGetLastError();
}

// --------------------------------------------------------------------------
// Activation update in two launches (constant levels, update every step, no
// shutdown, one pool slot per block key, so that a block's slot is its key).
// The active set of step n is the bitmap act(n) = (n & 1 ? bitmap2 : bitmap).
//
// k_fast_plan: one 64-lane wave per bitmap word (lane = key), FAST_WORDS
//   words per workgroup (a "fast chunk").  Each key pulls its decision from
//   the stencil's flag bytes: an active block stays if its keep bit is set
//   (the stencil also sets it while the block's source pin holds); any block
//   is in the next set if an active face neighbour's face toward it is above
//   the trigger ("Updating active cells", items 3 and 4).  The workgroup
//   writes every one of its words of the next set (the other bitmap, so
//   neither bitmap is ever cleared), releases and allocates (zero levels, C2
//   from the media) its own blocks, and stores its counts; no two workgroups
//   touch the same word, so nothing waits on another workgroup (beyond
//   FAST_DIRECT_CHUNKS chunks the counts of each run of FAST_BLK chunks are
//   also summed with device atomics).
// k_fast_emit: each workgroup sums the counts of the fast chunks before its
//   own (its offset in the next list) and of all (the list's length), then
//   compacts its words into the list and its rows in key order; workgroup 0
//   commits the step.
// --------------------------------------------------------------------------
__device__ __forceinline__ unsigned long long* fast_bm(const Tables& t, int par) {
    return par ? t.bitmap2 : t.bitmap;
}

// A run's block, activation and release counts in one word, 21 bits each
// (a run holds at most FAST_BLK * 256 keys); its in-domain node counts in
// another, 32 bits each (at most FAST_BLK * 256 * 512 nodes).
constexpr unsigned long long FAST_FIELD = (1ull << 21) - 1ull;
constexpr int FAST_SUM_BATCH = 4;
static_assert(FAST_BLK <= 64 * FAST_WORDS, "a run's chunk counts take one load per thread");
static_assert(FAST_BLK * 64 * FAST_WORDS < (1 << 21) && FAST_BLK * 64 * FAST_WORDS * 512ll < (1ll << 32),
              "run sums fit their fields");
__device__ __forceinline__ unsigned long long fast_pack3(unsigned a, unsigned b, unsigned c) {
    return (unsigned long long)a | ((unsigned long long)b << 21) | ((unsigned long long)c << 42);
}

// ONE: a single-shot handle (every word belongs to shot 0: no shot lookup)
template <bool ONE>
__global__ __launch_bounds__(64 * FAST_WORDS) void k_fast_plan(Tables t) {
    DevState* st = t.st;
    __shared__ int s_new[64 * FAST_WORDS];
    __shared__ int s_nnew, s_nret;
    __shared__ unsigned s_cnt[FAST_WORDS];
    __shared__ unsigned long long s_cells[FAST_WORDS], s_cellsu[FAST_WORDS], s_cellsl[FAST_WORDS];
    // the state's fields and a single shot's record in one round of loads
    // (each dependent round is a memory latency of this short kernel)
    const int n = st->step, err = st->error, nfs = st->nf_step;
    Shot S1;
    if (ONE) S1 = t.shots[0];
    // (no short-circuit: it would let the compiler load nf_step after error)
    if ((err != 0) | ((nfs != 0) & (nfs != n + 1))) return;     // halted before this step
    const int p = n & 1;
    const unsigned long long* cur = fast_bm(t, p);
    unsigned long long* nxt = fast_bm(t, 1 - p);
    const bool failed = nfs != 0;             // this step wrote a non-finite value
    const int lane = lane_id();
    const int wid = threadIdx.x >> 6;
    if (blockIdx.x == 0 && threadIdx.x == 0) st->fast_par = 1 - p;   // read by k_fast_emit
    // receivers: traces[n - trace_step0][r] = phi^{n+1} (slot = key)
    const int row = n - t.trace_step0;
    if (blockIdx.x == 0 && row >= 0 && row < t.trace_cap) {
        for (int r = threadIdx.x; r < t.nrec; r += blockDim.x) {
            const Rec e = t.rec[r];
            const bool on = (cur[e.key >> 6] >> (e.key & 63)) & 1ull;
            t.traces[(size_t)row * t.nrec + r] = on ? plane_of(t, e.key, 1 - p)[e.local] : 0.f;
        }
    }
    if (failed) {
        // the step keeps its list: the next set is the current one (the
        // emit only advances the step)
        for (int c = blockIdx.x; c < t.nfchunks; c += gridDim.x) {
            const long long w = (long long)c * FAST_WORDS + wid;
            if (lane == 0 && w < t.nwords) nxt[w] = cur[w];
        }
        return;
    }
    const float trig = t.trigger;
    (void)trig;
    for (int c = blockIdx.x; c < t.nfchunks; c += gridDim.x) {       // uniform over the workgroup
        if (threadIdx.x == 0) { s_nnew = 0; s_nret = 0; }
        __syncthreads();
        const long long w = (long long)c * FAST_WORDS + wid;
        const long long G = w * 64 + lane;
        const bool in_range = w < t.nwords;
        Shot S;
        if constexpr (ONE) S = S1;
        else S = t.shots[in_range ? shot_of_word(t, w) : 0];
        // (keys outside a shot's domain are never active: their word bits
        // are only loaded for keys inside it)
        bool active = false, survive = false, in_dom = false;
        float c2u = 0.f;
        int bx = 0, by = 0, bz = 0;
        if (in_range) {
            key_to_block(S, (unsigned)(G - S.key_base), bx, by, bz);
            in_dom = bx < S.bx && by < S.by && bz < S.bz;
            if (in_dom) {
                // the neighbours' keys first, then every load of the decision
                // at once (the key's word, flags and scalar C2, each
                // neighbour's word and flags), then decide; a source pin is
                // in the key's keep flag (the stencil folds it in)
                long long nk[6], kk[6];
#pragma unroll
                for (int d = 0; d < 6; d++) {
                    nk[d] = neighbour_key(S, bx, by, bz, d);
                    kk[d] = nk[d] >= 0 ? nk[d] : G;
                }
                const unsigned long long curw = cur[w];
                const unsigned own = t.flags[G];
                c2u = t.slot_c2u[G];
                unsigned long long nwd[6];
                unsigned nfl[6];
                // (a missing neighbour loads the key's own entries, ignored
                // below: conditional loads compile to branches that wait
                // after each load)
#pragma unroll
                for (int d = 0; d < 6; d++) {
                    nwd[d] = cur[kk[d] >> 6];
                    nfl[d] = t.flags[kk[d]];
                }
                active = (curw >> lane) & 1ull;
                survive = active && (own & KEEP_BIT) != 0;
                // (bitwise, not short-circuit: a load that only one branch
                // uses is moved into that branch and waited for there)
#pragma unroll
                for (int d = 0; d < 6; d++)
                    survive |= (nk[d] >= 0) & (((nwd[d] >> (nk[d] & 63)) & 1ull) != 0) &
                               (((nfl[d] >> (d ^ 1)) & 1u) != 0);
            }
        }
        const unsigned long long nw = __ballot(survive);
        if (lane == 0) {
            nxt[w] = nw;
            s_cnt[wid] = (unsigned)__popcll(nw);
        }
        if (active && !survive) {                        // released ("Updating active cells", item 7)
            t.cell2box[G] = EMPTY;
            t.slot_key[G] = -1;
            atomicAdd(&s_nret, 1);
        }
        if (survive && !active) s_new[atomicAdd(&s_nnew, 1)] = (int)(G - (long long)c * FAST_WORDS * 64);
        __syncthreads();
        // new blocks, one wave each: zero levels, C2 from the media (item 8)
        const int nnew = s_nnew;
        for (int k = wid; k < nnew; k += FAST_WORDS) {
            const long long G2 = (long long)c * FAST_WORDS * 64 + s_new[k];
            if (t.c2_ready) {
                // the C2 plane and scalar were filled when the pool was made:
                // only stores, nothing for the loop to wait on
                zero_levels(t, G2);
            } else {
                const int sh = shot_of_word(t, G2 >> 6);
                const Shot& S = t.shots[sh];
                int x2, y2, z2;
                key_to_block(S, (unsigned)(G2 - S.key_base), x2, y2, z2);
                const float c2u = fill_slot(t, S, G2, x2, y2, z2);
                if (lane == 0) t.slot_c2u[G2] = c2u;
            }
            if (lane == 0) {
                t.sdlog[G2] = 0;
                t.cell2box[G2] = (int)G2;
                t.slot_key[G2] = G2;
                t.pin_until[2 * (size_t)(G2)] = 0;
                t.pin_until[2 * (size_t)(G2) + 1] = -1;
            }
        }
        __syncthreads();
        // in-domain nodes of the next set (and of its blocks with a scalar C2;
        // a new block's scalar C2 is the one filling it left in slot_c2u)
        unsigned long long bc = 0, bu = 0, bl = 0;
        if (survive) {
            bc = (unsigned long long)block_cells(S, bx, by, bz);
            const float u = active || t.c2_ready ? c2u : t.slot_c2u[G];
            if (u == u) bu = bc;
            if (__float_as_uint(u) == LAT_C2_BITS) bl = bc;
        }
        for (int o = 32; o > 0; o >>= 1) {
            bc += __shfl_xor(bc, o);
            bu += __shfl_xor(bu, o);
            bl += __shfl_xor(bl, o);
        }
        if (lane == 0) {
            s_cells[wid] = bc;
            s_cellsu[wid] = bu;
            s_cellsl[wid] = bl;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            unsigned cnt = 0;
            unsigned long long cc = 0, cu = 0, cl = 0;
            for (int k = 0; k < FAST_WORDS; k++) {
                cnt += s_cnt[k];
                cc += s_cells[k];
                cu += s_cellsu[k];
                cl += s_cellsl[k];
            }
            t.fc_cnt[c] = (int)cnt;
            if (t.nfblk) {
                // the run's sums, three packed words (this step's parity; the
                // compaction clears the other parity's for the next step)
                unsigned long long* b = t.fc_blk + ((size_t)p * t.nfblk + (size_t)(c / FAST_BLK)) * 3;
                const unsigned long long k3 = fast_pack3(cnt, (unsigned)s_nnew, (unsigned)s_nret);
                const unsigned long long k2 = cc | (cu << 32);
                if (k3) atomicAdd(&b[0], k3);
                if (k2) atomicAdd(&b[1], k2);
                if (cl) atomicAdd(&b[2], cl);
            } else {
                t.fc_new[c] = s_nnew;
                t.fc_ret[c] = s_nret;
                t.fc_cells[3 * (size_t)c] = cc;
                t.fc_cells[3 * (size_t)c + 1] = cu;
                t.fc_cells[3 * (size_t)c + 2] = cl;
            }
        }
        __syncthreads();                                   // LDS is reused by the next chunk
    }
}

template <bool ONE>
__global__ __launch_bounds__(64 * FAST_WORDS) void k_fast_emit(Tables t) {
    DevState* st = t.st;
    __shared__ unsigned long long s_red[FAST_WORDS][7];
    __shared__ unsigned s_word[FAST_WORDS];
    // the state's fields and a single shot's record in one round of loads
    const int err = st->error, nfs = st->nf_step, par = st->fast_par;
    Shot S1;
    if (ONE) S1 = t.shots[0];
    if ((err | nfs) != 0) {
        // the step that wrote a non-finite value completes (its phi^{n+1} is
        // kept) with the same list; thread 0 of workgroup 0 is the only
        // reader and writer of the step counter in this launch
        if (blockIdx.x == 0 && threadIdx.x == 0 && !err && nfs == st->step + 1) {
            st->updates += st->cells_cur;
            st->updates_u += st->cells_cur_u;
            st->updates_l += st->cells_cur_l;
            st->step += 1;
        }
        return;
    }
    // the plan wrote every word of the next set (so neither bitmap is ever
    // cleared: the current one becomes the plan's output two steps on)
    const unsigned long long* nxt = fast_bm(t, par);
    const int lane = lane_id();
    const int wid = threadIdx.x >> 6;
    const int nf = t.nfchunks;
    // the plan summed the runs into parity 1 - par; the next step's plan sums
    // into parity par, cleared here (nothing in this launch reads it)
    const unsigned long long* blk = t.fc_blk + (size_t)(1 - par) * t.nfblk * 3;
    if (t.nfblk) {
        unsigned long long* clr = t.fc_blk + (size_t)par * t.nfblk * 3;
        const long long gs = (long long)gridDim.x * blockDim.x;
        for (long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x; k < 3ll * t.nfblk; k += gs) clr[k] = 0ull;
    }
    for (int c = blockIdx.x; c < nf; c += gridDim.x) {          // uniform over the workgroup
        // this wave's word and its shot first: their loads overlap the sums below
        const long long w = (long long)c * FAST_WORDS + wid;
        const bool in_range = w < t.nwords;
        const unsigned long long myw = in_range ? nxt[w] : 0ull;
        int shot = 0;
        Shot S;
        if constexpr (ONE) {
            S = S1;
        } else {
            shot = in_range ? shot_of_word(t, w) : 0;
            S = t.shots[shot];
        }
        // offset of this fast chunk in the next list: the sums of the runs
        // before its own, then the counts of its run's chunks before it (or,
        // with up to FAST_DIRECT_CHUNKS chunks, the counts of all chunks
        // before it); the workgroup of chunk 0 also sums the list's length
        // and the step's statistics
        // before, total, cells, scalar-C2 cells, new, released, lattice-record cells
        unsigned long long sums[7] = {0, 0, 0, 0, 0, 0, 0};
        // (the direct sums take FAST_SUM_BATCH strided entries per thread at a
        // time, so that their loads are in flight together: 6.8 against 7.2
        // us per launch at 512^3; the same for the run sums cost 4.6 us per
        // launch on the 64-shot batch)
        const int bd = blockDim.x;
        if (!t.nfblk) {
            if (c == 0) {
                for (int k0 = threadIdx.x; k0 < nf; k0 += FAST_SUM_BATCH * bd) {
                    int n1[FAST_SUM_BATCH], n4[FAST_SUM_BATCH], n5[FAST_SUM_BATCH];
                    unsigned long long n2[FAST_SUM_BATCH], n3[FAST_SUM_BATCH], n6[FAST_SUM_BATCH];
#pragma unroll
                    for (int u = 0; u < FAST_SUM_BATCH; u++) {
                        const int k = k0 + u * bd;
                        const bool in = k < nf;
                        n1[u] = in ? t.fc_cnt[k] : 0;
                        n2[u] = in ? t.fc_cells[3 * (size_t)k] : 0ull;
                        n3[u] = in ? t.fc_cells[3 * (size_t)k + 1] : 0ull;
                        n6[u] = in ? t.fc_cells[3 * (size_t)k + 2] : 0ull;
                        n4[u] = in ? t.fc_new[k] : 0;
                        n5[u] = in ? t.fc_ret[k] : 0;
                    }
#pragma unroll
                    for (int u = 0; u < FAST_SUM_BATCH; u++) {
                        sums[1] += (unsigned)n1[u];
                        sums[2] += n2[u];
                        sums[3] += n3[u];
                        sums[4] += (unsigned)n4[u];
                        sums[5] += (unsigned)n5[u];
                        sums[6] += n6[u];
                    }
                }
                for (int o = 32; o > 0; o >>= 1) {
#pragma unroll
                    for (int q = 1; q < 7; q++) sums[q] += __shfl_xor(sums[q], o);
                }
            } else {
                for (int k0 = threadIdx.x; k0 < c; k0 += FAST_SUM_BATCH * bd) {
                    int n1[FAST_SUM_BATCH];
#pragma unroll
                    for (int u = 0; u < FAST_SUM_BATCH; u++) n1[u] = k0 + u * bd < c ? t.fc_cnt[k0 + u * bd] : 0;
#pragma unroll
                    for (int u = 0; u < FAST_SUM_BATCH; u++) sums[0] += (unsigned)n1[u];
                }
                for (int o = 32; o > 0; o >>= 1) sums[0] += __shfl_xor(sums[0], o);
            }
        } else if (c == 0) {
            for (int k = threadIdx.x; k < t.nfblk; k += bd) {
                const unsigned long long k3 = blk[3 * (size_t)k], k2 = blk[3 * (size_t)k + 1];
                sums[1] += k3 & FAST_FIELD;
                sums[2] += k2 & 0xffffffffull;
                sums[3] += k2 >> 32;
                sums[4] += (k3 >> 21) & FAST_FIELD;
                sums[5] += k3 >> 42;
                sums[6] += blk[3 * (size_t)k + 2];
            }
            for (int o = 32; o > 0; o >>= 1) {
#pragma unroll
                for (int q = 1; q < 7; q++) sums[q] += __shfl_xor(sums[q], o);
            }
        } else {
            const int cb = c / FAST_BLK;
            for (int k = threadIdx.x; k < cb; k += bd) sums[0] += blk[3 * (size_t)k] & FAST_FIELD;
            const int k = cb * FAST_BLK + (int)threadIdx.x;        // FAST_BLK <= blockDim.x
            if (k < c) sums[0] += (unsigned)t.fc_cnt[k];
            for (int o = 32; o > 0; o >>= 1) sums[0] += __shfl_xor(sums[0], o);
        }
        if (lane == 0) {
#pragma unroll
            for (int q = 0; q < 7; q++) s_red[wid][q] = sums[q];
        }
        if (lane == 0) s_word[wid] = (unsigned)__popcll(myw);
        // the rows' neighbour bits, loaded before the barrier so that they
        // overlap the sums
        const bool mine = (myw >> lane) & 1ull;
        const long long G = w * 64 + lane;
        const unsigned key = (unsigned)(G - S.key_base);
        int nb[6] = {EMPTY, EMPTY, EMPTY, EMPTY, EMPTY, EMPTY};
        int bx = 0, by = 0, bz = 0, kf = 0;
        if (mine) {
            kf = row_key_field(t, G, G);
            key_to_block(S, key, bx, by, bz);
            long long nk[6];
            unsigned long long nw[6];
#pragma unroll
            for (int d = 0; d < 6; d++) nk[d] = neighbour_key(S, bx, by, bz, d);
#pragma unroll
            for (int d = 0; d < 6; d++) nw[d] = nxt[(nk[d] >= 0 ? nk[d] : G) >> 6];   // all loads at once
#pragma unroll
            for (int d = 0; d < 6; d++) nb[d] = (nk[d] >= 0 && ((nw[d] >> (nk[d] & 63)) & 1ull)) ? (int)nk[d] : EMPTY;
        }
        __syncthreads();
        unsigned long long base = 0, ntot = 0;
        for (int k = 0; k < FAST_WORDS; k++) {
            base += s_red[k][0];
            ntot += s_red[k][1];
        }
        unsigned long long cc = 0, cu = 0, na = 0, nr = 0, cl = 0;
        for (int k = 0; k < FAST_WORDS; k++) {
            cc += s_red[k][2];
            cu += s_red[k][3];
            na += s_red[k][4];
            nr += s_red[k][5];
            cl += s_red[k][6];
        }
        for (int k = 0; k < wid; k++) base += s_word[k];
        if (mine) {
            const unsigned off = (unsigned)(base + (unsigned long long)__popcll(myw & ((1ull << lane) - 1ull)));
            t.act_slot[off] = (int)G;
            t.act_shot[off] = shot;
            t.act_key[off] = key;
            int4* rp = (int4*)(t.rows + 8 * (size_t)off);
            rp[0] = make_int4((int)G, nb[0], nb[1], nb[2]);
            rp[1] = make_int4(nb[3], nb[4], nb[5], kf);
        }
        // commit (workgroup 0, once): no other workgroup of this launch reads
        // the fields it changes
        if (c == 0 && threadIdx.x == 0) {
            st->updates += st->cells_cur;
            st->updates_u += st->cells_cur_u;
            st->updates_l += st->cells_cur_l;
            st->cells_cur = cc;
            st->cells_cur_u = cu;
            st->cells_cur_l = cl;
            st->activations += na;
            st->retirements += nr;
            st->n_act = (int)ntot;
            if ((int)ntot > st->peak_act) st->peak_act = (int)ntot;
            st->free_cnt = t.cap - (int)ntot;
            st->free_next = st->free_cnt;
            st->step += 1;
            st->maxbits = 0u;
        }
        __syncthreads();                                   // LDS is reused by the next chunk
    }
}

hipError_t launch_fast_update(const Tables& t, int grid, hipStream_t s) {
    if (!t.fast || t.nfchunks > FAST_MAX_CHUNKS) return hipErrorInvalidValue;
    if (t.nshots == 1) {
        hipLaunchKernelGGL(k_fast_plan<true>, dim3(grid), dim3(64 * FAST_WORDS), 0, s, t);
    } else {
        hipLaunchKernelGGL(k_fast_plan<false>, dim3(grid), dim3(64 * FAST_WORDS), 0, s, t);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (t.nshots == 1) {
        hipLaunchKernelGGL(k_fast_emit<true>, dim3(grid), dim3(64 * FAST_WORDS), 0, s, t);
    } else {
        hipLaunchKernelGGL(k_fast_emit<false>, dim3(grid), dim3(64 * FAST_WORDS), 0, s, t);
    }
    return hipGetLastError();
}

// --------------------------------------------------------------------------
// Table invariants between two steps (tcm_check): the active list, the
// block table (Table 1 Cell2box), the slots' keys (Box2cell) and the
// current-set bitmap of the two-launch update agree; every listed slot is
// listed once; every neighbour slot in a row is that neighbour's slot.
// Violations are counted in bad[0]; bad[1] counts keys with a slot.
// --------------------------------------------------------------------------
__global__ void k_check_list(Tables t, int* mark, unsigned long long* bad) {
    const DevState* st = t.st;
    const int nact = min(st->n_act, t.cap);     // a longer list is counted on the host
    const int p = st->step & 1;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < nact;
         i += (long long)gridDim.x * blockDim.x) {
        unsigned long long nbad = 0;
        const int s = t.act_slot[i];
        const int shot = t.act_shot[i];
        if (s < 0 || s >= t.cap || shot < 0 || shot >= t.nshots) {
            atomicAdd(bad, 1ull);
            continue;
        }
        const Shot& S = t.shots[shot];
        const long long G = S.key_base + (long long)t.act_key[i];
        if (G < 0 || G >= t.nkeys) {
            atomicAdd(bad, 1ull);
            continue;
        }
        atomicAdd(&mark[s], 1);
        nbad += t.cell2box[G] != s;
        nbad += t.slot_key[s] != G;
        nbad += t.rows[8 * (size_t)i] != s;
        nbad += row_key(t.rows[8 * (size_t)i + 7]) != (int)G;
        nbad += (t.rows[8 * (size_t)i + 7] < 0) != slot_has_pin_or_src(t, s);
        int bx, by, bz;
        key_to_block(S, t.act_key[i], bx, by, bz);
        nbad += !(bx < S.bx && by < S.by && bz < S.bz);
        for (int d = 0; d < 6; d++) {
            const long long nk = neighbour_key(S, bx, by, bz, d);
            nbad += t.rows[8 * (size_t)i + 1 + d] != (nk >= 0 ? t.cell2box[nk] : EMPTY);
        }
        if (t.fast) nbad += !((fast_bm(t, p)[G >> 6] >> (G & 63)) & 1ull);
        if (nbad) atomicAdd(bad, nbad);
    }
}

__global__ void k_check_keys(Tables t, const int* mark, unsigned long long* bad) {
    const int p = t.st->step & 1;
    for (long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x; k < t.nkeys;
         k += (long long)gridDim.x * blockDim.x) {
        const int c = t.cell2box[k];
        unsigned long long nbad = 0;
        if (c >= 0) {
            atomicAdd(&bad[1], 1ull);
            nbad += c >= t.cap || t.slot_key[c] != k || mark[c] != 1;
        } else {
            nbad += c != EMPTY;                  // no claim is left between steps
        }
        if (t.fast) nbad += ((fast_bm(t, p)[k >> 6] >> (k & 63)) & 1ull) != (unsigned long long)(c >= 0);
        if (nbad) atomicAdd(bad, nbad);
    }
}

__global__ void k_check_slots(Tables t, const int* mark, unsigned long long* bad) {
    for (long long s = (long long)blockIdx.x * blockDim.x + threadIdx.x; s < t.cap;
         s += (long long)gridDim.x * blockDim.x) {
        const long long k = t.slot_key[s];
        unsigned long long nbad = mark[s] > 1;
        if (k >= 0) nbad += k >= t.nkeys || t.cell2box[k] != (int)s;
        else nbad += k != -1 || mark[s] != 0;
        if (nbad) atomicAdd(bad, nbad);
    }
}

hipError_t launch_check(const Tables& t, int* mark, unsigned long long* bad, hipStream_t s) {
    hipLaunchKernelGGL(k_check_list, dim3(1024), dim3(256), 0, s, t, mark, bad);
    hipLaunchKernelGGL(k_check_keys, dim3(1024), dim3(256), 0, s, t, mark, bad);
    hipLaunchKernelGGL(k_check_slots, dim3(1024), dim3(256), 0, s, t, mark, bad);
    return hipGetLastError();
}

// --------------------------------------------------------------------------
// source activation: box the blocks of new sources by hand, one wave per
// block (distinct keys), appending them to the active list
// --------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_activate_list(Tables t, const long long* keys, const int* shots,
                                                       const unsigned* lkeys, const int* pins, const int* heads,
                                                       int n) {
    DevState* st = t.st;
    const int lane = lane_id();
    const int k = (int)((blockIdx.x * blockDim.x + threadIdx.x) >> 6);
    if (k >= n) return;                      // uniform over the wave
    const long long G = keys[k];
    const int pin = pins[k];
    const int head = heads[k];
    const int cur = t.cell2box[G];
    if (pin < 0) {                           // an earlier source block: refresh or clear its range
        if (cur >= 0 && lane == 0) {
            if (pin == -2) {
                t.pin_until[2 * (size_t)(cur)] = 0;
                t.pin_until[2 * (size_t)(cur) + 1] = -1;
            } else if (head >= 0) {
                t.pin_until[2 * (size_t)(cur) + 1] = head;
            }
        }
        return;
    }
    if (cur >= 0) {                          // active already: raise its pin
        if (lane == 0) {
            if (t.pin_until[2 * (size_t)(cur)] < pin) t.pin_until[2 * (size_t)(cur)] = pin;
            if (head >= 0) t.pin_until[2 * (size_t)(cur) + 1] = head;
        }
        return;
    }
    int ok = 1;
    if (lane == 0) {
        if (atomicSub(&st->free_cnt, 1) <= 0) {
            atomicAdd(&st->free_cnt, 1);
            st->add_error = -3;
            ok = 0;
        }
    }
    if (!__shfl(ok, 0)) return;
    const int slot = t.cap >= t.nkeys ? (int)G : place_slot(t, G);
    if (slot < 0) {                          // unreachable: a slot was reserved above
        if (lane == 0) st->add_error = -6;
        return;
    }
    const int shot = shots[k];
    const unsigned key = lkeys[k];
    const Shot& S = t.shots[shot];
    int bx, by, bz;
    key_to_block(S, key, bx, by, bz);
    const float c2u = fill_slot(t, S, slot, bx, by, bz);
    if (lane == 0) {
        t.slot_c2u[slot] = c2u;
        t.sdlog[slot] = 0;
        t.cell2box[G] = slot;
        t.slot_key[slot] = G;
        t.pin_until[2 * (size_t)(slot)] = pin;
        t.pin_until[2 * (size_t)(slot) + 1] = head;
        if (t.fast) atomicOr(&fast_bm(t, st->step & 1)[G >> 6], 1ull << (G & 63));
        const int i = atomicAdd(&st->n_act, 1);
        t.act_slot[i] = slot;
        t.act_shot[i] = shot;
        t.act_key[i] = key;
        atomicMax(&st->peak_act, i + 1);
        const unsigned long long bc = (unsigned long long)block_cells(S, bx, by, bz);
        atomicAdd(&st->cells_cur, bc);
        if (c2u == c2u) atomicAdd(&st->cells_cur_u, bc);
        if (__float_as_uint(c2u) == LAT_C2_BITS) atomicAdd(&st->cells_cur_l, bc);
        atomicAdd(&st->activations, 1ull);
    }
}

hipError_t launch_activate_list(const Tables& t, const long long* keys, const int* shots,
                                const unsigned* local_keys, const int* pins, const int* heads, int n,
                                hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_activate_list, dim3((unsigned)((n + 3) / 4)), dim3(256), 0, s, t, keys, shots,
                       local_keys, pins, heads, n);
    return hipGetLastError();
}

// Rewrite the neighbour row of every active entry from the block table
// (after blocks were activated outside the step sequence).
__global__ void k_refresh_rows(Tables t) {
    const int nact = t.st->n_act;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < nact; i += gridDim.x * blockDim.x) {
        const int shot = t.act_shot[i];
        const unsigned key = t.act_key[i];
        const Shot& S = t.shots[shot];
        int bx, by, bz;
        key_to_block(S, key, bx, by, bz);
        int nb[6];
        for (int d = 0; d < 6; d++) {
            const long long nk = neighbour_key(S, bx, by, bz, d);
            nb[d] = nk >= 0 ? t.cell2box[nk] : EMPTY;
        }
        int4* rp = (int4*)(t.rows + 8 * (size_t)i);
        rp[0] = make_int4(t.act_slot[i], nb[0], nb[1], nb[2]);
        rp[1] = make_int4(nb[3], nb[4], nb[5], row_key_field(t, t.act_slot[i], S.key_base + (long long)key));
    }
}

hipError_t launch_refresh_rows(const Tables& t, hipStream_t s) {
    hipLaunchKernelGGL(k_refresh_rows, dim3(256), dim3(256), 0, s, t);
    return hipGetLastError();
}


// --------------------------------------------------------------------------
// read: gather a box of phi^n / phi^{n-1} (inactive nodes -> 0)
// --------------------------------------------------------------------------
// One thread per node of a box row (x fastest); each thread takes RB rows at
// a time, issuing all their block-table loads, then all pool loads, then the
// stores, so the dependent loads of different rows overlap.  The output is
// written once and read much later (the adjoint's snapshots), so it is stored
// past the caches.
constexpr int READ_RB = 8;

__global__ void k_read(Tables t, int shot, int which, int x0, int y0, int z0, int sx, int sy,
                       int sz, float* __restrict__ out) {
    const int lx = blockIdx.x * blockDim.x + threadIdx.x;
    if (lx >= sx) return;
    const int plane = which == 0 ? (t.st->step & 1) : 1 - (t.st->step & 1);
    const Shot& S = t.shots[shot];
    const int gx = x0 + lx;
    const long long rows = (long long)sy * sz;
    for (long long r0 = (long long)blockIdx.y * READ_RB; r0 < rows; r0 += (long long)gridDim.y * READ_RB) {
        int slot[READ_RB], loc[READ_RB];
#pragma unroll
        for (int k = 0; k < READ_RB; k++) {
            slot[k] = EMPTY;
            loc[k] = 0;
            const long long row = r0 + k;
            if (row < rows) {
                const int gy = y0 + (int)(row % sy), gz = z0 + (int)(row / sy);
                slot[k] = t.cell2box[S.key_base + (long long)block_to_key(S, gx >> 3, gy >> 3, gz >> 3)];
                loc[k] = ((gz & 7) * 8 + (gy & 7)) * 8 + (gx & 7);
            }
        }
        float v[READ_RB];
#pragma unroll
        for (int k = 0; k < READ_RB; k++)
            v[k] = slot[k] >= 0 ? plane_of(t, slot[k], plane)[loc[k]] : 0.f;
#pragma unroll
        for (int k = 0; k < READ_RB; k++)
            if (r0 + k < rows) __builtin_nontemporal_store(v[k], &out[(size_t)(r0 + k) * sx + lx]);
    }
}

// The same with each thread taking two neighbouring nodes of a row (x0 and
// sx even, out 8-byte aligned): both lie in one block, so one 8-byte load
// from its plane and one 8-byte store.
typedef float read_f2 __attribute__((ext_vector_type(2)));

__global__ void k_read_pairs(Tables t, int shot, int which, int x0, int y0, int z0, int sx, int sy,
                             int sz, float* __restrict__ out) {
    const int lp = blockIdx.x * blockDim.x + threadIdx.x;
    if (2 * lp >= sx) return;
    const int plane = which == 0 ? (t.st->step & 1) : 1 - (t.st->step & 1);
    const Shot& S = t.shots[shot];
    const int gx = x0 + 2 * lp;
    const long long rows = (long long)sy * sz;
    for (long long r0 = (long long)blockIdx.y * READ_RB; r0 < rows; r0 += (long long)gridDim.y * READ_RB) {
        int slot[READ_RB], loc[READ_RB];
#pragma unroll
        for (int k = 0; k < READ_RB; k++) {
            slot[k] = EMPTY;
            loc[k] = 0;
            const long long row = r0 + k;
            if (row < rows) {
                const int gy = y0 + (int)(row % sy), gz = z0 + (int)(row / sy);
                slot[k] = t.cell2box[S.key_base + (long long)block_to_key(S, gx >> 3, gy >> 3, gz >> 3)];
                loc[k] = ((gz & 7) * 8 + (gy & 7)) * 8 + (gx & 7);
            }
        }
        read_f2 v[READ_RB];
#pragma unroll
        for (int k = 0; k < READ_RB; k++) {
            v[k] = read_f2{0.f, 0.f};
            if (slot[k] >= 0) v[k] = *(const read_f2*)(plane_of(t, slot[k], plane) + loc[k]);
        }
#pragma unroll
        for (int k = 0; k < READ_RB; k++)
            if (r0 + k < rows)
                __builtin_nontemporal_store(v[k], (read_f2*)&out[(size_t)(r0 + k) * sx + 2 * lp]);
    }
}

hipError_t launch_read(const Tables& t, int shot, int which, int x0, int y0, int z0, int sx, int sy,
                       int sz, float* out, hipStream_t s) {
    if (sx <= 0 || sy <= 0 || sz <= 0) return hipSuccess;
    if (x0 % 2 == 0 && sx % 2 == 0 && ((uintptr_t)out & 7u) == 0) {
        const long long groups = ((long long)sy * sz + READ_RB - 1) / READ_RB;
        dim3 grid((unsigned)((sx / 2 + 255) / 256), (unsigned)std::min<long long>(groups, 65535));
        hipLaunchKernelGGL(k_read_pairs, grid, dim3(256), 0, s, t, shot, which, x0, y0, z0, sx, sy, sz, out);
        return hipGetLastError();
    }
    const long long groups = ((long long)sy * sz + READ_RB - 1) / READ_RB;
    dim3 grid((unsigned)((sx + 255) / 256), (unsigned)std::min<long long>(groups, 65535));
    hipLaunchKernelGGL(k_read, grid, dim3(256), 0, s, t, shot, which, x0, y0, z0, sx, sy, sz, out);
    return hipGetLastError();
}

// --------------------------------------------------------------------------
// dense engine: eq.(3) on every node (the same arithmetic, no activation)
// --------------------------------------------------------------------------
__global__ void k_media_c2(const Shot* dshot, double dt, double dx, float* c2) {
    const Shot& S = *dshot;
    const long long total = (long long)S.nx * S.ny * S.nz;
    const long long gs = (long long)gridDim.x * blockDim.x;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += gs) {
        const int gx = (int)(i % S.nx);
        const long long r = i / S.nx;
        const int gy = (int)(r % S.ny), gz = (int)(r / S.ny);
        c2[i] = coeff_c2(media_speed(S, gx, gy, gz), dt, dx);
    }
}

hipError_t launch_media_c2(const Shot& shot, const Shot* dshot, double dt, double dx, float* c2,
                           hipStream_t s) {
    const long long total = (long long)shot.nx * shot.ny * shot.nz;
    long long grid = (total + 255) / 256;
    if (grid > 65536) grid = 65536;
    if (grid < 1) grid = 1;
    hipLaunchKernelGGL(k_media_c2, dim3((unsigned)grid), dim3(256), 0, s, dshot, dt, dx, c2);
    return hipGetLastError();
}

// 2.5-D z-marching: a 128 x 4 workgroup owns an (x, y) tile and walks DZ
// planes, keeping z-1, z, z+1 of its column in registers; x/y neighbours come
// through the L1/L2 caches.
constexpr int DENSE_TX = 128, DENSE_TY = 4, DENSE_DZ = 32;   // fastest of a measured sweep

__global__ __launch_bounds__(DENSE_TX * DENSE_TY) void k_dense_step(DenseArgs a) {
    const int x = blockIdx.x * DENSE_TX + (int)(threadIdx.x % DENSE_TX);
    const int y = blockIdx.y * DENSE_TY + (int)(threadIdx.x / DENSE_TX);
    const int z0 = blockIdx.z * DENSE_DZ;
    if (x >= a.nx || y >= a.ny) return;
    const size_t sy = (size_t)a.nx, sz = (size_t)a.nx * a.ny;
    const int z1 = min(a.nz, z0 + DENSE_DZ);
    size_t i = (size_t)z0 * sz + (size_t)y * sy + (size_t)x;
    float zm = z0 > 0 ? a.cur[i - sz] : 0.f;
    float c = a.cur[i];
    for (int z = z0; z < z1; z++, i += sz) {
        const float zp = z + 1 < a.nz ? a.cur[i + sz] : 0.f;
        const float xm = x > 0 ? a.cur[i - 1] : 0.f;
        const float xp = x + 1 < a.nx ? a.cur[i + 1] : 0.f;
        const float ym = y > 0 ? a.cur[i - sy] : 0.f;
        const float yp = y + 1 < a.ny ? a.cur[i + sy] : 0.f;
        const float s = ((xp + xm) + (yp + ym)) + (zp + zm);
        const float lap = s - 6.0f * c;
        // phi^{n-1}, C2 and phi^{n+1} are touched once per step: streamed past
        // L2, which keeps the phi^n planes the neighbouring columns re-read
        const float prev = __builtin_nontemporal_load(&a.nxt[i]);
        const float k2 = __builtin_nontemporal_load(&a.c2[i]);
        __builtin_nontemporal_store((2.0f * c - prev) + k2 * lap, &a.nxt[i]);
        zm = c;
        c = zp;
    }
}

hipError_t launch_dense_step(const DenseArgs& a, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
    dim3 grid((a.nx + DENSE_TX - 1) / DENSE_TX, (a.ny + DENSE_TY - 1) / DENSE_TY,
              (a.nz + DENSE_DZ - 1) / DENSE_DZ);
    if (e0 || e1)
        hipExtLaunchKernelGGL(k_dense_step, grid, dim3(DENSE_TX * DENSE_TY), 0, s, e0, e1, 0, a);
    else
        hipLaunchKernelGGL(k_dense_step, grid, dim3(DENSE_TX * DENSE_TY), 0, s, a);
    return hipGetLastError();
}

// sources (in table order) then receivers, single thread: a handful of nodes.
// Src::key / Rec::key hold linear node indices here.
__global__ void k_dense_inject(float* nxt, int n, const Src* src, int nsrc, const float* srcw,
                               const Rec* rec, int nrec, float* traces, int trace_row) {
    if (threadIdx.x != 0) return;
    for (int s = 0; s < nsrc; s++) {
        const int k = n - src[s].t0;
        if (k >= 0 && k < src[s].ns) nxt[src[s].key] = nxt[src[s].key] + srcw[src[s].w_off + k];
    }
    if (trace_row >= 0)
        for (int r = 0; r < nrec; r++) traces[(size_t)trace_row * nrec + r] = nxt[rec[r].key];
}

hipError_t launch_dense_inject(float* nxt, int n, const Src* src, int nsrc, const float* srcw,
                               const Rec* rec, int nrec, float* traces, int trace_row,
                               hipStream_t s) {
    hipLaunchKernelGGL(k_dense_inject, dim3(1), dim3(64), 0, s, nxt, n, src, nsrc, srcw, rec, nrec,
                       traces, trace_row);
    return hipGetLastError();
}

// box copy out of a dense level
__global__ void k_read_dense(const float* f, int nx, int ny, int x0, int y0, int z0, int sx, int sy,
                             int sz, float* out) {
    const long long total = (long long)sx * sy * sz;
    const long long gs = (long long)gridDim.x * blockDim.x;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += gs) {
        const int lx = (int)(i % sx);
        const long long r = i / sx;
        const int ly = (int)(r % sy), lz = (int)(r / sy);
        out[i] = f[(size_t)(x0 + lx) + (size_t)nx * ((size_t)(y0 + ly) + (size_t)ny * (size_t)(z0 + lz))];
    }
}

hipError_t launch_read_dense(const float* f, int nx, int ny, int x0, int y0, int z0, int sx, int sy,
                             int sz, float* out, hipStream_t s) {
    const long long total = (long long)sx * sy * sz;
    long long grid = (total + 255) / 256;
    if (grid > 16384) grid = 16384;
    if (grid < 1) grid = 1;
    hipLaunchKernelGGL(k_read_dense, dim3((unsigned)grid), dim3(256), 0, s, f, nx, ny, x0, y0, z0,
                       sx, sy, sz, out);
    return hipGetLastError();
}

// --------------------------------------------------------------------------
// adjoint support: receiver coefficients, gradient accumulation, final scale
// --------------------------------------------------------------------------
__global__ void k_receiver_c2(const Shot* shots, const int* xyz, const int* rshot, int nrec,
                              double dt, double dx, float* out) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= nrec) return;
    const Shot& S = shots[rshot ? rshot[r] : 0];
    out[r] = coeff_c2(media_speed(S, xyz[3 * r], xyz[3 * r + 1], xyz[3 * r + 2]), dt, dx);
}

hipError_t launch_receiver_c2(const Shot* shots, const int* xyz, const int* rshot, int nrec,
                              double dt, double dx, float* out, hipStream_t s) {
    hipLaunchKernelGGL(k_receiver_c2, dim3((nrec + 255) / 256), dim3(256), 0, s, shots, xyz, rshot,
                       nrec, dt, dx, out);
    return hipGetLastError();
}


// g_acc += g_gs, g_gs = 0 over the gradient blocks handed out so far (end of
// a group of adjoint steps)
__global__ void k_grad_flush(Tables mu) {
    const long long n = (long long)min(mu.st->n_gblocks, mu.g_cap) * BV;   // the counter may run past the cap
    const long long gs = (long long)gridDim.x * blockDim.x;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gs) {
        mu.g_acc[i] += (double)mu.g_gs[i];
        mu.g_gs[i] = 0.f;
    }
}

hipError_t launch_grad_flush(const Tables& mu, hipStream_t s) {
    long long grid = ((long long)mu.g_cap * BV + 255) / 256;
    if (grid > 16384) grid = 16384;
    if (grid < 1) grid = 1;
    hipLaunchKernelGGL(k_grad_flush, dim3((unsigned)grid), dim3(256), 0, s, mu);
    return hipGetLastError();
}

// dJ/dc = (2 / c) g at every node of shot 0, g the FP64 sum of the node's
// gradient block (0 where its key never had a term, and where c = 0: there
// dC2/dc = 0)
__global__ void k_grad_finish(Tables mu, const Shot* dshot, float* out) {
    const Shot& S = *dshot;
    const long long total = (long long)S.nx * S.ny * S.nz;
    const long long gs = (long long)gridDim.x * blockDim.x;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += gs) {
        const int gx = (int)(i % S.nx);
        const long long r = i / S.nx;
        const int gy = (int)(r % S.ny), gz = (int)(r / S.ny);
        const int gb = mu.g_slot[S.key_base + (long long)block_to_key(S, gx >> 3, gy >> 3, gz >> 3)];
        float v = 0.f;
        if (gb >= 0) {
            const double c = media_speed(S, gx, gy, gz);
            const double g = mu.g_acc[(size_t)gb * BV + (size_t)(((gz & 7) * 8 + (gy & 7)) * 8 + (gx & 7))];
            v = c != 0.0 ? (float)(2.0 / c * g) : 0.f;
        }
        out[i] = v;
    }
}

hipError_t launch_grad_finish(const Tables& mu, const Shot& shot, const Shot* dshot, float* out,
                              hipStream_t s) {
    const long long total = (long long)shot.nx * shot.ny * shot.nz;
    long long grid = (total + 255) / 256;
    if (grid > 65536) grid = 65536;
    if (grid < 1) grid = 1;
    hipLaunchKernelGGL(k_grad_finish, dim3((unsigned)grid), dim3(256), 0, s, mu, dshot, out);
    return hipGetLastError();
}

__global__ void k_fill_int(int* p, long long n, int v) {
    const long long gs = (long long)gridDim.x * blockDim.x;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gs) p[i] = v;
}

hipError_t launch_fill_int(int* p, long long n, int v, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    long long grid = (n + 255) / 256;
    if (grid > 16384) grid = 16384;
    hipLaunchKernelGGL(k_fill_int, dim3((unsigned)grid), dim3(256), 0, s, p, n, v);
    return hipGetLastError();
}

// --------------------------------------------------------------------------
// sparse state copy (checkpoints, snapshots): the device counters, then per
// active entry its list row and slot tables, then its slot's two phi planes;
// the C2 plane is a function of the block and the media and is filled again
// at restore, as at the block's allocation
// --------------------------------------------------------------------------
struct CkEntry {
    int slot, shot;
    unsigned key;
    int pin;
    float c2u;
    unsigned char flags, sdlog, pad0, pad1;
    long long slot_key;
    int row[8];
    int src_head, pad2;
};
static_assert(sizeof(CkEntry) == 72, "checkpoint entries are 72 bytes");

struct CkLayout {
    size_t entries, planes, total;
};

__host__ __device__ inline CkLayout ck_layout(long long n) {
    CkLayout L;
    const size_t head = (sizeof(DevState) + 255) / 256 * 256;
    L.entries = head;
    L.planes = head + ((size_t)n * sizeof(CkEntry) + 255) / 256 * 256;
    L.total = L.planes + (size_t)n * 2 * BV * sizeof(float);
    return L;
}

size_t ck_sparse_bytes(long long n) { return ck_layout(n).total; }

// one wave per entry
__global__ __launch_bounds__(256) void k_ck_gather(Tables t, long long n, char* buf) {
    const CkLayout L = ck_layout(n);
    const long long i = ((long long)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int lane = lane_id();
    if (i >= n) return;
    const int slot = t.act_slot[i];
    float* dst = (float*)(buf + L.planes) + (size_t)i * 2 * BV;
#pragma unroll
    for (int k = 0; k < 2; k++) {
        const float* src = plane_of(t, slot, k);
#pragma unroll
        for (int z = 0; z < 8; z++) dst[k * BV + z * 64 + lane] = src[z * 64 + lane];
    }
    if (lane == 0) {
        CkEntry e;
        e.slot = slot;
        e.shot = t.act_shot[i];
        e.key = t.act_key[i];
        e.pin = t.pin_until[2 * (size_t)(slot)];
        e.c2u = t.slot_c2u[slot];
        e.flags = t.flags[slot];
        e.sdlog = t.sdlog[slot];
        e.pad0 = e.pad1 = 0;
        e.src_head = t.pin_until[2 * (size_t)(slot) + 1];
        e.pad2 = 0;
        e.slot_key = t.slot_key[slot];
        for (int k = 0; k < 8; k++) e.row[k] = t.rows[8 * (size_t)i + k];
        ((CkEntry*)(buf + L.entries))[i] = e;
    }
}

__global__ __launch_bounds__(256) void k_ck_scatter(Tables t, long long n, const char* buf) {
    const CkLayout L = ck_layout(n);
    const long long i = ((long long)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int lane = lane_id();
    if (i >= n) return;
    const CkEntry e = ((const CkEntry*)(buf + L.entries))[i];
    const float* src = (const float*)(buf + L.planes) + (size_t)i * 2 * BV;
#pragma unroll
    for (int k = 0; k < 2; k++) {
        float* dst = plane_of(t, e.slot, k);
#pragma unroll
        for (int z = 0; z < 8; z++) dst[z * 64 + lane] = src[k * BV + z * 64 + lane];
    }
    if (!t.c2_ready) {
        const Shot& S = t.shots[e.shot];
        int bx, by, bz;
        key_to_block(S, e.key, bx, by, bz);
        (void)fill_c2(t, S, e.slot, bx, by, bz);
    }
    if (lane == 0) {
        t.act_slot[i] = e.slot;
        t.act_shot[i] = e.shot;
        t.act_key[i] = e.key;
        for (int k = 0; k < 8; k++) t.rows[8 * (size_t)i + k] = e.row[k];
        t.pin_until[2 * (size_t)(e.slot)] = e.pin;
        t.pin_until[2 * (size_t)(e.slot) + 1] = e.src_head;
        t.slot_c2u[e.slot] = e.c2u;
        t.flags[e.slot] = e.flags;
        t.sdlog[e.slot] = e.sdlog;
        t.slot_key[e.slot] = e.slot_key;
        t.cell2box[e.slot_key] = e.slot;
        if (t.fast) {
            const int step = ((const DevState*)buf)->step;
            atomicOr(&fast_bm(t, step & 1)[e.slot_key >> 6], 1ull << (e.slot_key & 63));
        }
    }
}

hipError_t launch_ck_gather(const Tables& t, long long n, char* buf, hipStream_t s) {
    if (n > 0)
        hipLaunchKernelGGL(k_ck_gather, dim3((unsigned)((n + 3) / 4)), dim3(256), 0, s, t, n, buf);
    return hipGetLastError();
}

hipError_t launch_ck_scatter(const Tables& t, long long n, const char* buf, hipStream_t s) {
    if (n > 0)
        hipLaunchKernelGGL(k_ck_scatter, dim3((unsigned)((n + 3) / 4)), dim3(256), 0, s, t, n, buf);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// HBM ceiling probe.  dst = src_0 (+ src_1 (+ src_2)) in the fastest streaming
// shape found by a sweep of load widths, unrolls and grid sizes: each lane
// moves two consecutive floats (a wave 512 contiguous bytes per access), every
// thread handles PROBE_UNROLL such pairs 512 floats apart so that its loads
// are in flight together (a workgroup pass covers 16 KiB of each stream), and
// loads and stores are non-temporal.  With three sources the read:write mix
// is the stencil's 12:4 bytes per node.
constexpr int PROBE_UNROLL = 8;
constexpr long long PROBE_CHUNK = 512LL * PROBE_UNROLL;   // floats per workgroup pass
typedef float probe_f2 __attribute__((ext_vector_type(2)));

template <int NR>
__global__ __launch_bounds__(256) void k_hbm_probe(const float* __restrict__ src, float* __restrict__ dst,
                                                  long long n) {
    const long long nchunks = n / PROBE_CHUNK;
    const long long n2 = n / 2;                 // pairs per stream (n is a multiple of PROBE_CHUNK)
    const probe_f2* __restrict__ s2 = (const probe_f2*)src;
    probe_f2* __restrict__ d2 = (probe_f2*)dst;
    for (long long c = blockIdx.x; c < nchunks; c += gridDim.x) {
        const long long base = c * (PROBE_CHUNK / 2) + threadIdx.x;
        probe_f2 v[PROBE_UNROLL];
#pragma unroll
        for (int u = 0; u < PROBE_UNROLL; u++) v[u] = __builtin_nontemporal_load(&s2[base + u * 256]);
        if (NR >= 2) {
#pragma unroll
            for (int u = 0; u < PROBE_UNROLL; u++) v[u] += __builtin_nontemporal_load(&s2[n2 + base + u * 256]);
        }
        if (NR >= 3) {
#pragma unroll
            for (int u = 0; u < PROBE_UNROLL; u++)
                v[u] += __builtin_nontemporal_load(&s2[2 * n2 + base + u * 256]);
        }
#pragma unroll
        for (int u = 0; u < PROBE_UNROLL; u++) __builtin_nontemporal_store(v[u], &d2[base + u * 256]);
    }
}

long long hbm_probe_chunk() { return PROBE_CHUNK; }

hipError_t launch_hbm_probe(const float* src, float* dst, long long n, int nread, int grid, hipStream_t s,
                            hipEvent_t e0, hipEvent_t e1) {
    void (*k)(const float*, float*, long long) =
        nread == 1 ? k_hbm_probe<1> : nread == 2 ? k_hbm_probe<2> : k_hbm_probe<3>;
    hipExtLaunchKernelGGL(k, dim3(grid), dim3(256), 0, s, e0, e1, 0, src, dst, n);
    return hipGetLastError();
}

}  // namespace tcmk
