/*
 * CPU oracle, body instantiated once per precision (REAL = float, double).
 * TEST INFRASTRUCTURE ONLY -- see tcm_oracle.c for the rules of use.
 *
 * Expression order of the per-node update (the "basic calculation", eq.(3)),
 * fixed here and stated once for every user of the oracle:
 *     s    = ((x+ + x-) + (y+ + y-)) + (z+ + z-)
 *     lap  = s - 6 phi
 *     next = (2 phi - prev) + C2 lap,       C2 = REAL(t*t), t = (double)c * dt / dx
 * Nodes outside [0,nx)x[0,ny)x[0,nz) hold zero (no absorbing layer).
 */

/* ======================================================================= */
/* O1: dense leapfrog over the whole grid (Introduction, eq.(3); two arrays  */
/*     with phi^{n+1} written over phi^{n-1}, as the paper describes).       */
/* ======================================================================= */
int SFX(oracle_dense)(int nx, int ny, int nz, int ndim,
                      const REAL* c, double dt, double dx,
                      REAL* phi, REAL* phi_prev, int step0, int nsteps,
                      int nsrc, const int64_t* src_idx, const int* src_t0,
                      const int* src_ns, const int64_t* src_off, const REAL* src_w,
                      int nrec, const int64_t* rec_idx, REAL* traces)
{
    if (nx <= 0 || ny <= 0 || nz <= 0 || nsteps < 0 || ndim < 1 || ndim > 3) return -1;
    const size_t N = (size_t)nx * ny * nz;
    const size_t sy = (size_t)nx, sz = (size_t)nx * ny;
    REAL* c2 = (REAL*)malloc(N * sizeof(REAL));
    if (!c2) return -7;
    for (size_t i = 0; i < N; i++) {
        double t = (double)c[i] * dt / dx;          /* c dt / dx */
        c2[i] = (REAL)(t * t);                       /* (c dt / dx)^2, one rounding */
    }
    REAL* cur = phi;        /* phi^n       */
    REAL* prv = phi_prev;   /* phi^{n-1}, overwritten by phi^{n+1} */
    for (int it = 0; it < nsteps; it++) {
        const int n = step0 + it;
        #pragma omp parallel for schedule(static)
        for (int z = 0; z < nz; z++) {
            for (int y = 0; y < ny; y++) {
                const size_t row = (size_t)z * sz + (size_t)y * sy;
                for (int x = 0; x < nx; x++) {
                    const size_t i = row + (size_t)x;
                    const REAL p = cur[i];
                    const REAL xm = x > 0 ? cur[i - 1] : (REAL)0;
                    const REAL xp = x + 1 < nx ? cur[i + 1] : (REAL)0;
                    REAL lap;
                    if (ndim == 1) {
                        lap = (xp + xm) - (REAL)2 * p;
                    } else {
                        const REAL ym = y > 0 ? cur[i - sy] : (REAL)0;
                        const REAL yp = y + 1 < ny ? cur[i + sy] : (REAL)0;
                        if (ndim == 2) {
                            lap = ((xp + xm) + (yp + ym)) - (REAL)4 * p;
                        } else {
                            const REAL zm = z > 0 ? cur[i - sz] : (REAL)0;
                            const REAL zp = z + 1 < nz ? cur[i + sz] : (REAL)0;
                            const REAL s = ((xp + xm) + (yp + ym)) + (zp + zm);
                            lap = s - (REAL)6 * p;
                        }
                    }
                    prv[i] = ((REAL)2 * p - prv[i]) + c2[i] * lap;
                }
            }
        }
        /* additive source insertion into phi^{n+1} ("Source insertion") */
        for (int s = 0; s < nsrc; s++) {
            const int k = n - src_t0[s];
            if (k >= 0 && k < src_ns[s]) prv[src_idx[s]] = prv[src_idx[s]] + src_w[src_off[s] + k];
        }
        for (int r = 0; r < nrec; r++) traces[(size_t)it * nrec + r] = prv[rec_idx[r]];
        REAL* t = cur; cur = prv; prv = t;
    }
    if (cur != phi) {   /* odd step count: hand back phi = phi^n, phi_prev = phi^{n-1} */
        for (size_t i = 0; i < N; i++) { REAL t = phi[i]; phi[i] = phi_prev[i]; phi_prev[i] = t; }
    }
    free(c2);
    return 0;
}

/* ======================================================================= */
/* O2: CPU TCM with the paper's cell/box bookkeeping (Table 1, Figure 1).    */
/* ======================================================================= */
typedef struct SFX(otcm) {
    int nx, ny, nz, B, mx, my, mz;
    int64_t M;                 /* number of cells (coarse grid) */
    int B3;
    double dt, dx;
    REAL trigger, retire;
    REAL* c;                   /* media as a dense array ("Media") */
    /* Table 1 */
    unsigned char* triggered;  /* Triggered_cells */
    unsigned char* hist;       /* Triggered_hist  */
    REAL* max_val;             /* Max_cell_val    (max |phi^{n+1}| of the cell) */
    int* cell2box;             /* Cell2box */
    int* box2cell;             /* Box2cell */
    /* boxes: each [phi plane 0 | phi plane 1 | C^2], B^3 values per plane */
    int cap, nboxes;           /* cap on boxes, boxes created so far */
    REAL* boxes;
    int* vacant; int nvacant;  /* unboxed (initialised) boxes ready for reuse */
    int cur;                   /* plane holding phi^n */
    int step;
    int64_t* active; int64_t nactive;   /* triggered cells, ascending id */
    /* sources */
    int nsrc; int64_t* src_cell; int* src_local; int* src_t0; int* src_ns;
    int64_t* src_off; REAL* src_w; int64_t nw;
    int nrec; int64_t* rec_cell; int* rec_local;
    int error;
    int64_t peak_active, activations, retirements, updates;
    /* shutdown process (eq.(6)): decay steps and factor; Table 1 Shutdown_log */
    int sd_steps;
    REAL sd_alpha;
    int* shutdown_log;
    int64_t decays;
    /* adaptive trigger (Table 1 Trig_level relative to the domain maximum) */
    REAL trig_rel, ret_rel;
    REAL last_trig, last_ret;
    /* activation update every `interval` steps (eq.(5)); > 1 uses the 26 nearest
     * and diagonal cells (Table 1 Linked_cells + Diag_cells, Figure 3) */
    int interval;
} SFX(otcm);

void SFX(otcm_destroy)(SFX(otcm)* t);

static REAL* SFX(box_plane)(SFX(otcm)* t, int box, int plane) {
    return t->boxes + ((size_t)box * 3 + (size_t)plane) * (size_t)t->B3;
}

static void SFX(cell_coords)(const SFX(otcm)* t, int64_t cell, int* cx, int* cy, int* cz) {
    *cx = (int)(cell % t->mx);
    *cy = (int)((cell / t->mx) % t->my);
    *cz = (int)(cell / ((int64_t)t->mx * t->my));
}

/* face-adjacent cell across face f (0:-x 1:+x 2:-y 3:+y 4:-z 5:+z), -1 outside */
static int64_t SFX(linked_cell)(const SFX(otcm)* t, int64_t cell, int f) {
    int cx, cy, cz;
    SFX(cell_coords)(t, cell, &cx, &cy, &cz);
    switch (f) {
        case 0: cx--; break; case 1: cx++; break;
        case 2: cy--; break; case 3: cy++; break;
        case 4: cz--; break; default: cz++; break;
    }
    if (cx < 0 || cy < 0 || cz < 0 || cx >= t->mx || cy >= t->my || cz >= t->mz) return -1;
    return (int64_t)cx + (int64_t)t->mx * ((int64_t)cy + (int64_t)t->my * cz);
}

static int SFX(cell_ncells)(const SFX(otcm)* t, int64_t cell) {
    int cx, cy, cz;
    SFX(cell_coords)(t, cell, &cx, &cy, &cz);
    int ex = t->nx - cx * t->B; if (ex > t->B) ex = t->B;
    int ey = t->ny - cy * t->B; if (ey > t->B) ey = t->B;
    int ez = t->nz - cz * t->B; if (ez > t->B) ez = t->B;
    return ex * ey * ez;
}

/* Box a cell: take a vacant box, or create a new one ("Boxes", Figure 1). */
static int SFX(box_cell)(SFX(otcm)* t, int64_t cell) {
    int j;
    if (t->nvacant > 0) {
        j = t->vacant[--t->nvacant];
    } else {
        if (t->nboxes >= t->cap) return -1;
        j = t->nboxes++;
    }
    const int B = t->B;
    REAL* p0 = SFX(box_plane)(t, j, 0);
    REAL* p1 = SFX(box_plane)(t, j, 1);
    REAL* k2 = SFX(box_plane)(t, j, 2);
    memset(p0, 0, sizeof(REAL) * (size_t)t->B3);
    memset(p1, 0, sizeof(REAL) * (size_t)t->B3);
    int cx, cy, cz;
    SFX(cell_coords)(t, cell, &cx, &cy, &cz);
    for (int z = 0; z < B; z++)
        for (int y = 0; y < B; y++)
            for (int x = 0; x < B; x++) {
                const int gx = cx * B + x, gy = cy * B + y, gz = cz * B + z;
                REAL v = 0;
                if (gx < t->nx && gy < t->ny && gz < t->nz) {
                    double tt = (double)t->c[(size_t)gx + (size_t)t->nx * ((size_t)gy + (size_t)t->ny * gz)] * t->dt / t->dx;
                    v = (REAL)(tt * tt);
                }
                k2[(z * B + y) * B + x] = v;
            }
    t->cell2box[cell] = j;
    t->box2cell[j] = (int)cell;   /* cell ids of tested grids fit in int */
    t->triggered[cell] = 1;
    t->shutdown_log[cell] = 0;
    return j;
}

/* Unbox a cell: initialise its box and put it on the vacant list. */
static void SFX(unbox_cell)(SFX(otcm)* t, int64_t cell) {
    const int j = t->cell2box[cell];
    memset(SFX(box_plane)(t, j, 0), 0, sizeof(REAL) * 2 * (size_t)t->B3);
    t->vacant[t->nvacant++] = j;
    t->cell2box[cell] = -1;
    t->box2cell[j] = -1;
    t->triggered[cell] = 0;
}

SFX(otcm)* SFX(otcm_create)(int nx, int ny, int nz, int B, const REAL* c, double dt, double dx,
                            REAL trigger, REAL retire, int cap)
{
    if (nx <= 0 || ny <= 0 || nz <= 0 || B <= 0) return NULL;
    SFX(otcm)* t = (SFX(otcm)*)calloc(1, sizeof(SFX(otcm)));
    t->nx = nx; t->ny = ny; t->nz = nz; t->B = B; t->B3 = B * B * B;
    t->mx = (nx + B - 1) / B; t->my = (ny + B - 1) / B; t->mz = (nz + B - 1) / B;
    t->M = (int64_t)t->mx * t->my * t->mz;
    t->dt = dt; t->dx = dx; t->trigger = trigger; t->retire = retire;
    t->cap = cap > 0 && cap < t->M ? cap : (int)t->M;
    const size_t N = (size_t)nx * ny * nz;
    t->c = (REAL*)malloc(N * sizeof(REAL));
    memcpy(t->c, c, N * sizeof(REAL));
    t->triggered = (unsigned char*)calloc((size_t)t->M, 1);
    t->hist = (unsigned char*)calloc((size_t)t->M, 1);
    t->max_val = (REAL*)calloc((size_t)t->M, sizeof(REAL));
    t->cell2box = (int*)malloc((size_t)t->M * sizeof(int));
    for (int64_t i = 0; i < t->M; i++) t->cell2box[i] = -1;
    t->box2cell = (int*)malloc((size_t)t->cap * sizeof(int));
    for (int i = 0; i < t->cap; i++) t->box2cell[i] = -1;
    t->boxes = (REAL*)malloc((size_t)t->cap * 3 * (size_t)t->B3 * sizeof(REAL));
    t->vacant = (int*)malloc((size_t)t->cap * sizeof(int));
    t->active = (int64_t*)malloc((size_t)t->M * sizeof(int64_t));
    t->shutdown_log = (int*)calloc((size_t)t->M, sizeof(int));
    t->sd_alpha = (REAL)1;
    t->interval = 1;
    if (!t->shutdown_log ||
        !t->c || !t->triggered || !t->hist || !t->max_val || !t->cell2box || !t->box2cell ||
        !t->boxes || !t->vacant || !t->active) {
        SFX(otcm_destroy)(t);
        return NULL;
    }
    return t;
}

void SFX(otcm_destroy)(SFX(otcm)* t)
{
    if (!t) return;
    free(t->c); free(t->triggered); free(t->hist); free(t->max_val); free(t->cell2box);
    free(t->box2cell); free(t->boxes); free(t->vacant); free(t->active); free(t->shutdown_log);
    free(t->src_cell); free(t->src_local); free(t->src_t0); free(t->src_ns); free(t->src_off);
    free(t->src_w); free(t->rec_cell); free(t->rec_local);
    free(t);
}

static void SFX(rebuild_active)(SFX(otcm)* t) {
    int64_t k = 0;
    for (int64_t i = 0; i < t->M; i++) if (t->triggered[i]) t->active[k++] = i;
    t->nactive = k;
    if (k > t->peak_active) t->peak_active = k;
}

static void SFX(locate)(const SFX(otcm)* t, int x, int y, int z, int64_t* cell, int* local) {
    const int B = t->B;
    *cell = (int64_t)(x / B) + (int64_t)t->mx * ((int64_t)(y / B) + (int64_t)t->my * (z / B));
    *local = ((z % B) * B + (y % B)) * B + (x % B);
}

/* Source insertion: the source cell is activated by hand and stays active
 * while the source still has samples to insert. Returns 0, -4 (outside), -3 (pool). */
int SFX(otcm_add_source)(SFX(otcm)* t, int x, int y, int z, const REAL* w, int ns)
{
    if (x < 0 || y < 0 || z < 0 || x >= t->nx || y >= t->ny || z >= t->nz) return -4;
    if (ns < 0) return -1;
    int64_t cell; int local;
    SFX(locate)(t, x, y, z, &cell, &local);
    if (t->cell2box[cell] < 0) {
        if (SFX(box_cell)(t, cell) < 0) return -3;
        t->activations++;
    }
    if (t->interval > 1) {
        /* the source reaches the cells around it before the next update */
        int cx, cy, cz;
        SFX(cell_coords)(t, cell, &cx, &cy, &cz);
        for (int dz = -1; dz <= 1; dz++)
            for (int dy = -1; dy <= 1; dy++)
                for (int dx = -1; dx <= 1; dx++) {
                    const int x2 = cx + dx, y2 = cy + dy, z2 = cz + dz;
                    if (x2 < 0 || y2 < 0 || z2 < 0 || x2 >= t->mx || y2 >= t->my || z2 >= t->mz) continue;
                    const int64_t nb = (int64_t)x2 + (int64_t)t->mx * ((int64_t)y2 + (int64_t)t->my * z2);
                    if (t->cell2box[nb] >= 0) continue;
                    if (SFX(box_cell)(t, nb) < 0) return -3;
                    t->activations++;
                }
    }
    const int s = t->nsrc++;
    t->src_cell = (int64_t*)realloc(t->src_cell, sizeof(int64_t) * t->nsrc);
    t->src_local = (int*)realloc(t->src_local, sizeof(int) * t->nsrc);
    t->src_t0 = (int*)realloc(t->src_t0, sizeof(int) * t->nsrc);
    t->src_ns = (int*)realloc(t->src_ns, sizeof(int) * t->nsrc);
    t->src_off = (int64_t*)realloc(t->src_off, sizeof(int64_t) * t->nsrc);
    t->src_w = (REAL*)realloc(t->src_w, sizeof(REAL) * (size_t)(t->nw + ns + 1));
    t->src_cell[s] = cell; t->src_local[s] = local; t->src_t0[s] = t->step; t->src_ns[s] = ns;
    t->src_off[s] = t->nw;
    memcpy(t->src_w + t->nw, w, sizeof(REAL) * (size_t)ns);
    t->nw += ns;
    SFX(rebuild_active)(t);
    return 0;
}

int SFX(otcm_set_receivers)(SFX(otcm)* t, const int* xyz, int nrec)
{
    for (int r = 0; r < nrec; r++) {
        const int x = xyz[3 * r], y = xyz[3 * r + 1], z = xyz[3 * r + 2];
        if (x < 0 || y < 0 || z < 0 || x >= t->nx || y >= t->ny || z >= t->nz) return -4;
    }
    t->nrec = nrec;
    t->rec_cell = (int64_t*)realloc(t->rec_cell, sizeof(int64_t) * (size_t)(nrec + 1));
    t->rec_local = (int*)realloc(t->rec_local, sizeof(int) * (size_t)(nrec + 1));
    for (int r = 0; r < nrec; r++)
        SFX(locate)(t, xyz[3 * r], xyz[3 * r + 1], xyz[3 * r + 2], &t->rec_cell[r], &t->rec_local[r]);
    return 0;
}

static int SFX(pinned)(const SFX(otcm)* t, int64_t cell, int n) {
    for (int s = 0; s < t->nsrc; s++)
        if (t->src_cell[s] == cell && n < t->src_t0[s] + t->src_ns[s]) return 1;
    return 0;
}

/* Time stepping of one box: pad it with its neighbours' phi^n boundaries
 * ("Time stepping"), then apply the basic calculation to its nodes. */
static void SFX(step_box)(SFX(otcm)* t, int64_t cell, REAL* pad) {
    const int B = t->B, P = B + 2;
    const int j = t->cell2box[cell];
    const REAL* cur = SFX(box_plane)(t, j, t->cur);
    REAL* nxt = SFX(box_plane)(t, j, 1 - t->cur);
    const REAL* k2 = SFX(box_plane)(t, j, 2);
    memset(pad, 0, sizeof(REAL) * (size_t)P * P * P);
#define PAD(x, y, z) pad[(((z) + 1) * P + ((y) + 1)) * P + ((x) + 1)]
    for (int z = 0; z < B; z++)
        for (int y = 0; y < B; y++)
            for (int x = 0; x < B; x++) PAD(x, y, z) = cur[(z * B + y) * B + x];
    for (int f = 0; f < 6; f++) {
        const int64_t nb = SFX(linked_cell)(t, cell, f);
        if (nb < 0 || t->cell2box[nb] < 0) continue;    /* outside or untriggered: zeros */
        const REAL* q = SFX(box_plane)(t, t->cell2box[nb], t->cur);
        for (int a = 0; a < B; a++)
            for (int b = 0; b < B; b++) {
                switch (f) {
                    case 0: PAD(-1, a, b) = q[(b * B + a) * B + (B - 1)]; break;
                    case 1: PAD(B, a, b) = q[(b * B + a) * B + 0]; break;
                    case 2: PAD(a, -1, b) = q[(b * B + (B - 1)) * B + a]; break;
                    case 3: PAD(a, B, b) = q[(b * B + 0) * B + a]; break;
                    case 4: PAD(a, b, -1) = q[((B - 1) * B + b) * B + a]; break;
                    default: PAD(a, b, B) = q[(0 * B + b) * B + a]; break;
                }
            }
    }
    int cx, cy, cz;
    SFX(cell_coords)(t, cell, &cx, &cy, &cz);
    for (int z = 0; z < B; z++)
        for (int y = 0; y < B; y++)
            for (int x = 0; x < B; x++) {
                const int gx = cx * B + x, gy = cy * B + y, gz = cz * B + z;
                if (gx >= t->nx || gy >= t->ny || gz >= t->nz) continue;  /* outside the domain */
                /* out-of-domain pad nodes are zero ghosts */
                const REAL xp = gx + 1 < t->nx ? PAD(x + 1, y, z) : (REAL)0;
                const REAL yp = gy + 1 < t->ny ? PAD(x, y + 1, z) : (REAL)0;
                const REAL zp = gz + 1 < t->nz ? PAD(x, y, z + 1) : (REAL)0;
                const REAL xm = PAD(x - 1, y, z), ym = PAD(x, y - 1, z), zm = PAD(x, y, z - 1);
                const REAL p = PAD(x, y, z);
                const int i = (z * B + y) * B + x;
                const REAL s = ((xp + xm) + (yp + ym)) + (zp + zm);
                const REAL lap = s - (REAL)6 * p;
                nxt[i] = ((REAL)2 * p - nxt[i]) + k2[i] * lap;
            }
#undef PAD
}

/* Advance nsteps. traces (nsteps x nrec) may be NULL. order_seed != 0 runs
 * the boxes sequentially in a seeded random order (the result must not
 * depend on it). Returns 0, or -3 when the pool cap is exceeded: the state
 * then holds the last complete step (phi^{n+1} of the active cells) and
 * further steps are refused. */
int SFX(otcm_step)(SFX(otcm)* t, int nsteps, REAL* traces, unsigned order_seed)
{
    if (t->error) return t->error;
    const int B = t->B;
    const int P = B + 2;
    unsigned char* next = (unsigned char*)malloc((size_t)t->M);
    int64_t* order = (int64_t*)malloc(sizeof(int64_t) * (size_t)(t->M > 0 ? t->M : 1));
    for (int it = 0; it < nsteps; it++) {
        const int n = t->step;
        /* ---- time stepping of the active boxes ---- */
        if (order_seed == 0) {
            #pragma omp parallel
            {
                REAL* pad = (REAL*)malloc(sizeof(REAL) * (size_t)P * P * P);
                #pragma omp for schedule(dynamic, 16)
                for (int64_t a = 0; a < t->nactive; a++) SFX(step_box)(t, t->active[a], pad);
                free(pad);
            }
        } else {
            uint64_t st = 0x9E3779B97F4A7C15ull ^ ((uint64_t)order_seed * 0xD1B54A32D192ED03ull) ^ (uint64_t)n;
            for (int64_t a = 0; a < t->nactive; a++) order[a] = t->active[a];
            for (int64_t a = t->nactive - 1; a > 0; a--) {       /* Fisher-Yates */
                st ^= st << 13; st ^= st >> 7; st ^= st << 17;
                const int64_t b = (int64_t)(st % (uint64_t)(a + 1));
                const int64_t tmp = order[a]; order[a] = order[b]; order[b] = tmp;
            }
            REAL* pad = (REAL*)malloc(sizeof(REAL) * (size_t)P * P * P);
            for (int64_t a = 0; a < t->nactive; a++) SFX(step_box)(t, order[a], pad);
            free(pad);
        }
        /* ---- source insertion into the source boxes ---- */
        for (int s = 0; s < t->nsrc; s++) {
            const int k = n - t->src_t0[s];
            if (k < 0 || k >= t->src_ns[s]) continue;
            REAL* nxt = SFX(box_plane)(t, t->cell2box[t->src_cell[s]], 1 - t->cur);
            nxt[t->src_local[s]] = nxt[t->src_local[s]] + t->src_w[t->src_off[s] + k];
        }
        for (int r = 0; r < t->nrec; r++) {
            REAL v = 0;
            const int j = t->cell2box[t->rec_cell[r]];
            if (j >= 0) v = SFX(box_plane)(t, j, 1 - t->cur)[t->rec_local[r]];
            if (traces) traces[(size_t)it * t->nrec + r] = v;
        }
        for (int64_t a = 0; a < t->nactive; a++) t->updates += SFX(cell_ncells)(t, t->active[a]);

        /* ---- activation process ("Updating active cells"), every `interval` steps ---- */
        if ((n + 1) % t->interval != 0) {
            t->cur ^= 1;
            t->step++;
            continue;
        }
        /* 1. maximal absolute value per active cell (whole box, each face, and phi^n) */
        memset(next, 0, (size_t)t->M);
        REAL* cmax = (REAL*)malloc(sizeof(REAL) * 8 * (size_t)(t->nactive > 0 ? t->nactive : 1));
        REAL dom_max = 0;
        for (int64_t a = 0; a < t->nactive; a++) {
            const int64_t cell = t->active[a];
            const int j = t->cell2box[cell];
            const REAL* nw = SFX(box_plane)(t, j, 1 - t->cur);
            const REAL* nn = SFX(box_plane)(t, j, t->cur);
            REAL mx = 0, mprev = 0, face[6] = {0, 0, 0, 0, 0, 0};
            for (int z = 0; z < B; z++)
                for (int y = 0; y < B; y++)
                    for (int x = 0; x < B; x++) {
                        const int i = (z * B + y) * B + x;
                        const REAL v = nw[i] < 0 ? -nw[i] : nw[i];
                        const REAL u = nn[i] < 0 ? -nn[i] : nn[i];
                        if (v > mx) mx = v;
                        if (u > mprev) mprev = u;
                        if (x == 0 && v > face[0]) face[0] = v;
                        if (x == B - 1 && v > face[1]) face[1] = v;
                        if (y == 0 && v > face[2]) face[2] = v;
                        if (y == B - 1 && v > face[3]) face[3] = v;
                        if (z == 0 && v > face[4]) face[4] = v;
                        if (z == B - 1 && v > face[5]) face[5] = v;
                    }
            t->max_val[cell] = mx;
            for (int f = 0; f < 6; f++) cmax[8 * a + f] = face[f];
            cmax[8 * a + 6] = mx;
            cmax[8 * a + 7] = mprev;
            if (mx > dom_max) dom_max = mx;
        }
        /* trigger and keep levels: constant, or relative to the domain maximum */
        REAL trig = t->trigger, ret = t->retire;
        if (t->trig_rel > 0 || t->ret_rel > 0) {
            const REAL at = t->trig_rel * dom_max, ar = t->ret_rel * dom_max;
            if (at > trig) trig = at;
            if (ar > ret) ret = ar;
        }
        t->last_trig = trig;
        t->last_ret = ret;
        for (int64_t a = 0; a < t->nactive; a++) {
            const int64_t cell = t->active[a];
            const REAL* m = cmax + 8 * a;
            /* 2. register the current active cells */
            t->hist[cell] = 1;
            /* 3. keep cells whose field (new or current level) is above the retire level,
             *    and source cells that still insert samples */
            if (m[6] > ret || m[7] > ret || SFX(pinned)(t, cell, n + 1)) next[cell] = 1;
            if (t->interval == 1) {
                /* 4. trigger the face neighbours across faces whose field exceeds the trigger */
                for (int f = 0; f < 6; f++) {
                    if (!(m[f] > trig)) continue;
                    const int64_t nb = SFX(linked_cell)(t, cell, f);
                    if (nb >= 0) next[nb] = 1;
                }
            } else if (m[6] > trig || m[7] > trig || SFX(pinned)(t, cell, n + 1)) {
                /* 4-5. a cell above the trigger anywhere (either level), or one whose
                 *      source still inserts, triggers its nearest and diagonal
                 *      neighbours (Figure 3 a-c) */
                int cx, cy, cz;
                SFX(cell_coords)(t, cell, &cx, &cy, &cz);
                for (int dz = -1; dz <= 1; dz++)
                    for (int dy = -1; dy <= 1; dy++)
                        for (int dx = -1; dx <= 1; dx++) {
                            const int x = cx + dx, y = cy + dy, z = cz + dz;
                            if ((dx | dy | dz) == 0 || x < 0 || y < 0 || z < 0 || x >= t->mx ||
                                y >= t->my || z >= t->mz)
                                continue;
                            next[(int64_t)x + (int64_t)t->mx * ((int64_t)y + (int64_t)t->my * z)] = 1;
                        }
            }
        }
        free(cmax);
        /* 6. shutdown process (eq.(6)) for active cells that are no longer triggered */
        unsigned char* decay = NULL;
        if (t->sd_steps > 0) {
            decay = (unsigned char*)calloc((size_t)t->M, 1);
            for (int64_t a = 0; a < t->nactive; a++) {
                const int64_t cell = t->active[a];
                int* lg = &t->shutdown_log[cell];
                if (next[cell]) {
                    *lg = 0;                       /* triggered again: shutdown cancelled */
                } else if (*lg == 0) {
                    *lg = t->sd_steps;             /* start */
                    next[cell] = 1;
                    decay[cell] = 1;
                } else if (*lg > 1) {
                    *lg -= 1;
                    next[cell] = 1;
                    decay[cell] = 1;
                }                                  /* *lg == 1: finished, unboxed below */
            }
        }
        int64_t count = 0;
        for (int64_t i = 0; i < t->M; i++) count += next[i];
        if (count > t->cap) {
            free(decay);
            /* pool exhausted: keep phi^{n+1} with the current active set and stop */
            for (int64_t a = 0; a < t->nactive; a++) t->hist[t->active[a]] = 0;
            t->cur ^= 1;
            t->step++;
            t->error = -3;
            break;
        }
        if (decay) {
            for (int64_t a = 0; a < t->nactive; a++) {
                const int64_t cell = t->active[a];
                if (!decay[cell]) continue;
                REAL* q = SFX(box_plane)(t, t->cell2box[cell], 0);
                for (int k = 0; k < 2 * B * B * B; k++) q[k] = q[k] * t->sd_alpha;
                t->decays++;
            }
            free(decay);
        }
        /* 7. cells that finished the shutdown (or have none) are unboxed */
        for (int64_t a = 0; a < t->nactive; a++) {
            const int64_t cell = t->active[a];
            if (!next[cell]) { SFX(unbox_cell)(t, cell); t->retirements++; }
        }
        /* 8. box newly triggered cells in vacant or newly created boxes */
        for (int64_t i = 0; i < t->M; i++) {
            if (next[i] && !t->hist[i]) {
                if (SFX(box_cell)(t, i) < 0) { t->error = -3; break; }   /* cannot happen: count <= cap */
                t->activations++;
            }
        }
        for (int64_t a = 0; a < t->nactive; a++) t->hist[t->active[a]] = 0;
        t->cur ^= 1;
        t->step++;
        SFX(rebuild_active)(t);
        if (t->error) break;
    }
    free(next);
    free(order);
    return t->error;
}

/* Dense copy of phi^n (which = 0) or phi^{n-1} (which = 1); inactive cells read 0. */
int SFX(otcm_read)(const SFX(otcm)* t, int which, REAL* out)
{
    const size_t N = (size_t)t->nx * t->ny * t->nz;
    memset(out, 0, N * sizeof(REAL));
    const int B = t->B;
    const int plane = which == 0 ? t->cur : 1 - t->cur;
    for (int64_t a = 0; a < t->nactive; a++) {
        const int64_t cell = t->active[a];
        int cx, cy, cz;
        SFX(cell_coords)(t, cell, &cx, &cy, &cz);
        const REAL* q = SFX(box_plane)((SFX(otcm)*)t, t->cell2box[cell], plane);
        for (int z = 0; z < B; z++)
            for (int y = 0; y < B; y++)
                for (int x = 0; x < B; x++) {
                    const int gx = cx * B + x, gy = cy * B + y, gz = cz * B + z;
                    if (gx >= t->nx || gy >= t->ny || gz >= t->nz) continue;
                    out[(size_t)gx + (size_t)t->nx * ((size_t)gy + (size_t)t->ny * gz)] = q[(z * B + y) * B + x];
                }
    }
    return 0;
}

/* stats: [step, nactive, peak_active, nboxes (memory high-water), activations,
 *         retirements, updates, error] */
int SFX(otcm_stats)(const SFX(otcm)* t, int64_t* out)
{
    out[0] = t->step; out[1] = t->nactive; out[2] = t->peak_active; out[3] = t->nboxes;
    out[4] = t->activations; out[5] = t->retirements; out[6] = t->updates; out[7] = t->error;
    return 0;
}

/* Triggered_cells flags (M bytes, cell id = cx + mx (cy + my cz)). */
int SFX(otcm_triggered)(const SFX(otcm)* t, unsigned char* out)
{
    memcpy(out, t->triggered, (size_t)t->M);
    return 0;
}

/* Shutdown process of eq.(6): a cell that is no longer triggered is kept for
 * n more activation updates while both of its field levels are multiplied by
 * alpha after each of them (total attenuation A = alpha^n), then unboxed.
 * n = 0 unboxes at once. */
int SFX(otcm_set_shutdown)(SFX(otcm)* t, int n, REAL alpha)
{
    if (n < 0 || n > 255) return -1;
    t->sd_steps = n;
    t->sd_alpha = alpha;
    return 0;
}

/* Adaptive levels: at each activation update the trigger is
 * max(trigger, trig_rel * M) and the keep level max(retire, ret_rel * M), M
 * the maximal |phi^{n+1}| over the active cells (item 1 of the update). */
int SFX(otcm_set_adaptive)(SFX(otcm)* t, REAL trig_rel, REAL ret_rel)
{
    if (!(trig_rel >= 0) || !(ret_rel >= 0) || ret_rel > trig_rel) return -1;
    t->trig_rel = trig_rel;
    t->ret_rel = ret_rel;
    return 0;
}

/* Run the activation update after every k-th step (1 <= k <= block edge).
 * With k > 1 a cell holding any |phi^{n+1}| above the trigger activates all 26
 * cells around it (nearest and diagonal), so that a value moving one node per
 * step cannot leave the active region before the next update. */
int SFX(otcm_set_interval)(SFX(otcm)* t, int k)
{
    if (k < 1 || k > t->B) return -1;
    t->interval = k;
    return 0;
}

/* Levels used by the last activation update: out[0] trigger, out[1] keep level. */
int SFX(otcm_levels)(const SFX(otcm)* t, REAL* out)
{
    out[0] = t->last_trig;
    out[1] = t->last_ret;
    return 0;
}

/* Bookkeeping invariants; returns the number of violations. */
int SFX(otcm_check)(const SFX(otcm)* t)
{
    int bad = 0;
    unsigned char* seen = (unsigned char*)calloc((size_t)(t->nboxes > 0 ? t->nboxes : 1), 1);
    for (int64_t i = 0; i < t->M; i++) {
        const int j = t->cell2box[i];
        if ((j >= 0) != (t->triggered[i] != 0)) bad++;
        if (j >= 0) {
            if (j >= t->nboxes || t->box2cell[j] != (int)i) bad++;
            else if (seen[j]++) bad++;
        }
    }
    for (int v = 0; v < t->nvacant; v++) {
        const int j = t->vacant[v];
        if (j < 0 || j >= t->nboxes || seen[j]++) { bad++; continue; }
        if (t->box2cell[j] != -1) bad++;
        const REAL* q = SFX(box_plane)((SFX(otcm)*)t, j, 0);
        for (int k = 0; k < 2 * t->B3; k++) if (q[k] != 0) { bad++; break; }
    }
    for (int j = 0; j < t->nboxes; j++) if (!seen[j]) bad++;   /* every box is active or vacant */
    int64_t na = 0;
    for (int64_t i = 0; i < t->M; i++) na += t->triggered[i];
    if (na != t->nactive) bad++;
    free(seen);
    return bad;
}

/* ======================================================================= */
/* O3 (FP64 only): discrete adjoint of the dense leapfrog.                   */
/* ======================================================================= */
#if SFX_IS_F64
/* L u with zero ghosts (the 7-point Laplacian of eq.(3) without the C^2 factor) */
static void lap3_f64(int nx, int ny, int nz, const double* u, double* out)
{
    const size_t sy = (size_t)nx, sz = (size_t)nx * ny;
    #pragma omp parallel for schedule(static)
    for (int z = 0; z < nz; z++)
        for (int y = 0; y < ny; y++)
            for (int x = 0; x < nx; x++) {
                const size_t i = (size_t)z * sz + (size_t)y * sy + (size_t)x;
                const double xm = x > 0 ? u[i - 1] : 0.0, xp = x + 1 < nx ? u[i + 1] : 0.0;
                const double ym = y > 0 ? u[i - sy] : 0.0, yp = y + 1 < ny ? u[i + sy] : 0.0;
                const double zm = z > 0 ? u[i - sz] : 0.0, zp = z + 1 < nz ? u[i + sz] : 0.0;
                out[i] = (((xp + xm) + (yp + ym)) + (zp + zm)) - 6.0 * u[i];
            }
}

/* Gradient of J with respect to c for traces[n][r] = u^{n+1}[rec r]
 * (n = 0..nt-1) and dJ/dtraces = resid (nt x nrec).  Forward
 *   u^{n+1} = 2u^n - u^{n-1} + D L u^n + f^n,   D = diag((c dt/dx)^2),
 * adjoint in the mu = D lambda form, m = nt .. 1:
 *   mu^m = 2 mu^{m+1} - mu^{m+2} + D L mu^{m+1} + D R^T r^{m-1},
 *   dJ/dc_i = (2 / c_i) sum_m mu^m_i (L u^{m-1})_i     (0 where c_i = 0).
 * The forward is recomputed from checkpoints every ckpt steps. */
int oracle_adjoint_f64(int nx, int ny, int nz, const double* c, double dt, double dx,
                       int nsrc, const int64_t* src_idx, const int* src_t0, const int* src_ns,
                       const int64_t* src_off, const double* src_w,
                       int nrec, const int64_t* rec_idx, int nt, const double* resid,
                       int ckpt, double* grad)
{
    if (nt <= 0 || ckpt <= 0) return -1;
    const size_t N = (size_t)nx * ny * nz;
    const int nseg = (nt + ckpt - 1) / ckpt;
    double* D = (double*)malloc(N * sizeof(double));
    for (size_t i = 0; i < N; i++) { double t = c[i] * dt / dx; D[i] = t * t; }
    double* ck = (double*)malloc(N * sizeof(double) * 2 * (size_t)nseg);   /* (u^{kK}, u^{kK-1}) */
    double* seg = (double*)malloc(N * sizeof(double) * (size_t)(ckpt + 1)); /* u^{kK-1} .. u^{kK+K-1} */
    double* a = (double*)calloc(N, sizeof(double));
    double* b = (double*)calloc(N, sizeof(double));
    double* mu1 = (double*)calloc(N, sizeof(double));   /* mu^{m+1} */
    double* mu2 = (double*)calloc(N, sizeof(double));   /* mu^{m+2}, overwritten by mu^m */
    double* lu = (double*)malloc(N * sizeof(double));
    double* g = (double*)calloc(N, sizeof(double));
    if (!D || !ck || !seg || !a || !b || !mu1 || !mu2 || !lu || !g) return -7;
    /* forward pass, storing checkpoints; u^0 = u^{-1} = 0 */
    for (int k = 0; k < nseg; k++) {
        memcpy(ck + (size_t)(2 * k) * N, a, N * sizeof(double));
        memcpy(ck + (size_t)(2 * k + 1) * N, b, N * sizeof(double));
        const int n0 = k * ckpt;
        const int len = (n0 + ckpt <= nt ? ckpt : nt - n0);
        oracle_dense_f64(nx, ny, nz, 3, c, dt, dx, a, b, n0, len, nsrc, src_idx, src_t0, src_ns,
                         src_off, src_w, 0, NULL, NULL);
    }
    /* backward pass over the segments, last to first */
    for (int k = nseg - 1; k >= 0; k--) {
        const int n0 = k * ckpt;
        const int len = (n0 + ckpt <= nt ? ckpt : nt - n0);
        /* seg[j] = u^{n0 + j}, j = 0 .. len-1 (u^{n0} is the checkpoint's current level) */
        memcpy(a, ck + (size_t)(2 * k) * N, N * sizeof(double));
        memcpy(b, ck + (size_t)(2 * k + 1) * N, N * sizeof(double));
        memcpy(seg, a, N * sizeof(double));
        for (int j = 1; j < len; j++) {
            oracle_dense_f64(nx, ny, nz, 3, c, dt, dx, a, b, n0 + j - 1, 1, nsrc, src_idx, src_t0,
                             src_ns, src_off, src_w, 0, NULL, NULL);
            memcpy(seg + (size_t)j * N, a, N * sizeof(double));
        }
        for (int m = n0 + len; m > n0; m--) {
            /* mu^m from mu^{m+1} (mu1) and mu^{m+2} (mu2) */
            lap3_f64(nx, ny, nz, mu1, lu);
            #pragma omp parallel for schedule(static)
            for (size_t i = 0; i < N; i++) mu2[i] = (2.0 * mu1[i] - mu2[i]) + D[i] * lu[i];
            for (int r = 0; r < nrec; r++)
                mu2[rec_idx[r]] += D[rec_idx[r]] * resid[(size_t)(m - 1) * nrec + r];
            /* gradient term with L u^{m-1} */
            lap3_f64(nx, ny, nz, seg + (size_t)(m - 1 - n0) * N, lu);
            #pragma omp parallel for schedule(static)
            for (size_t i = 0; i < N; i++) g[i] += mu2[i] * lu[i];
            double* t = mu1; mu1 = mu2; mu2 = t;
        }
    }
    for (size_t i = 0; i < N; i++) grad[i] = c[i] != 0.0 ? (2.0 / c[i]) * g[i] : 0.0;
    free(D); free(ck); free(seg); free(a); free(b); free(mu1); free(mu2); free(lu); free(g);
    return 0;
}
#endif
