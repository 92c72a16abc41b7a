// C ABI of libpl.so: argument validation, context and scratch, item tables,
// hipGraph record/replay, and dispatch to the kernels.
#include <hip/hip_runtime.h>

#include <math.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <new>
#include <vector>

#include "pl_internal.h"

using namespace pl;

#define PL_TRY_HIP(expr)                        \
    do {                                        \
        hipError_t e_ = (expr);                 \
        if (e_ != hipSuccess) return PL_EHIP;   \
    } while (0)

namespace {

bool aligned(const void *p, size_t a) { return ((uintptr_t)p % a) == 0; }

bool finite_pos(double v) { return isfinite(v) && v > 0.0; }

pl_status validate_desc(const pl_init_desc *d)
{
    if (!d) return PL_EINVAL;
    if (d->ndim != 2 && d->ndim != 3) return PL_EINVAL;
    if (d->prec != PL_F64 && d->prec != PL_F32_OFFSET) return PL_EINVAL;
    if (d->shape != PL_CIC && d->shape != PL_TSC) return PL_EINVAL;
    if (d->algo != PL_ALGO_PLAIN && d->algo != PL_ALGO_TILED && d->algo != PL_ALGO_RUNS) return PL_EINVAL;
    if (d->algo == PL_ALGO_RUNS &&
        ((d->key_mode != PL_KEY_TILE_CELL && d->key_mode != PL_KEY_TILE_RUN) || d->max_np >= (int64_t)1 << 29))
        return PL_EINVAL;
    if (d->key_mode == PL_KEY_TILE_RUN && d->algo != PL_ALGO_RUNS) return PL_EINVAL;
    if (d->key_mode != PL_KEY_TILE && d->key_mode != PL_KEY_TILE_CELL && d->key_mode != PL_KEY_TILE_RANK &&
        d->key_mode != PL_KEY_TILE_RUN)
        return PL_EINVAL;
    if (!finite_pos(d->c)) return PL_EINVAL;
    if (d->nboxes < 1 || !d->boxes || d->nspecies < 1 || !d->species) return PL_EINVAL;
    if (d->max_items < 1 || d->max_items > 4096) return PL_EINVAL;
    if (d->max_np < 0 || d->max_np >= (int64_t)1 << 31) return PL_EINVAL;
    if (d->algo == PL_ALGO_RUNS) {
        if (d->block != 0 && d->block != 512) return PL_EINVAL;
    } else if (d->block != 0 && (d->block < 64 || d->block > 512 || d->block % 64)) {
        return PL_EINVAL;
    }
    for (int b = 0; b < d->nboxes; ++b) {
        const pl_box_desc &x = d->boxes[b];
        for (int a = 0; a < 3; ++a) {
            if (x.n[a] < 1 || x.n[a] > kMaxN) return PL_EINVAL;
            if (!finite_pos(x.dx[a])) return PL_EINVAL;
            if (x.tile[a] < 0 || (x.tile[a] > 0 && x.n[a] % x.tile[a] != 0)) return PL_EINVAL;
        }
        if (d->ndim == 2 && (x.n[2] != 1 || x.tile[2] > 1)) return PL_EINVAL;
        int zeros = (x.tile[0] == 0) + (x.tile[1] == 0) + (x.tile[2] == 0);
        if (zeros != 0 && zeros != 3) return PL_EINVAL;
    }
    for (int s = 0; s < d->nspecies; ++s) {
        const pl_species_desc &p = d->species[s];
        if (p.kind != PL_LORENTZ && p.kind != PL_DUST && p.kind != PL_TRACER) return PL_EINVAL;
        if (!finite_pos(p.m) || !isfinite(p.q) || !isfinite(p.weight)) return PL_EINVAL;
        if (p.kind == PL_DUST && !finite_pos(p.t_stop)) return PL_EINVAL;
        if (p.kind == PL_TRACER && p.rk_stages != 0 && p.rk_stages != 2 && p.rk_stages != 3) return PL_EINVAL;
    }
    return PL_OK;
}

// Largest divisor of n that is <= want.
int divisor_at_most(int n, int want)
{
    for (int t = std::min(n, want); t >= 1; --t)
        if (n % t == 0) return t;
    return 1;
}

void read_tune_cache(const char *path, int &block, int tile[3], int &runs, int &runs_block, int &one_launch)
{
    if (!path) return;
    FILE *f = fopen(path, "r");
    if (!f) return;
    char key[64];
    while (fscanf(f, "%63s", key) == 1) {
        if (!strcmp(key, "block")) {
            int v;
            if (fscanf(f, "%d", &v) == 1 && v >= 64 && v <= 512 && v % 64 == 0) block = v;
        } else if (!strcmp(key, "runs")) {
            int v;
            if (fscanf(f, "%d", &v) == 1) runs = v != 0;
        } else if (!strcmp(key, "one_launch")) {
            int v;
            if (fscanf(f, "%d", &v) == 1) one_launch = v != 0;
        } else if (!strcmp(key, "runs_block")) {
            int v;
            if (fscanf(f, "%d", &v) == 1 && v == 512) runs_block = v;
        } else if (!strcmp(key, "tile")) {
            int a, b, c;
            if (fscanf(f, "%d %d %d", &a, &b, &c) == 3 && a > 0 && b > 0 && c > 0) {
                tile[0] = a; tile[1] = b; tile[2] = c;
            }
        } else {
            int ch;
            while ((ch = fgetc(f)) != EOF && ch != '\n') {}
        }
    }
    fclose(f);
}

void free_ctx(Ctx *c)
{
    if (!c) return;
    for (auto &g : c->graphs) {
        if (g.exec) (void)hipGraphExecDestroy(g.exec);
        if (g.graph) (void)hipGraphDestroy(g.graph);
        if (g.table) (void)hipFree(g.table);
    }
    (void)hipFree(c->table);
    (void)hipFree(c->counters);
    (void)hipFree(c->errflags);
    (void)hipFree(c->sums);
    for (int k = 0; k < 2; ++k) {
        (void)hipFree(c->keys[k]);
        (void)hipFree(c->idx[k]);
    }
    (void)hipFree(c->hist);
    (void)hipFree(c->hist_scan);
    (void)hipFree(c->cell_start);
    for (int k = 0; k < Ctx::kRing; ++k)
        if (c->ring_ev[k]) (void)hipEventDestroy(c->ring_ev[k]);
    if (c->pinned) (void)hipHostFree(c->pinned);
    delete c;
}

// ---------------------------------------------------------------------------
// Item validation and descriptor construction
// ---------------------------------------------------------------------------

enum Mode { MODE_STEP, MODE_DEPOSIT, MODE_QUERY, MODE_SPECTRA };  // QUERY: sort, pack, sums, boundary

pl_status make_desc(const Ctx *c, const pl_item &it, double dt, Mode mode, bool deposit, ItemDesc &D)
{
    const pl_init_desc &d = c->d;
    if (it.box < 0 || it.box >= d.nboxes || it.species < 0 || it.species >= d.nspecies) return PL_EINVAL;
    const pl_box_desc &bx = d.boxes[it.box];
    const pl_species_desc &sp = d.species[it.species];
    const pl_particles &p = it.p;
    if (p.n < 0 || p.n > c->max_np) return PL_EINVAL;
    if (p.cur != 0 && p.cur != 1) return PL_EINVAL;
    const size_t es = d.prec == PL_F64 ? 8 : 4;
    const int cur = p.cur;
    const bool need = p.n > 0;
    auto chk = [&](const void *ptr, size_t al, bool required) {
        if (!ptr) return !required;
        return aligned(ptr, al);
    };
    if (d.prec == PL_F32_OFFSET && !chk(p.cell[cur], 4, need)) return PL_EINVAL;
    for (int a = 0; a < d.ndim; ++a)
        if (!chk(p.x[cur][a], es, need)) return PL_EINVAL;
    for (int a = 0; a < 3; ++a)
        if (!chk(p.u[cur][a], es, need)) return PL_EINVAL;
    if (!chk(p.w[cur], es, false)) return PL_EINVAL;
    int nfp = (p.fp[0] != nullptr) + (p.fp[1] != nullptr) + (p.fp[2] != nullptr);
    if (nfp != 0 && nfp != 3) return PL_EINVAL;
    for (int a = 0; a < 3; ++a)
        if (!chk(p.fp[a], es, false)) return PL_EINVAL;
    if (d.algo != PL_ALGO_PLAIN && !chk(p.tile_start, 4, true)) return PL_EINVAL;
    if (d.algo == PL_ALGO_RUNS && !chk(p.runs, 4, true)) return PL_EINVAL;
    if (!chk(p.id[cur], 8, false)) return PL_EINVAL;
    // spectral rows: both arrays or neither, float64 aligned
    if (p.nbins < 0 || p.nbins > kMaxBins) return PL_EINVAL;
    if ((p.eng[cur] != nullptr) != (p.chi[cur] != nullptr)) return PL_EINVAL;
    if (!chk(p.eng[cur], 8, false) || !chk(p.chi[cur], 8, false)) return PL_EINVAL;
    if (mode == MODE_SPECTRA) {
        if (p.nbins < 1 || !chk(p.eng[cur], 8, need) || !chk(p.chi[cur], 8, need)) return PL_EINVAL;
        for (int a = 0; a < 3; ++a)
            if (!chk(it.f.B[a], 8, true) || !chk(it.f.vg[a], 8, true)) return PL_EINVAL;
        if (!chk(it.f.divu, 8, true)) return PL_EINVAL;
    }

    // fields the kind reads (only when pushing)
    if (mode == MODE_STEP) {
        if (sp.kind == PL_LORENTZ) {
            for (int a = 0; a < 3; ++a)
                if (!chk(it.f.E[a], 8, true) || !chk(it.f.B[a], 8, true)) return PL_EINVAL;
        } else {
            for (int a = 0; a < 3; ++a)
                if (!chk(it.f.vg[a], 8, true)) return PL_EINVAL;
        }
    }
    // moment channels the kind defines
    const pl_moments &m = it.m;
    int nJ = (m.J[0] != nullptr) + (m.J[1] != nullptr) + (m.J[2] != nullptr);
    int nF = (m.F[0] != nullptr) + (m.F[1] != nullptr) + (m.F[2] != nullptr);
    if ((nJ != 0 && nJ != 3) || (nF != 0 && nF != 3)) return PL_EINVAL;
    double *M[kMaxCh] = {m.rho, m.J[0], m.J[1], m.J[2], m.F[0], m.F[1], m.F[2], m.eng};
    for (int ch = 0; ch < kMaxCh; ++ch)
        if (!chk(M[ch], 8, false)) return PL_EINVAL;
    if (sp.kind == PL_TRACER && (m.rho || nJ || nF || m.eng)) return PL_EINVAL;
    if (sp.kind == PL_DUST && (nJ || m.eng)) return PL_EINVAL;
    if (mode == MODE_DEPOSIT) {
        if (m.eng) return PL_EINVAL;
        if (nF && nfp != 3) return PL_EINVAL;
        if (nF && std::find(c->fp_stale.begin(), c->fp_stale.end(), (const void *)p.fp[0]) != c->fp_stale.end())
            return PL_EINVAL;
    }

    memset(&D, 0, sizeof(D));
    for (int a = 0; a < 3; ++a) {
        D.n[a] = bx.n[a];
        D.tile[a] = bx.tile[a];
        D.ntile[a] = bx.n[a] / bx.tile[a];
        D.dtdx[a] = dt / bx.dx[a];
        D.dtdx_f[a] = (float)D.dtdx[a];
    }
    D.ntiles = D.ntile[0] * D.ntile[1] * D.ntile[2];
    double dv = bx.dx[0] * bx.dx[1] * (d.ndim == 3 ? bx.dx[2] : 1.0);
    D.inv_dv = 1.0 / dv;
    D.kind = sp.kind;
    D.rk = (sp.kind == PL_TRACER && sp.rk_stages == 3) ? 3 : 2;
    D.q = sp.q;
    D.m = sp.m;
    D.wdef = sp.weight;
    D.h = (sp.q / sp.m) * dt * 0.5;
    D.inv_dt = dt != 0.0 ? 1.0 / dt : 0.0;
    D.c2 = d.c * d.c;
    D.inv_c2 = 1.0 / D.c2;
    if (sp.kind == PL_DUST) {
        D.decay = exp(-dt / sp.t_stop);
        D.one_m_decay = -expm1(-dt / sp.t_stop);
    }
    D.np = (int)p.n;
    D.cell = p.cell[cur];
    for (int a = 0; a < 3; ++a) {
        D.x[a] = a < d.ndim ? p.x[cur][a] : nullptr;
        D.u[a] = p.u[cur][a];
        D.fp[a] = p.fp[a];
        D.E[a] = it.f.E[a];
        D.B[a] = it.f.B[a];
        D.vg[a] = it.f.vg[a];
    }
    D.w = p.w[cur];
    D.id = p.id[cur];
    D.dt = dt;
    D.tile_start = p.tile_start;
    D.runs = p.runs;
    D.nb = p.eng[cur] ? p.nbins : 0;
    D.eng = p.eng[cur];
    D.chi = p.chi[cur];
    D.divu = it.f.divu;
    D.nslot = 0;
    for (int ch = 0; ch < kMaxCh; ++ch) {
        D.M[ch] = M[ch];
        D.slot[ch] = (deposit && M[ch]) ? D.nslot++ : -1;
    }
    return PL_OK;
}

// Build the descriptor list of a call: validated, ordered largest first, with
// work units assigned.  `order` maps table position -> caller index.
pl_status build_table(Ctx *c, const pl_item *items, int nitems, double dt, Mode mode, bool deposit,
                      std::vector<ItemDesc> &host, int &total_units)
{
    if (!items || nitems < 1 || nitems > c->d.max_items) return PL_EINVAL;
    std::vector<ItemDesc> descs(nitems);
    for (int i = 0; i < nitems; ++i) {
        pl_status st = make_desc(c, items[i], dt, mode, deposit, descs[i]);
        if (st != PL_OK) return st;
        descs[i].psum = c->sums + 16 * i + 8;
    }
    // items must not share particle storage
    for (int i = 0; i < nitems; ++i)
        for (int j = i + 1; j < nitems; ++j)
            if (descs[i].np > 0 && descs[j].np > 0 && descs[i].u[0] == descs[j].u[0]) return PL_EINVAL;
    // grouped by species kind (one launch per kind), largest items first
    std::vector<int> order(nitems);
    for (int i = 0; i < nitems; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
        if (descs[a].kind != descs[b].kind) return descs[a].kind < descs[b].kind;
        return descs[a].np > descs[b].np;
    });
    host.clear();
    total_units = 0;
    const bool tiled = c->d.algo != PL_ALGO_PLAIN;
    const int chunk = c->block * 4;
    // a fused run-based step whose LDS fits takes every kind in one launch
    // (units numbered across all items); otherwise one launch per kind
    bool one_launch = false;
    if (c->one_launch && c->d.algo == PL_ALGO_RUNS && mode == MODE_STEP && deposit) {
        std::vector<ItemDesc> all(nitems);
        for (int k = 0; k < nitems; ++k) all[k] = descs[order[k]];
        RunsPlan pl;
        one_launch = runs_plan(c, all.data(), nitems, pl);
    }
    int group_units = 0;
    for (int k = 0; k < nitems; ++k) {
        ItemDesc D = descs[order[k]];
        if (k > 0 && D.kind != host.back().kind && !one_launch) group_units = 0;
        D.unit_begin = group_units;
        D.chunk = chunk;
        D.nunits = tiled ? D.ntiles : (D.np + chunk - 1) / chunk;
        if (D.np == 0) D.nunits = 0;
        group_units += D.nunits;
        total_units += D.nunits;
        host.push_back(D);
    }
    return PL_OK;
}

// Stage the table through the pinned ring and queue its upload.
pl_status upload_table(Ctx *c, const std::vector<ItemDesc> &host, ItemDesc *dst)
{
    int slot = c->ring_pos;
    c->ring_pos = (c->ring_pos + 1) % Ctx::kRing;
    PL_TRY_HIP(hipEventSynchronize(c->ring_ev[slot]));
    ItemDesc *stage = c->pinned + (size_t)slot * c->d.max_items;
    memcpy(stage, host.data(), host.size() * sizeof(ItemDesc));
    PL_TRY_HIP(hipMemcpyAsync(dst, stage, host.size() * sizeof(ItemDesc), hipMemcpyHostToDevice, c->stream));
    PL_TRY_HIP(hipEventRecord(c->ring_ev[slot], c->stream));
    return PL_OK;
}

pl_status enqueue_step(Ctx *c, const ItemDesc *table, const std::vector<ItemDesc> &host, int total_units,
                       uint32_t flags, bool push, bool deposit)
{
    if (deposit && (flags & PL_ZERO_FIRST)) PL_TRY_HIP(launch_zero(c, table, host));
    if (flags & PL_SUMS) PL_TRY_HIP(launch_zero_sums(c, c->sums, 16 * c->d.max_items));
    hipError_t e = launch_step(c, table, host, (int)host.size(), total_units, flags, deposit, push);
    if (e == hipErrorInvalidConfiguration) return PL_EUNSUPPORTED;
    if (e != hipSuccess) return PL_EHIP;
    return PL_OK;
}

uint64_t fnv1a(const void *p, size_t n, uint64_t h)
{
    const unsigned char *b = (const unsigned char *)p;
    for (size_t i = 0; i < n; ++i) {
        h ^= b[i];
        h *= 1099511628211ull;
    }
    return h;
}

pl_status sort_args(const Ctx *c, const pl_item &it, SortArgs &a);

// One gather_push or deposit call: validate, optionally sort first, build the
// item table, then queue the launches directly or through a recorded graph.
pl_status run_call(Ctx *c, pl_item *items, int nitems, double dt, uint32_t flags, Mode mode)
{
    const bool push = mode == MODE_STEP;
    const bool deposit = mode == MODE_DEPOSIT || (flags & PL_FUSE_DEPOSIT);
    const bool sort_first = (flags & PL_SORT_FIRST) != 0;
    if (!items || nitems < 1 || nitems > c->d.max_items) return PL_EINVAL;
    // with PL_SORT_FIRST the step sees every item after its sort: the other set
    std::vector<SortArgs> sargs;
    std::vector<pl_item> sorted;
    const pl_item *step_items = items;
    if (sort_first) {
        if (!push || c->d.algo == PL_ALGO_PLAIN) return PL_EINVAL;
        sargs.resize(nitems);
        sorted.assign(items, items + nitems);
        for (int i = 0; i < nitems; ++i) {
            pl_status st = sort_args(c, items[i], sargs[i]);
            if (st != PL_OK) return st;
            sorted[i].p.cur = 1 - sorted[i].p.cur;
        }
        step_items = sorted.data();
    }
    std::vector<ItemDesc> host;
    int total = 0;
    pl_status st = build_table(c, step_items, nitems, dt, mode, deposit, host, total);
    if (st != PL_OK) return st;

    auto enqueue = [&](const ItemDesc *table) -> pl_status {
        for (const SortArgs &a : sargs)
            if (launch_sort(c, a) != hipSuccess) return PL_EHIP;
        return enqueue_step(c, table, host, total, flags, push, deposit);
    };
    // host bookkeeping once the launches are queued: the sort flipped the sets,
    // and this step rewrites p.fp in the items' (new) order
    auto done = [&]() {
        for (int i = 0; i < nitems; ++i) {
            if (sort_first) {
                items[i].p.cur = 1 - items[i].p.cur;
                c->stats[3]++;
            }
            if (push) {
                auto it = std::find(c->fp_stale.begin(), c->fp_stale.end(), (const void *)items[i].p.fp[0]);
                if (it != c->fp_stale.end()) c->fp_stale.erase(it);
            }
        }
        return PL_OK;
    };

    if (!(flags & PL_GRAPH)) {
        st = upload_table(c, host, c->table);
        if (st != PL_OK) return st;
        st = enqueue(c->table);
        return st == PL_OK ? done() : st;
    }

    if (!c->stream) return PL_EINVAL;   // the null stream cannot be captured
    uint64_t key = fnv1a(host.data(), host.size() * sizeof(ItemDesc), 1469598103934665603ull);
    uint32_t tag[2] = {flags, (uint32_t)mode};
    key = fnv1a(tag, sizeof(tag), key);
    if (!sargs.empty()) key = fnv1a(sargs.data(), sargs.size() * sizeof(SortArgs), key);
    c->use_clock++;
    for (auto &g : c->graphs) {
        if (g.valid && g.key == key && g.nitems == (int)host.size()) {
            g.last_use = c->use_clock;
            PL_TRY_HIP(hipGraphLaunch(g.exec, c->stream));
            c->stats[1]++;
            return done();
        }
    }
    // record a new graph in the least recently used slot
    GraphEntry *slot = &c->graphs[0];
    for (auto &g : c->graphs) {
        if (!g.valid) { slot = &g; break; }
        if (g.last_use < slot->last_use) slot = &g;
    }
    if (slot->exec) { (void)hipGraphExecDestroy(slot->exec); slot->exec = nullptr; }
    if (slot->graph) { (void)hipGraphDestroy(slot->graph); slot->graph = nullptr; }
    slot->valid = false;
    // the graph's own table: written now, read by every replay
    PL_TRY_HIP(hipStreamSynchronize(c->stream));
    PL_TRY_HIP(hipMemcpy(slot->table, host.data(), host.size() * sizeof(ItemDesc), hipMemcpyHostToDevice));
    PL_TRY_HIP(hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
    pl_status est = enqueue(slot->table);
    hipGraph_t graph = nullptr;
    hipError_t ce = hipStreamEndCapture(c->stream, &graph);
    if (est != PL_OK) {
        if (graph) (void)hipGraphDestroy(graph);
        return est;
    }
    if (ce != hipSuccess) return PL_EHIP;
    hipGraphExec_t exec = nullptr;
    if (hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0) != hipSuccess) {
        (void)hipGraphDestroy(graph);
        return PL_EHIP;
    }
    slot->graph = graph;
    slot->exec = exec;
    slot->key = key;
    slot->nitems = (int)host.size();
    slot->valid = true;
    slot->last_use = c->use_clock;
    c->stats[2]++;
    PL_TRY_HIP(hipGraphLaunch(exec, c->stream));
    c->stats[1]++;
    return done();
}

}  // namespace

// ---------------------------------------------------------------------------
// Exported entry points
// ---------------------------------------------------------------------------

extern "C" {

pl_status pl_part_init(pl_ctx **out, const pl_init_desc *d)
{
    if (!out) return PL_EINVAL;
    *out = nullptr;
    pl_status st = validate_desc(d);
    if (st != PL_OK) return st;
    Ctx *c = new (std::nothrow) Ctx();
    if (!c) return PL_ENOMEM;
    c->d = *d;
    c->d.tune_cache = nullptr;
    c->boxes.assign(d->boxes, d->boxes + d->nboxes);
    c->species.assign(d->species, d->species + d->nspecies);
    c->d.boxes = c->boxes.data();
    c->d.species = c->species.data();
    c->stream = (hipStream_t)d->stream;
    c->max_np = d->max_np;
    c->fp_stale.reserve(4 * (size_t)d->max_items + 16);

    int tuned_block = 256, tuned_tile[3] = {8, 8, 8}, tuned_runs = 0, tuned_runs_block = 512, tuned_one = 1;
    if (d->prec == PL_F64 && d->algo == PL_ALGO_TILED) { tuned_tile[1] = 4; tuned_tile[2] = 4; }
    if (d->prec == PL_F64 && d->algo == PL_ALGO_RUNS) tuned_tile[2] = 4;
    read_tune_cache(d->tune_cache, tuned_block, tuned_tile, tuned_runs, tuned_runs_block, tuned_one);
    c->one_launch = tuned_one != 0;
    const bool runs_algo = d->algo == PL_ALGO_RUNS;
    c->block = (d->block && !runs_algo) ? d->block : tuned_block;
    c->runs = tuned_runs != 0;
    c->runs_block = (d->block && runs_algo) ? d->block : tuned_runs_block;
    for (auto &b : c->boxes) {
        if (b.tile[0] == 0) {
            for (int a = 0; a < 3; ++a) b.tile[a] = divisor_at_most(b.n[a], tuned_tile[a]);
            if (d->ndim == 2) b.tile[2] = 1;
        }
        c->max_ntiles = std::max(c->max_ntiles, (b.n[0] / b.tile[0]) * (b.n[1] / b.tile[1]) * (b.n[2] / b.tile[2]));
        if (d->algo == PL_ALGO_RUNS && b.tile[0] * b.tile[1] * b.tile[2] > kRunsMaxTileCells) {
            delete c;
            return PL_EUNSUPPORTED;
        }
    }
    int64_t max_cells = 0;
    for (const auto &b : c->boxes) {
        max_cells = std::max<int64_t>(max_cells, (int64_t)b.n[0] * b.n[1] * b.n[2]);
        if (d->key_mode == PL_KEY_TILE_RANK) {
            // tile bits + cell-in-tile bits must leave at least 3 bits for the rank
            int64_t nt = (int64_t)(b.n[0] / b.tile[0]) * (b.n[1] / b.tile[1]) * (b.n[2] / b.tile[2]);
            int64_t pt = (int64_t)b.tile[0] * b.tile[1] * b.tile[2];
            int tb = 0, cb = 0;
            while (((int64_t)1 << tb) < nt) ++tb;
            while (((int64_t)1 << cb) < pt) ++cb;
            if (32 - tb - cb < 3) {
                delete c;
                return PL_EUNSUPPORTED;
            }
        }
    }

    if (hipGetDevice(&c->device) != hipSuccess ||
        hipDeviceGetAttribute(&c->num_cu, hipDeviceAttributeMultiprocessorCount, c->device) != hipSuccess ||
        hipDeviceGetAttribute(&c->lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, c->device) != hipSuccess) {
        delete c;
        return PL_EHIP;
    }
    if (c->num_cu < 1) c->num_cu = 1;

    const size_t mi = (size_t)d->max_items;
    const size_t np = (size_t)std::max<int64_t>(d->max_np, 1);
    const size_t nblocks = (np + 8191) / 8192;
    c->hist_cap = (int64_t)((nblocks << kMaxDigitBits) + 1024);    // digit-major counts of one radix pass
    bool ok = hipMalloc(&c->table, mi * sizeof(ItemDesc)) == hipSuccess &&
              hipMalloc(&c->counters, kCounterSlots * sizeof(unsigned)) == hipSuccess &&
              hipMalloc(&c->errflags, 4 * sizeof(int)) == hipSuccess &&
              hipMalloc(&c->sums, 16 * mi * sizeof(double)) == hipSuccess &&
              hipMalloc(&c->hist, (size_t)c->hist_cap * sizeof(uint32_t)) == hipSuccess &&
              hipMalloc(&c->hist_scan, (size_t)c->hist_cap * sizeof(uint32_t)) == hipSuccess &&
              hipHostMalloc(&c->pinned, Ctx::kRing * mi * sizeof(ItemDesc), hipHostMallocDefault) == hipSuccess;
    for (int k = 0; ok && k < 2; ++k)
        ok = hipMalloc(&c->keys[k], np * sizeof(uint32_t)) == hipSuccess &&
             hipMalloc(&c->idx[k], np * sizeof(uint32_t)) == hipSuccess;
    if (ok && d->key_mode == PL_KEY_TILE_RANK)
        ok = hipMalloc(&c->cell_start, (size_t)max_cells * sizeof(int32_t)) == hipSuccess;
    for (int k = 0; ok && k < Ctx::kGraphs; ++k)
        ok = hipMalloc(&c->graphs[k].table, mi * sizeof(ItemDesc)) == hipSuccess;
    for (int k = 0; ok && k < Ctx::kRing; ++k)
        ok = hipEventCreateWithFlags(&c->ring_ev[k], hipEventDisableTiming) == hipSuccess;
    if (!ok) {
        free_ctx(c);
        return PL_ENOMEM;
    }
    if (hipMemset(c->counters, 0, kCounterSlots * sizeof(unsigned)) != hipSuccess ||
        hipMemset(c->errflags, 0, 4 * sizeof(int)) != hipSuccess ||
        hipMemset(c->sums, 0, 16 * mi * sizeof(double)) != hipSuccess || hipDeviceSynchronize() != hipSuccess) {
        free_ctx(c);
        return PL_EHIP;
    }
    *out = reinterpret_cast<pl_ctx *>(c);
    return PL_OK;
}

pl_status pl_part_gather_push(pl_ctx *ctx, pl_item *items, int nitems, double dt, uint32_t flags)
{
    Ctx *c = reinterpret_cast<Ctx *>(ctx);
    if (!c || !isfinite(dt) || dt == 0.0) return PL_EINVAL;
    if (flags & ~(PL_FUSE_DEPOSIT | PL_ZERO_FIRST | PL_GRAPH | PL_SUMS | PL_SORT_FIRST)) return PL_EINVAL;
    return run_call(c, items, nitems, dt, flags, MODE_STEP);
}

pl_status pl_part_deposit(pl_ctx *ctx, const pl_item *items, int nitems, uint32_t flags)
{
    Ctx *c = reinterpret_cast<Ctx *>(ctx);
    if (!c) return PL_EINVAL;
    if (flags & ~(PL_ZERO_FIRST | PL_GRAPH)) return PL_EINVAL;
    return run_call(c, const_cast<pl_item *>(items), nitems, 0.0, flags, MODE_DEPOSIT);
}

}  // extern "C"

namespace {

// Validate one item of a sort call and describe it to the sort launcher.
pl_status sort_args(const Ctx *c, const pl_item &it, SortArgs &a)
{
    const bool f64 = c->d.prec == PL_F64;
    const size_t es = f64 ? 8 : 4;
    {
        ItemDesc D;
        pl_status st = make_desc(c, it, 1.0, MODE_QUERY, false, D);
        if (st != PL_OK) return st;
        const pl_particles &p = it.p;
        if (!p.tile_start || !aligned(p.tile_start, 4)) return PL_EINVAL;
        if (c->d.algo == PL_ALGO_RUNS && !p.runs) return PL_EINVAL;
        const int cur = p.cur, nxt = 1 - p.cur;
        memset(&a, 0, sizeof(a));
        a.prec = c->d.prec;
        a.ndim = c->d.ndim;
        a.key_mode = c->d.key_mode;
        for (int k = 0; k < 3; ++k) {
            a.n[k] = D.n[k];
            a.tile[k] = D.tile[k];
            a.x[k] = (f64 && k < c->d.ndim) ? (const double *)p.x[cur][k] : nullptr;
        }
        a.np = D.np;
        a.ntiles = D.ntiles;
        a.cell = p.cell[cur];
        a.tile_start = p.tile_start;
        a.runs = c->d.algo == PL_ALGO_RUNS ? p.runs : nullptr;
        auto add = [&](const void *s, void *dd, int esz) -> bool {
            if (!s) return true;
            if (!dd || !aligned(dd, (size_t)esz) || a.narrays >= SortArgs::kMaxArrays) return false;
            a.src[a.narrays] = s;
            a.dst[a.narrays] = dd;
            a.esize[a.narrays] = esz;
            a.narrays++;
            return true;
        };
        bool ok = true;
        if (!f64) ok = ok && add(p.cell[cur], p.cell[nxt], 4);
        for (int k = 0; k < c->d.ndim; ++k) ok = ok && add(p.x[cur][k], p.x[nxt][k], (int)es);
        for (int k = 0; k < 3; ++k) ok = ok && add(p.u[cur][k], p.u[nxt][k], (int)es);
        ok = ok && add(p.w[cur], p.w[nxt], (int)es);
        ok = ok && add(p.id[cur], p.id[nxt], 8);
        if (p.id[cur] && !aligned(p.id[cur], 8)) ok = false;
        if (!ok) return PL_EINVAL;
        if (D.nb > 0) {
            // the spectral rows move with their particles
            if (!p.eng[nxt] || !p.chi[nxt] || !aligned(p.eng[nxt], 8) || !aligned(p.chi[nxt], 8)) return PL_EINVAL;
            a.nb = D.nb;
            a.rsrc[0] = p.eng[cur];
            a.rsrc[1] = p.chi[cur];
            a.rdst[0] = p.eng[nxt];
            a.rdst[1] = p.chi[nxt];
        }
    }
    return PL_OK;
}

}  // namespace

extern "C" {

pl_status pl_part_sort(pl_ctx *ctx, pl_item *items, int nitems)
{
    Ctx *c = reinterpret_cast<Ctx *>(ctx);
    if (!c || !items || nitems < 1 || nitems > c->d.max_items) return PL_EINVAL;
    std::vector<SortArgs> args(nitems);
    for (int i = 0; i < nitems; ++i) {
        pl_status st = sort_args(c, items[i], args[i]);
        if (st != PL_OK) return st;
    }
    for (int i = 0; i < nitems; ++i) {
        if (launch_sort(c, args[i]) != hipSuccess) return PL_EHIP;
        items[i].p.cur = 1 - items[i].p.cur;
        c->stats[3]++;
        const void *fp = items[i].p.fp[0];
        if (fp && std::find(c->fp_stale.begin(), c->fp_stale.end(), fp) == c->fp_stale.end()) {
            // bounded: the oldest entry goes first
            if (c->fp_stale.size() >= c->fp_stale.capacity()) c->fp_stale.erase(c->fp_stale.begin());
            c->fp_stale.push_back(fp);
        }
    }
    return PL_OK;
}

pl_status pl_part_spectra(pl_ctx *ctx, const pl_item *items, int nitems, double dt, const pl_spectra_desc *sd)
{
    Ctx *c = reinterpret_cast<Ctx *>(ctx);
    if (!c || !sd || !items || nitems < 1 || nitems > c->d.max_items) return PL_EINVAL;
    if (!isfinite(dt) || dt == 0.0) return PL_EINVAL;
    if (!isfinite(sd->cr) || !isfinite(sd->u_rad) || !isfinite(sd->ub) || sd->cr < 0.0 || sd->u_rad < 0.0 ||
        sd->ub < 0.0)
        return PL_EINVAL;
    std::vector<ItemDesc> host(nitems);
    int units = 0;
    for (int i = 0; i < nitems; ++i) {
        pl_status st = make_desc(c, items[i], dt, MODE_SPECTRA, false, host[i]);
        if (st != PL_OK) return st;
        host[i].unit_begin = units;
        host[i].nunits = host[i].np > 0 ? (host[i].np + 255) / 256 : 0;
        units += host[i].nunits;
    }
    pl_status st = upload_table(c, host, c->table);
    if (st != PL_OK) return st;
    hipError_t e = launch_spectra(c, c->table, host, sd->cr, sd->u_rad, sd->ub);
    if (e == hipErrorInvalidConfiguration) return PL_EUNSUPPORTED;
    return e == hipSuccess ? PL_OK : PL_EHIP;
}

pl_status pl_part_boundary(pl_ctx *ctx, pl_item *items, int nitems, const pl_boundary_desc *bc, int64_t *removed)
{
    Ctx *c = reinterpret_cast<Ctx *>(ctx);
    if (!c || !bc || !items || nitems < 1 || nitems > c->d.max_items) return PL_EINVAL;
    std::vector<ItemDesc> descs(nitems);
    for (int i = 0; i < nitems; ++i) {
        pl_status st = make_desc(c, items[i], 1.0, MODE_QUERY, false, descs[i]);
        if (st != PL_OK) return st;
        for (int d = 0; d < c->d.ndim; ++d)
            if (bc->open[d] && (bc->ghost < 2 || 2 * bc->ghost >= descs[i].n[d])) return PL_EINVAL;
    }
    for (int i = 0; i < nitems; ++i) {
        int64_t keep = 0, gone = 0;
        if (launch_boundary(c, descs[i], *bc, c->d.ndim, &keep, &gone) != hipSuccess) return PL_EHIP;
        items[i].p.n = keep;
        if (removed) removed[i] = gone;
        const void *fp = items[i].p.fp[0];
        if (gone > 0 && fp && std::find(c->fp_stale.begin(), c->fp_stale.end(), fp) == c->fp_stale.end()) {
            if (c->fp_stale.size() >= c->fp_stale.capacity()) c->fp_stale.erase(c->fp_stale.begin());
            c->fp_stale.push_back(fp);
        }
    }
    return PL_OK;
}

pl_status pl_part_inject(pl_ctx *ctx, pl_item *item, int64_t k, const double *x[3], const double *u[3],
                         const double *w, const uint64_t *id, const double *eng, const double *chi, int64_t cap)
{
    Ctx *c = reinterpret_cast<Ctx *>(ctx);
    if (!c || !item || !x || !u || k < 0) return PL_EINVAL;
    ItemDesc D;
    pl_status st = make_desc(c, *item, 1.0, MODE_QUERY, false, D);
    if (st != PL_OK) return st;
    const int64_t n = item->p.n;
    if (n + k > cap || n + k > c->max_np) return PL_EINVAL;
    if (k == 0) return PL_OK;
    // the destination set must hold every array the item carries
    const int cur = item->p.cur;
    if ((c->d.prec == PL_F32_OFFSET && !item->p.cell[cur]) || !item->p.u[cur][0]) return PL_EINVAL;
    for (int a = 0; a < c->d.ndim; ++a)
        if (!item->p.x[cur][a]) return PL_EINVAL;
    const double *xs[3] = {nullptr, nullptr, nullptr}, *us[3];
    for (int a = 0; a < 3; ++a) {
        if (a < c->d.ndim) {
            if (!x[a] || !aligned(x[a], 8)) return PL_EINVAL;
            xs[a] = x[a];
        }
        if (!u[a] || !aligned(u[a], 8)) return PL_EINVAL;
        us[a] = u[a];
    }
    if (!aligned(w, 8) || !aligned(id, 8) || !aligned(eng, 8) || !aligned(chi, 8)) return PL_EINVAL;
    if (D.nb > 0 && (!eng || !chi)) return PL_EINVAL;
    // positions and velocities through the pack kernel, at [n, n + k)
    const size_t es = c->d.prec == PL_F64 ? 8 : 4;
    ItemDesc T = D;
    T.np = (int)k;
    if (T.cell) T.cell += n;
    for (int a = 0; a < 3; ++a) {
        if (T.x[a]) T.x[a] = static_cast<char *>(T.x[a]) + n * es;
        T.u[a] = static_cast<char *>(T.u[a]) + n * es;
    }
    if (launch_pack(c, T, c->d.prec, c->d.ndim, xs, us) != hipSuccess) return PL_EHIP;
    const pl_species_desc &sp = c->d.species[item->species];
    if (launch_inject_rest(c, D, k, w, D.w != nullptr, sp.weight, id, D.id, eng, chi) != hipSuccess) return PL_EHIP;
    item->p.n = n + k;
    return PL_OK;
}

pl_status pl_sort_noalloc(const pl_init_desc *d, pl_item *items, int nitems)
{
    pl_status st = validate_desc(d);
    if (st != PL_OK) return st;
    if (!items || nitems < 1 || nitems > d->max_items) return PL_EINVAL;
    if (d->key_mode == PL_KEY_TILE_RANK) return PL_EUNSUPPORTED;       // needs per-cell scratch
    for (int b = 0; b < d->nboxes; ++b)
        if (d->boxes[b].tile[0] == 0) return PL_EINVAL;                 // no tune cache here: tiles are given
    for (int i = 0; i < nitems; ++i)
        if (items[i].p.n > PL_NOALLOC_MAX_NP) return PL_ENOSPACE;
    // a context on the stack that only carries the description: nothing is
    // allocated, the sort scratch is the library's fixed device array
    Ctx c;
    c.d = *d;
    c.max_np = d->max_np;
    c.stream = (hipStream_t)d->stream;
    SortArgs a[8];
    for (int i0 = 0; i0 < nitems; i0 += 8) {
        const int i1 = std::min(nitems, i0 + 8);
        for (int i = i0; i < i1; ++i) {
            st = sort_args(&c, items[i], a[i - i0]);
            if (st != PL_OK) return st;
        }
        for (int i = i0; i < i1; ++i) {
            hipError_t e = launch_sort_noalloc(&c, a[i - i0]);
            if (e == hipErrorInvalidDevice) return PL_EUNSUPPORTED;
            if (e != hipSuccess) return PL_EHIP;
            items[i].p.cur = 1 - items[i].p.cur;
        }
    }
    return PL_OK;
}

pl_status pl_part_pack(pl_ctx *ctx, const pl_item *item, const double *x[3], const double *u[3])
{
    Ctx *c = reinterpret_cast<Ctx *>(ctx);
    if (!c || !item || !x || !u) return PL_EINVAL;
    ItemDesc D;
    pl_status st = make_desc(c, *item, 1.0, MODE_QUERY, false, D);
    if (st != PL_OK) return st;
    const double *xs[3] = {nullptr, nullptr, nullptr}, *us[3];
    for (int a = 0; a < 3; ++a) {
        if (a < c->d.ndim) {
            if ((D.np > 0 && !x[a]) || !aligned(x[a], 8)) return PL_EINVAL;
            xs[a] = x[a];
        }
        if ((D.np > 0 && !u[a]) || !aligned(u[a], 8)) return PL_EINVAL;
        us[a] = u[a];
    }
    return launch_pack(c, D, c->d.prec, c->d.ndim, xs, us) == hipSuccess ? PL_OK : PL_EHIP;
}

pl_status pl_part_unpack(pl_ctx *ctx, const pl_item *item, double *x[3], double *u[3])
{
    Ctx *c = reinterpret_cast<Ctx *>(ctx);
    if (!c || !item || !x || !u) return PL_EINVAL;
    ItemDesc D;
    pl_status st = make_desc(c, *item, 1.0, MODE_QUERY, false, D);
    if (st != PL_OK) return st;
    double *xs[3] = {nullptr, nullptr, nullptr}, *us[3];
    for (int a = 0; a < 3; ++a) {
        if (a < c->d.ndim) {
            if ((D.np > 0 && !x[a]) || !aligned(x[a], 8)) return PL_EINVAL;
            xs[a] = x[a];
        }
        if ((D.np > 0 && !u[a]) || !aligned(u[a], 8)) return PL_EINVAL;
        us[a] = u[a];
    }
    return launch_unpack(c, D, c->d.prec, c->d.ndim, xs, us) == hipSuccess ? PL_OK : PL_EHIP;
}

pl_status pl_part_sums(pl_ctx *ctx, const pl_item *items, int nitems, double *out)
{
    Ctx *c = reinterpret_cast<Ctx *>(ctx);
    if (!c || !items || !out || nitems < 1 || nitems > c->d.max_items) return PL_EINVAL;
    std::vector<ItemDesc> descs(nitems);
    for (int i = 0; i < nitems; ++i) {
        pl_status st = make_desc(c, items[i], 1.0, MODE_QUERY, true, descs[i]);
        if (st != PL_OK) return st;
    }
    for (int i = 0; i < nitems; ++i) {
        PL_TRY_HIP(launch_zero_sums(c, c->sums + 16 * i, 8));
        PL_TRY_HIP(launch_grid_sums(c, descs[i], c->sums + 16 * i));
    }
    PL_TRY_HIP(hipMemcpyAsync(out, c->sums, 16 * (size_t)nitems * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    PL_TRY_HIP(hipStreamSynchronize(c->stream));
    return PL_OK;
}

pl_status pl_part_sync(pl_ctx *ctx)
{
    Ctx *c = reinterpret_cast<Ctx *>(ctx);
    if (!c) return PL_EINVAL;
    PL_TRY_HIP(hipStreamSynchronize(c->stream));
    int flags = 0;
    PL_TRY_HIP(hipMemcpy(&flags, c->errflags, sizeof(int), hipMemcpyDeviceToHost));
    if (flags) PL_TRY_HIP(hipMemset(c->errflags, 0, sizeof(int)));
    if (flags & ERR_UNSORTED) return PL_ENOTSORTED;
    if (flags & ERR_NONFINITE) return PL_ENONFINITE;
    if (flags & ERR_CFL) return PL_ECFL;
    return PL_OK;
}

pl_status pl_part_set_stream(pl_ctx *ctx, void *stream)
{
    Ctx *c = reinterpret_cast<Ctx *>(ctx);
    if (!c) return PL_EINVAL;
    PL_TRY_HIP(hipStreamSynchronize(c->stream));
    for (auto &g : c->graphs) {
        if (g.exec) (void)hipGraphExecDestroy(g.exec);
        if (g.graph) (void)hipGraphDestroy(g.graph);
        g.exec = nullptr;
        g.graph = nullptr;
        g.valid = false;
    }
    c->stream = (hipStream_t)stream;
    return PL_OK;
}

pl_status pl_part_stats(pl_ctx *ctx, int64_t *out, int n)
{
    Ctx *c = reinterpret_cast<Ctx *>(ctx);
    if (!c || !out || n < 0) return PL_EINVAL;
    for (int k = 0; k < n && k < PL_NSTATS; ++k) out[k] = c->stats[k];
    return PL_OK;
}

void pl_part_finalize(pl_ctx *ctx)
{
    Ctx *c = reinterpret_cast<Ctx *>(ctx);
    if (!c) return;
    (void)hipStreamSynchronize(c->stream);
    free_ctx(c);
}

const char *pl_status_string(pl_status s)
{
    switch (s) {
    case PL_OK: return "success";
    case PL_EINVAL: return "invalid argument";
    case PL_ENOMEM: return "out of memory";
    case PL_EHIP: return "HIP runtime error";
    case PL_EUNSUPPORTED: return "unsupported request";
    case PL_ECFL: return "a particle moved a full cell or more in one step";
    case PL_ENONFINITE: return "non-finite or out-of-range particle coordinate";
    case PL_ENOSPACE: return "the request exceeds the fixed scratch of pl_sort_noalloc";
    case PL_ENOTSORTED: return "an item's tile offsets or run table do not cover its particles (sort it first)";
    default: return "unknown status";
    }
}

}  // extern "C"
