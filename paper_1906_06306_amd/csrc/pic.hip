// libpic: C ABI of the MI355X relativistic PIC step (see include/pic.h).
//
// Host side: configuration checks, workspace layout, tile tables and kernel
// launches on the context's stream.  All device memory belongs to the
// caller's workspace; nothing here allocates device memory.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <limits>
#include <mutex>
#include <string>
#include <type_traits>
#include <vector>

#include "../../include/pic.h"
#include "pic_adjoint.hpp"
#include "pic_aux_kernels.hpp"

using pic::Params;
using pic::TileDesc;

// particles per thread per group in the fused push kernel
#ifndef PUSH_UNROLL
#define PUSH_UNROLL 1
#endif

namespace {

// largest segment or outbox capacity: the push addresses slots by 32-bit
// byte offsets from the segment's base, 8 * 2^28 bytes at FP64
constexpr int64_t MAX_SLOTS = int64_t(1) << 28;

// the segments' visiting order (largest first) only balances the push: any
// permutation gives the same results, and counts change by a few percent a
// step, so it is recomputed every ORDER_EVERY pushes, at the first push after
// init or an injection, and at every push captured into a graph
constexpr int ORDER_EVERY = 8;

// text of the last error on this thread (a fixed buffer: reporting an
// error allocates nothing)
thread_local char g_last_error[512];

// Device scratch of pic_diagnostics_static, the diagnostics for callers that
// cannot allocate memory: the per-tile partial sums, the per-tile charge
// blocks and the reduced record.  Every device the library runs on holds
// one copy until the process ends; host code reaches a device's copy only
// through the address hipGetSymbolAddress returns for it (per device, at
// pic_init_tiles), never through the symbol itself.
constexpr uint64_t STATIC_SCRATCH_BYTES = uint64_t(16) << 20;
static __device__ __align__(256) unsigned char scratch[STATIC_SCRATCH_BYTES];

std::mutex g_scratch_mu;
std::vector<void *> g_scratch_dev;   // device id -> address of that device's scratch

pic_status fail(pic_status code, const char *fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_last_error, sizeof g_last_error, fmt, ap);
    va_end(ap);
    return code;
}

#define HIP_OK(expr)                                                                          \
    do {                                                                                      \
        hipError_t e_ = (expr);                                                               \
        if (e_ != hipSuccess) return fail(PIC_E_HIP, "%s: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

uint64_t align256(uint64_t v) { return (v + 255) & ~uint64_t(255); }

// Address of the current device's copy of `scratch` (looked up once per
// device, with that device current).
pic_status scratch_address(void **out)
{
    int dev = 0;
    HIP_OK(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if ((int)g_scratch_dev.size() <= dev) g_scratch_dev.resize(dev + 1, nullptr);
    if (!g_scratch_dev[dev]) {
        void *p = nullptr;
        HIP_OK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) return fail(PIC_E_HIP, "hipGetSymbolAddress returned a null address for the static scratch");
        g_scratch_dev[dev] = p;
    }
    *out = g_scratch_dev[dev];
    return PIC_OK;
}
int64_t round_up(int64_t v, int64_t m) { return (v + m - 1) / m * m; }

// Internal layout: the public offsets plus the staging regions.
struct Layout {
    pic_layout pub;
    uint64_t off_tmp, off_jblk, off_rblk, off_part, off_ob_pos, off_ob_u, off_ob_dir, off_ob_cnt;
    uint64_t off_tiles, off_charge, off_qm, off_mass, off_order, off_queue;
    uint64_t off_key, off_xl, off_hist;
    uint64_t off_ob_ids, off_adj_lj, off_adj_eblk, off_adj_bblk, off_ob_boff, off_ob_idx, off_jtmp, off_rho_prev;
    uint64_t off_nf_pre;
    int64_t fblk_cells, n_input;
    int64_t jblk_cells, rblk_cells, max_count, max_ntb, nchunks_max, ob_dir_stride;
    int32_t order_shift;   // segment counts are bucketed by count >> order_shift for the dispatch order
    std::vector<TileDesc> tiles;
    std::vector<int64_t> seg_off;
    std::vector<int32_t> seg_cap;
    std::vector<int64_t> box_cell0, box_tile0;
    std::vector<int32_t> order;
};

int dims_of(const pic_config *c, int b, int d) { return d < c->dim ? c->box_cells[3 * b + d] : 1; }

pic_status check_config(const pic_config *c)
{
    if (!c) return fail(PIC_E_ARG, "null config");
    if (c->dim < 1 || c->dim > 3) return fail(PIC_E_ARG, "dim must be 1, 2 or 3 (got %d)", c->dim);
    if (c->precision != PIC_FP32 && c->precision != PIC_FP64) return fail(PIC_E_ARG, "precision must be PIC_FP32 or PIC_FP64");
    if (c->n_species < 1 || c->n_species > PIC_MAX_SPECIES) return fail(PIC_E_ARG, "n_species must be 1..%d", PIC_MAX_SPECIES);
    if (c->n_boxes < 1) return fail(PIC_E_ARG, "n_boxes must be >= 1");
    if (!c->box_cells || !c->charge || !c->qm || !c->mass) return fail(PIC_E_ARG, "box_cells, charge, qm and mass are required");
    if (!(c->cfl > 0.0) || c->cfl * std::sqrt((double)c->dim) > 1.0) return fail(PIC_E_ARG, "cfl must satisfy 0 < c <= 1/sqrt(D)");
    if (c->pusher < PIC_PUSHER_BORIS || c->pusher > PIC_PUSHER_HC) return fail(PIC_E_ARG, "unknown pusher %d", c->pusher);
    if (c->filter_passes < 0) return fail(PIC_E_ARG, "filter_passes must be >= 0");
    if (c->fdtd_order != 0 && c->fdtd_order != 2 && c->fdtd_order != 4) return fail(PIC_E_ARG, "fdtd_order must be 2 or 4");
    for (int b = 0; c->fdtd_order == 4 && c->box_walls && b < c->n_boxes; ++b)
        if (c->box_walls[b] & PIC_WALL_X) return fail(PIC_E_ARG, "FDTD4 covers periodic boxes only");
    for (int b = 0; c->filter_passes > 0 && c->box_walls && b < c->n_boxes; ++b)
        if (c->box_walls[b] & PIC_WALL_X) return fail(PIC_E_ARG, "the current filter covers periodic boxes only");
    int blk = c->block ? c->block : 256;
    if (blk < 64 || blk > 1024 || blk % 64) return fail(PIC_E_ARG, "block must be a multiple of 64 in 64..1024");
    for (int d = 0; d < 3; ++d) {
        if (d < c->dim) {
            if (c->tile[d] < 2 || c->tile[d] % 2) return fail(PIC_E_ARG, "tile[%d] must be even and >= 2", d);
        } else if (c->tile[d] != 1) {
            return fail(PIC_E_ARG, "tile[%d] must be 1 beyond dim", d);
        }
    }
    for (int b = 0; b < c->n_boxes; ++b)
        for (int d = 0; d < c->dim; ++d) {
            int n = c->box_cells[3 * b + d];
            if (n < c->tile[d] || n % c->tile[d]) return fail(PIC_E_ARG, "tile[%d]=%d does not divide box %d (n=%d)", d, c->tile[d], b, n);
        }
    return PIC_OK;
}

pic_status make_layout(const pic_config *c, const int64_t *counts, Layout &L)
{
    pic_status st = check_config(c);
    if (st) return st;
    if (!counts) return fail(PIC_E_ARG, "counts required");
    const int D = c->dim, ns = c->n_species, nb = c->n_boxes;
    const int64_t w = c->precision == PIC_FP64 ? 8 : 4;
    const int *T = c->tile;
    int64_t cells = 0, tiles = 0;
    L.box_cell0.assign(nb, 0);
    L.box_tile0.assign(nb, 0);
    L.tiles.clear();
    L.max_ntb = 0;
    L.max_count = 1;
    for (int b = 0; b < nb; ++b) {
        int n[3], nt[3];
        for (int d = 0; d < 3; ++d) {
            n[d] = dims_of(c, b, d);
            nt[d] = n[d] / T[d];
        }
        L.box_cell0[b] = cells;
        L.box_tile0[b] = tiles;
        int64_t ntb = (int64_t)nt[0] * nt[1] * nt[2];
        L.max_ntb = std::max(L.max_ntb, ntb);
        for (int tz = 0; tz < nt[2]; ++tz)
            for (int ty = 0; ty < nt[1]; ++ty)
                for (int tx = 0; tx < nt[0]; ++tx) {
                    TileDesc td{};
                    td.box = b;
                    td.tc[0] = tx, td.tc[1] = ty, td.tc[2] = tz;
                    for (int d = 0; d < 3; ++d) td.nt[d] = nt[d], td.n[d] = n[d];
                    td.cell0 = cells;
                    td.tile0 = (int32_t)tiles;
                    if (c->box_walls && (c->box_walls[b] & PIC_WALL_X))
                        td.walls = (tx == 0 ? 1 : 0) | (tx == nt[0] - 1 ? 2 : 0);
                    L.tiles.push_back(td);
                }
        cells += (int64_t)n[0] * n[1] * n[2];
        tiles += ntb;
        for (int s = 0; s < ns; ++s) {
            if (counts[b * ns + s] < 0) return fail(PIC_E_ARG, "negative particle count");
            L.max_count = std::max(L.max_count, counts[b * ns + s]);
            L.max_count = std::max<int64_t>(L.max_count, c->inject_max);
        }
    }
    if (L.max_ntb > (int64_t(1) << 24)) return fail(PIC_E_ARG, "a box has %lld tiles; at most 2^24 are supported", (long long)L.max_ntb);
    if (tiles > INT32_MAX / 8) return fail(PIC_E_ARG, "too many tiles");
    // segment capacities: a multiple of the push kernel's group (threads x
    // particles per thread), so every lane of the last group of a segment
    // has a slot of its own to load from and store to
    const int64_t group = (int64_t)PUSH_UNROLL * (c->block ? c->block : 256);
    double factor = c->capacity_factor > 0 ? c->capacity_factor : 1.25;
    L.seg_off.assign(tiles * ns, 0);
    L.seg_cap.assign(tiles * ns, 0);
    int64_t cap_total = 0, max_cap = 0;
    for (int64_t t = 0; t < tiles; ++t) {
        const int b = L.tiles[t].box;
        const int64_t ntb = (int64_t)L.tiles[t].nt[0] * L.tiles[t].nt[1] * L.tiles[t].nt[2];
        for (int s = 0; s < ns; ++s) {
            int64_t cap;
            if (c->tile_capacity) {
                cap = round_up(std::max<int64_t>(c->tile_capacity[t * ns + s], 64), group);
            } else {
                double expect = (double)counts[b * ns + s] / (double)ntb;
                cap = round_up((int64_t)std::ceil(factor * expect) + 64, group);
            }
            // the push addresses a segment's slots by 32-bit byte offsets
            if (cap > MAX_SLOTS) return fail(PIC_E_ARG, "segment capacity too large (at most 2^28 slots)");
            L.seg_off[t * ns + s] = cap_total;
            L.seg_cap[t * ns + s] = (int32_t)cap;
            cap_total += cap;
            max_cap = std::max(max_cap, cap);
        }
    }
    // segment visiting order before the first push (largest capacity first);
    // every push launch re-sorts the segments by their current counts
    L.order.resize(tiles * ns);
    for (int64_t w = 0; w < tiles * ns; ++w) L.order[w] = (int32_t)w;
    std::stable_sort(L.order.begin(), L.order.end(),
                     [&](int32_t a, int32_t b) { return L.seg_cap[a] > L.seg_cap[b]; });
    L.order_shift = 0;
    while ((max_cap >> L.order_shift) >= pic::ORDER_BUCKETS) ++L.order_shift;
    const int64_t obcap = c->outbox_capacity > 0 ? round_up(c->outbox_capacity, 64)
                                                 : round_up(std::max<int64_t>(256, max_cap / 4), 64);
    int64_t cb = 1, rb = 1;
    for (int d = 0; d < D; ++d) {
        cb *= T[d] + 3;
        rb *= T[d] + 1;
    }
    L.jblk_cells = cb;
    L.rblk_cells = rb;
    L.nchunks_max = std::min<int64_t>(2048, std::max<int64_t>(1, (L.max_count + 4095) / 4096));
    int64_t fbk = 1;
    for (int d = 0; d < D; ++d) fbk *= T[d] + 2;
    L.fblk_cells = fbk;
    L.n_input = 0;
    for (int i = 0; i < nb * ns; ++i) L.n_input += counts[i];
    const bool track = (c->options & PIC_OPT_TRACK) != 0;
    if (track && (cap_total > INT32_MAX || L.n_input > INT32_MAX))
        return fail(PIC_E_ARG, "origin tracking stores int32 ids: at most 2^31-1 slots and input particles");

    uint64_t off = 0;
    auto take = [&](uint64_t bytes) {
        uint64_t o = off;
        off = align256(off + std::max<uint64_t>(bytes, 1));
        return o;
    };
    pic_layout &P = L.pub;
    memset(&P, 0, sizeof P);
    P.off_E = take(3 * cells * w);
    P.off_B = take(3 * cells * w);
    P.off_J = take(3 * cells * w);
    P.off_pos = take(D * cap_total * w);
    P.off_u = take(3 * cap_total * w);
    P.off_xold = take(D * cap_total * w);
    P.off_seg_offset = take(tiles * ns * 8);
    P.off_seg_capacity = take(tiles * ns * 4);
    P.off_seg_count = take(tiles * ns * 4);
    P.off_error = take(4);
    P.off_flags = take(tiles * ns * 4);
    P.off_ids = take(track ? cap_total * 4 : 0);
    L.off_tmp = take((D + 3) * cap_total * w);
    L.off_jblk = take(tiles * ns * 3 * cb * w);
    L.off_rblk = take(tiles * rb * 8);
    L.off_part = take(tiles * pic::NPART * 8);
    L.off_ob_pos = take(tiles * ns * obcap * D * w);
    L.off_ob_u = take(tiles * ns * obcap * 3 * w);
    if (obcap > MAX_SLOTS) return fail(PIC_E_ARG, "outbox capacity too large (at most 2^28 slots)");
    L.ob_dir_stride = obcap;
    L.off_ob_dir = take(tiles * ns * L.ob_dir_stride * 4);
    L.off_ob_cnt = take(tiles * ns * 4);
    L.off_ob_boff = take(tiles * ns * (pic::ncodes<3>() + 1) * 4);
    L.off_ob_idx = take(tiles * ns * obcap * 4);
    L.off_jtmp = take(3 * cells * w);
    L.off_rho_prev = take(cells * 8);
    L.off_nf_pre = take(tiles * ns * 8);
    L.off_tiles = take(tiles * sizeof(TileDesc));
    L.off_charge = take(nb * ns * w);
    L.off_qm = take(nb * ns * w);
    L.off_mass = take(nb * ns * 8);
    L.off_order = take(tiles * ns * 4);
    L.off_queue = take(4);
    L.off_key = take(L.max_count * 4);
    L.off_xl = take(D * L.max_count * w);
    L.off_hist = take(L.nchunks_max * L.max_ntb * 4);
    L.off_ob_ids = take(track ? tiles * ns * obcap * 4 : 0);
    L.off_adj_lj = take(track ? 3 * cells * w : 0);
    L.off_adj_eblk = take(track ? tiles * 3 * cb * w : 0);
    L.off_adj_bblk = take(track ? tiles * 3 * fbk * w : 0);
    P.total_bytes = off;
    P.cells_total = cells;
    P.tiles_total = tiles;
    P.capacity_total = cap_total;
    P.outbox_capacity = obcap;
    P.elem_bytes = (int32_t)w;
    return PIC_OK;
}

}  // namespace

struct pic_ctx {
    int D, prec, ns, nb, block;
    bool acc_working;   // LDS current block in the working precision
    bool persistent;    // push as a persistent tile walker
    bool track;         // origin tracking and adjoint scratch present
    bool walls;         // some box has conducting walls in x
    int pusher;         // PIC_PUSHER_*
    int filter_passes;  // binomial passes pic_step applies to J
    int order;          // FDTD order: 2 (App. B) or 4 (FDTD4)
    int64_t steps;      // completed steps
    int order_age;      // pushes since the visiting order was recomputed
    bool capturing;     // pic_graph_capture is recording steps
    int64_t diag_step;  // steps at the last diagnostics call, or -1
    int n_cu;           // compute units of the device
    hipGraphExec_t graph;   // captured steps, or null
    int graph_steps;
    int T[3];
    double c;
    Layout L;
    hipStream_t stream;
    uint8_t *ws;
    std::vector<double> mass;
    int state;          // 0 ready, 1 unfused push done, 2 fused push done, 3 unfused deposit done
    uint32_t all_species;   // mask of every species
    uint32_t pushed;        // species pushed in the current step
    uint32_t launch_mask;   // species of the next launch (Params::species_mask)
    uint8_t *scratch;       // this device's static scratch (pic_diagnostics_static)
};

namespace {

template <typename R>
Params<R> params(pic_ctx *x)
{
    Params<R> p{};
    const Layout &L = x->L;
    uint8_t *ws = x->ws;
    p.tiles = reinterpret_cast<const TileDesc *>(ws + L.off_tiles);
    p.ntiles = (int32_t)L.pub.tiles_total;
    p.nspecies = x->ns;
    for (int d = 0; d < 3; ++d) p.T[d] = x->T[d];
    p.c = (R)x->c;
    p.inv_c = (R)(1.0 / x->c);
    p.charge = reinterpret_cast<const R *>(ws + L.off_charge);
    p.qm = reinterpret_cast<const R *>(ws + L.off_qm);
    p.E = reinterpret_cast<R *>(ws + L.pub.off_E);
    p.B = reinterpret_cast<R *>(ws + L.pub.off_B);
    p.J = reinterpret_cast<R *>(ws + L.pub.off_J);
    p.cells_total = L.pub.cells_total;
    p.pos = reinterpret_cast<R *>(ws + L.pub.off_pos);
    p.u = reinterpret_cast<R *>(ws + L.pub.off_u);
    p.xold = reinterpret_cast<R *>(ws + L.pub.off_xold);
    p.cap_total = L.pub.capacity_total;
    p.seg_off = reinterpret_cast<const int64_t *>(ws + L.pub.off_seg_offset);
    p.seg_cap = reinterpret_cast<const int32_t *>(ws + L.pub.off_seg_capacity);
    p.seg_cnt = reinterpret_cast<int32_t *>(ws + L.pub.off_seg_count);
    p.jblk = reinterpret_cast<R *>(ws + L.off_jblk);
    p.ob_pos = reinterpret_cast<R *>(ws + L.off_ob_pos);
    p.ob_u = reinterpret_cast<R *>(ws + L.off_ob_u);
    p.ob_dir = reinterpret_cast<int32_t *>(ws + L.off_ob_dir);
    p.ob_cnt = reinterpret_cast<int32_t *>(ws + L.off_ob_cnt);
    p.ob_boff = reinterpret_cast<int32_t *>(ws + L.off_ob_boff);
    p.ob_idx = reinterpret_cast<int32_t *>(ws + L.off_ob_idx);
    p.ob_cap = L.pub.outbox_capacity;
    p.ob_dir_stride = L.ob_dir_stride;
    p.tmp = reinterpret_cast<R *>(ws + L.off_tmp);
    p.err = reinterpret_cast<int32_t *>(ws + L.pub.off_error);
    p.nf_seg = reinterpret_cast<int32_t *>(ws + L.pub.off_flags);
    for (int d = 0; d < 3; ++d) {
        // 2 ulps of R at the tile half-width: every particle within 1 ulp of a
        // face, and every one that an FP32 step can move across a face
        // relative to the FP64 step from the same input
        const R h = (R)(x->T[d] / 2 > 0 ? x->T[d] / 2 : 1);
        p.nf_band[d] = R(2) * (std::nextafter(h, std::numeric_limits<R>::infinity()) - h);
    }
    p.species_mask = x->launch_mask;
    p.mig_counts = nullptr;
    p.queue = reinterpret_cast<int32_t *>(ws + L.off_queue);
    p.order = reinterpret_cast<int32_t *>(ws + L.off_order);
    if (x->track) {
        p.ids = reinterpret_cast<int32_t *>(ws + L.pub.off_ids);
        p.ob_ids = reinterpret_cast<int32_t *>(ws + L.off_ob_ids);
    }
    return p;
}

template <typename K>
pic_status set_lds(K kernel, size_t bytes)
{
    if (bytes > 160 * 1024) return fail(PIC_E_ARG, "tile needs %zu bytes of LDS (max 163840); use a smaller tile", bytes);
    if (bytes > 64 * 1024)
        HIP_OK(hipFuncSetAttribute(reinterpret_cast<const void *>(kernel), hipFuncAttributeMaxDynamicSharedMemorySize,
                                   (int)bytes));
    return PIC_OK;
}

template <typename T>
pic_status fill(pic_ctx *x, T *p, int64_t n, T v)
{
    if (n <= 0) return PIC_OK;
    int grid = (int)std::min<int64_t>((n + 255) / 256, 4096);
    hipLaunchKernelGGL(pic::k_fill<T>, dim3(grid), dim3(256), 0, x->stream, p, n, v);
    HIP_OK(hipGetLastError());
    return PIC_OK;
}

template <typename R, int D>
struct Impl {
    static size_t push_lds(pic_ctx *x, bool fused, size_t acc_bytes)
    {
        int64_t fbn = 1, cbn = 1;
        for (int d = 0; d < D; ++d) {
            fbn *= x->T[d] + 2;
            cbn *= x->T[d] + 3;
        }
        return (3 * cbn + 3 * fbn) * sizeof(R) + (fused ? 3 * cbn * acc_bytes : 0) +
               (2 * PUSH_UNROLL * pic::MAX_WAVES + 4 + (fused ? pic::bucket_lds_ints<D>() : 0)) * sizeof(int);
    }

    template <int ORDER>
    static pic_status fdtd_order(pic_ctx *x, int phase)
    {
        Params<R> p = params<R>(x);
        dim3 g((unsigned)x->L.pub.tiles_total), b(256);
        const R c = (R)x->c;
        switch (phase) {
        case PIC_HALF_B: hipLaunchKernelGGL((pic::k_field<R, D, 0, ORDER>), g, b, 0, x->stream, p, R(0.5) * c); break;
        case PIC_CURL_E: hipLaunchKernelGGL((pic::k_field<R, D, 1, ORDER>), g, b, 0, x->stream, p, c); break;
        case PIC_ADD_J: hipLaunchKernelGGL((pic::k_field<R, D, 2, ORDER>), g, b, 0, x->stream, p, c); break;
        case PIC_CURL_E_ADD_J: hipLaunchKernelGGL((pic::k_field<R, D, 3, ORDER>), g, b, 0, x->stream, p, c); break;
        case PIC_TWO_HALF_B: hipLaunchKernelGGL((pic::k_field<R, D, 4, ORDER>), g, b, 0, x->stream, p, R(0.5) * c); break;
        default: return fail(PIC_E_ARG, "unknown fdtd phase %d", phase);
        }
        HIP_OK(hipGetLastError());
        return PIC_OK;
    }

    static pic_status fdtd(pic_ctx *x, int phase)
    {
        return x->order == 4 ? fdtd_order<4>(x, phase) : fdtd_order<2>(x, phase);
    }

    // segments by decreasing count into p.order (one work-group)
    static pic_status order_segments(pic_ctx *x, const Params<R> &p)
    {
        hipLaunchKernelGGL(pic::k_order, dim3(1), dim3(pic::ORDER_BUCKETS), 0, x->stream, p.seg_cnt,
                           (int32_t)(x->L.pub.tiles_total * x->ns), x->L.order_shift, p.order);
        HIP_OK(hipGetLastError());
        return PIC_OK;
    }

    template <bool FUSED, bool HALFB, typename A, int TC, bool WALLS, int PUSHER>
    static pic_status push_launch(pic_ctx *x)
    {
        Params<R> p = params<R>(x);
        size_t lds = push_lds(x, FUSED, sizeof(A));
        dim3 b(x->block);
        const int64_t items = x->L.pub.tiles_total * x->ns;
        if (x->capturing || x->order_age >= ORDER_EVERY) {
            pic_status st0 = order_segments(x, p);
            if (st0) return st0;
            x->order_age = 0;
        }
        ++x->order_age;
        if (x->persistent) {
            auto kern = pic::k_push_persistent<R, D, FUSED, HALFB, A, PUSH_UNROLL, TC, WALLS, PUSHER>;
            pic_status st = set_lds(kern, lds);
            if (st) return st;
            int per_cu = 0;
            HIP_OK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void *>(kern),
                                                                x->block, lds));
            const int64_t grid = std::min<int64_t>(items, (int64_t)std::max(per_cu, 1) * x->n_cu);
            st = fill<int32_t>(x, p.queue, 1, 0);
            if (st) return st;
            hipLaunchKernelGGL(kern, dim3((unsigned)grid), b, lds, x->stream, p);
        } else {
            auto kern = pic::k_push<R, D, FUSED, HALFB, A, PUSH_UNROLL, TC, WALLS, PUSHER>;
            pic_status st = set_lds(kern, lds);
            if (st) return st;
            hipLaunchKernelGGL(kern, dim3((unsigned)items), b, lds, x->stream, p);
        }
        HIP_OK(hipGetLastError());
        return PIC_OK;
    }

    // The fused push with the 8-byte current block is compiled for the common cubic
    // tile edges with the edge as a constant; other shapes use the
    // runtime-edge kernel.
    template <bool FUSED, bool HALFB, typename A>
    static pic_status push_with(pic_ctx *x)
    {
        if (x->pusher == PIC_PUSHER_VAY)
            return x->walls ? push_launch<FUSED, HALFB, A, 0, FUSED, pic::PUSHER_VAY>(x)
                            : push_launch<FUSED, HALFB, A, 0, false, pic::PUSHER_VAY>(x);
        if (x->pusher == PIC_PUSHER_HC)
            return x->walls ? push_launch<FUSED, HALFB, A, 0, FUSED, pic::PUSHER_HC>(x)
                            : push_launch<FUSED, HALFB, A, 0, false, pic::PUSHER_HC>(x);
        bool cubic = true;
        for (int d = 1; d < D; ++d) cubic = cubic && x->T[d] == x->T[0];
        if constexpr (FUSED) {
            if (x->walls) {
                // the 3D shock's tiles: edge 8 as a constant
                if constexpr (D == 3 && (std::is_same<A, double>::value || std::is_same<A, long long>::value))
                    if (cubic && x->T[0] == 8) return push_launch<FUSED, HALFB, A, 8, true, pic::PUSHER_BORIS>(x);
                return push_launch<FUSED, HALFB, A, 0, true, pic::PUSHER_BORIS>(x);
            }
        }
        if constexpr (FUSED && (std::is_same<A, double>::value || std::is_same<A, long long>::value)) {
            if (cubic && x->T[0] == 8) return push_launch<FUSED, HALFB, A, 8, false, pic::PUSHER_BORIS>(x);
            if (cubic && x->T[0] == 16) return push_launch<FUSED, HALFB, A, 16, false, pic::PUSHER_BORIS>(x);
            if constexpr (D < 3)
                if (cubic && x->T[0] == 32) return push_launch<FUSED, HALFB, A, 32, false, pic::PUSHER_BORIS>(x);
        }
        return push_launch<FUSED, HALFB, A, 0, false, pic::PUSHER_BORIS>(x);
    }

    static pic_status push(pic_ctx *x, bool fused, bool halfb)
    {
        if (!fused) return halfb ? push_with<false, true, R>(x) : push_with<false, false, R>(x);
        if (x->acc_working) return halfb ? push_with<true, true, R>(x) : push_with<true, false, R>(x);
        // FP32: 64-bit fixed-point current block; FP64: FP64 block
        using Acc = typename std::conditional<sizeof(R) == 4, long long, double>::type;
        return halfb ? push_with<true, true, Acc>(x) : push_with<true, false, Acc>(x);
    }

    static pic_status deposit(pic_ctx *x, bool unfused_part, bool curl_e)
    {
        Params<R> p = params<R>(x);
        dim3 g((unsigned)x->L.pub.tiles_total);
        if (unfused_part) {
            const dim3 gs((unsigned)(x->L.pub.tiles_total * x->ns));   // one work-group per segment
            if (x->acc_working) {
                size_t lds = 3 * x->L.jblk_cells * sizeof(R);
                pic_status st = set_lds(pic::k_deposit<R, D, R>, lds);
                if (st) return st;
                hipLaunchKernelGGL((pic::k_deposit<R, D, R>), gs, dim3(x->block), lds, x->stream, p);
            } else {
                size_t lds = 3 * x->L.jblk_cells * sizeof(double);
                pic_status st = set_lds(pic::k_deposit<R, D, double>, lds);
                if (st) return st;
                hipLaunchKernelGGL((pic::k_deposit<R, D, double>), gs, dim3(x->block), lds, x->stream, p);
            }
            HIP_OK(hipGetLastError());
        }
        if (curl_e)
            hipLaunchKernelGGL((pic::k_fold<R, D, true>), g, dim3(256), 0, x->stream, p, (R)x->c);
        else
            hipLaunchKernelGGL((pic::k_fold<R, D, false>), g, dim3(256), 0, x->stream, p, R(0));
        HIP_OK(hipGetLastError());
        return PIC_OK;
    }

    static pic_status migrate(pic_ctx *x, bool need_out, bool need_in, bool sort, int32_t *mig_counts,
                              int64_t *flagged, int64_t flagged_cap)
    {
        Params<R> p = params<R>(x);
        p.mig_counts = mig_counts;
        if (need_in) p.species_mask = x->pushed;   // only these species have leavers
        dim3 g((unsigned)x->L.pub.tiles_total);
        if (need_out) {
            hipLaunchKernelGGL((pic::k_migrate_out<R, D>), g, dim3(x->block), 0, x->stream, p);
            HIP_OK(hipGetLastError());
        }
        if (need_in) {
            // one small work-group per (tile, species) segment: both kernels
            // are chains of dependent loads, so many resident groups pay
            const dim3 gs((unsigned)(x->L.pub.tiles_total * x->ns));
            // the fused push buckets its own outbox; the unfused path (and a
            // call that wants the migration counts) runs the bucket pass here
            if (need_out || mig_counts)
                hipLaunchKernelGGL((pic::k_migrate_bucket<R, D>), gs, dim3(128), 0, x->stream, p);
            hipLaunchKernelGGL((pic::k_migrate_in<R, D>), gs, dim3(128), 0, x->stream, p);
            HIP_OK(hipGetLastError());
        }
        if (sort) {
            int ncell = x->T[0] * x->T[1] * x->T[2];
            size_t lds = (size_t)(4 + 1) * ncell * sizeof(int);
            pic_status st = set_lds(pic::k_cell_sort<R, D>, lds);
            if (st) return st;
            hipLaunchKernelGGL((pic::k_cell_sort<R, D>), g, dim3(256), lds, x->stream, p);
            HIP_OK(hipGetLastError());
        }
        if (flagged) {
            // per-segment counts of the stored positions, their prefix in
            // slot order (and the total into flagged[0]), then the slots
            const int64_t nseg = x->L.pub.tiles_total * x->ns;
            int64_t *pre = reinterpret_cast<int64_t *>(x->ws + x->L.off_nf_pre);
            hipLaunchKernelGGL((pic::k_count_near_face<R, D>), dim3((unsigned)nseg), dim3(256), 0, x->stream, p);
            hipLaunchKernelGGL(pic::k_flag_scan, dim3(1), dim3(1024), 0, x->stream, p.nf_seg, (int32_t)nseg, pre,
                               flagged);
            hipLaunchKernelGGL((pic::k_flag_list<R, D>), dim3((unsigned)nseg), dim3(256), 0, x->stream, p, pre,
                               flagged, flagged_cap);
            HIP_OK(hipGetLastError());
        }
        return PIC_OK;
    }

    // near-face count of every segment from the stored positions
    static pic_status count_near_face(pic_ctx *x)
    {
        Params<R> p = params<R>(x);
        hipLaunchKernelGGL((pic::k_count_near_face<R, D>), dim3((unsigned)(x->L.pub.tiles_total * x->ns)), dim3(256),
                           0, x->stream, p);
        HIP_OK(hipGetLastError());
        return PIC_OK;
    }

    // Bin count FP64 particles of (box b, species s) into their tiles and
    // append them to the segments (after the particles already there, input
    // order kept inside a tile); origin ids id_base + i, or -1 if id_base < 0.
    static pic_status bin_species(pic_ctx *x, int b, int s, int64_t count, const double *pos, const double *u,
                                  int64_t id_base)
    {
        Params<R> p = params<R>(x);
        const Layout &L = x->L;
        uint8_t *ws = x->ws;
        int32_t *key = reinterpret_cast<int32_t *>(ws + L.off_key);
        R *xl = reinterpret_cast<R *>(ws + L.off_xl);
        int32_t *hist = reinterpret_cast<int32_t *>(ws + L.off_hist);
        const TileDesc &t0 = L.tiles[L.box_tile0[b]];
        pic::BinGeom g{};
        for (int d = 0; d < 3; ++d) {
            g.n[d] = t0.n[d];
            g.T[d] = x->T[d];
            g.nt[d] = t0.nt[d];
        }
        g.ntb = t0.nt[0] * t0.nt[1] * t0.nt[2];
        g.count = count;
        g.nchunks = (int32_t)std::min<int64_t>(L.nchunks_max, std::max<int64_t>(1, (count + 4095) / 4096));
        g.chunk = (int32_t)((count + g.nchunks - 1) / g.nchunks);
        g.id_base = id_base;
        g.walls = L.tiles[L.box_tile0[b]].walls != 0 || L.tiles[L.box_tile0[b] + t0.nt[0] - 1].walls != 0;
        int kgrid = (int)std::min<int64_t>((count + 255) / 256, 16384);
        hipLaunchKernelGGL((pic::k_bin_keys<R, D>), dim3(kgrid), dim3(256), 0, x->stream, g, pos, key, xl, p.err);
        // per-chunk tile histograms in LDS up to 32,768 tiles per box, else
        // in global memory (zeroed here)
        g.hist_lds = g.ntb <= 32768;
        size_t lds = g.hist_lds ? (size_t)g.ntb * sizeof(int) : 0;
        pic_status st = PIC_OK;
        if (!g.hist_lds) st = fill<int32_t>(x, hist, (int64_t)g.nchunks * g.ntb, 0);
        if (!st) st = set_lds(pic::k_bin_hist, lds);
        if (st) return st;
        hipLaunchKernelGGL(pic::k_bin_hist, dim3(g.nchunks), dim3(256), lds, x->stream, g, key, hist);
        hipLaunchKernelGGL(pic::k_bin_scan, dim3((g.ntb + 255) / 256), dim3(256), 0, x->stream, g, hist, p.seg_cnt,
                           p.seg_cap, (int)L.box_tile0[b], x->ns, s, p.err);
        st = set_lds(pic::k_bin_scatter<R, D>, lds);
        if (st) return st;
        hipLaunchKernelGGL((pic::k_bin_scatter<R, D>), dim3(g.nchunks), dim3(64), lds, x->stream, g, key, xl, u, hist, p,
                           (int)L.box_tile0[b], s);
        HIP_OK(hipGetLastError());
        return PIC_OK;
    }

    static pic_status inject(pic_ctx *x, int b, int s, int64_t count, const double *pos, const double *u)
    {
        pic_status st = bin_species(x, b, s, count, pos, u, -1);
        return st ? st : count_near_face(x);
    }

    static pic_status init(pic_ctx *x, const int64_t *counts, const pic_init_data *in)
    {
        Params<R> p = params<R>(x);
        const Layout &L = x->L;
        pic_status st = fill<int32_t>(x, p.seg_cnt, L.pub.tiles_total * x->ns, 0);
        if (!st) st = fill<int32_t>(x, p.ob_cnt, L.pub.tiles_total * x->ns, 0);
        if (!st) st = fill<R>(x, p.J, 3 * L.pub.cells_total, R(0));
        if (!st) st = fill<R>(x, p.E, 3 * L.pub.cells_total, R(0));
        if (!st) st = fill<R>(x, p.B, 3 * L.pub.cells_total, R(0));
        if (!st) st = fill<R>(x, p.jblk, L.pub.tiles_total * x->ns * 3 * L.jblk_cells, R(0));
        if (st) return st;
        int64_t id_base = 0;
        for (int b = 0; b < x->nb; ++b) {
            const TileDesc &t0 = L.tiles[L.box_tile0[b]];
            const int64_t cells = (int64_t)t0.n[0] * t0.n[1] * t0.n[2];
            int grid = (int)std::min<int64_t>((3 * cells + 255) / 256, 8192);
            if (in->E && in->E[b])
                hipLaunchKernelGGL((pic::k_load_field<R>), dim3(grid), dim3(256), 0, x->stream, p.E, L.pub.cells_total,
                                   L.box_cell0[b], in->E[b], cells);
            if (in->B && in->B[b])
                hipLaunchKernelGGL((pic::k_load_field<R>), dim3(grid), dim3(256), 0, x->stream, p.B, L.pub.cells_total,
                                   L.box_cell0[b], in->B[b], cells);
            HIP_OK(hipGetLastError());
            for (int s = 0; s < x->ns; ++s) {
                const int64_t count = counts[b * x->ns + s];
                id_base += count;
                if (count == 0) continue;
                if (!in->pos || !in->u || !in->pos[b * x->ns + s] || !in->u[b * x->ns + s])
                    return fail(PIC_E_ARG, "missing particle data for box %d species %d", b, s);
                st = bin_species(x, b, s, count, in->pos[b * x->ns + s], in->u[b * x->ns + s], id_base - count);
                if (st) return st;
            }
        }
        if (x->walls) {
            hipLaunchKernelGGL((pic::k_hold_walls<R, D>), dim3((unsigned)L.pub.tiles_total), dim3(256), 0, x->stream, p);
            HIP_OK(hipGetLastError());
        }
        return count_near_face(x);
    }

    // Reverse of one fused step from the current state (Table 1 rows in
    // reverse order; the field rows reuse the forward stencils on the
    // adjoint fields, since (curl+)^T = curl- on the periodic lattice).
    static pic_status adjoint(pic_ctx *x, void *lpos, void *lu, void *lE, void *lB)
    {
        Params<R> p = params<R>(x);
        const Layout &L = x->L;
        pic::AdjParams<R> a{};
        a.lpos = reinterpret_cast<R *>(lpos);
        a.lu = reinterpret_cast<R *>(lu);
        a.lE = reinterpret_cast<R *>(lE);
        a.lB = reinterpret_cast<R *>(lB);
        a.lJ = reinterpret_cast<R *>(x->ws + L.off_adj_lj);
        a.eblk = reinterpret_cast<R *>(x->ws + L.off_adj_eblk);
        a.bblk = reinterpret_cast<R *>(x->ws + L.off_adj_bblk);
        const R c = (R)x->c;
        const int64_t n3 = 3 * L.pub.cells_total;
        dim3 g((unsigned)L.pub.tiles_total), b(256);
        // add_cur: E^{n+1} = ... - J  ->  lambda_J = -lambda_E
        hipLaunchKernelGGL((pic::k_adj_neg<R>), dim3((unsigned)std::min<int64_t>((n3 + 255) / 256, 8192)), b, 0,
                           x->stream, a.lJ, a.lE, n3);
        // push_e: E^{n+1} = E^n + c curl- B^{n+1/2}  ->  lambda_B += c curl+ lambda_E
        Params<R> q = p;
        q.E = a.lE;
        q.B = a.lB;
        hipLaunchKernelGGL((pic::k_field<R, D, 0>), g, b, 0, x->stream, q, -c);
        // push_half_b2: B^{n+1/2} = B^n - (c/2) curl+ E^n  ->  lambda_E -= (c/2) curl- lambda_B
        hipLaunchKernelGGL((pic::k_field<R, D, 1>), g, b, 0, x->stream, q, R(-0.5) * c);
        // comp_curr, position update, Boris, interp_em per particle
        const size_t lds = 3 * (L.jblk_cells + L.fblk_cells) * sizeof(double) +
                           (6 * L.jblk_cells + 3 * L.fblk_cells) * sizeof(R);
        pic_status st = set_lds(pic::k_adj_push<R, D>, lds);
        if (st) return st;
        hipLaunchKernelGGL((pic::k_adj_push<R, D>), g, b, lds, x->stream, p, a);
        hipLaunchKernelGGL((pic::k_adj_fold<R, D>), g, b, 0, x->stream, p, a);
        // push_half_b1: B^n = B^{n-1/2} - (c/2) curl+ E^n  ->  lambda_E -= (c/2) curl- lambda_B^n
        hipLaunchKernelGGL((pic::k_field<R, D, 1>), g, b, 0, x->stream, q, R(-0.5) * c);
        HIP_OK(hipGetLastError());
        return PIC_OK;
    }

    static pic_status filter(pic_ctx *x, int passes)
    {
        Params<R> p = params<R>(x);
        R *tmp = reinterpret_cast<R *>(x->ws + x->L.off_jtmp);
        dim3 g((unsigned)x->L.pub.tiles_total), b(256);
        for (int k = 0; k < passes; ++k) {
            const R *src = k % 2 ? tmp : p.J;
            R *dst = k % 2 ? p.J : tmp;
            hipLaunchKernelGGL((pic::k_filter<R, D>), g, b, 0, x->stream, p, src, dst);
        }
        if (passes % 2) {
            const int64_t n = 3 * x->L.pub.cells_total;
            hipLaunchKernelGGL((pic::k_copy<R>), dim3((unsigned)std::min<int64_t>((n + 255) / 256, 8192)), b, 0,
                               x->stream, p.J, tmp, n);
        }
        HIP_OK(hipGetLastError());
        return PIC_OK;
    }

    static pic_status unpermute(pic_ctx *x, const void *la, const void *ua, void *lb, void *ub, int64_t stride)
    {
        Params<R> p = params<R>(x);
        int64_t maxcap = 1;
        for (int32_t c : x->L.seg_cap) maxcap = std::max<int64_t>(maxcap, c);
        const dim3 grid((unsigned)(x->L.pub.tiles_total * x->ns), (unsigned)((maxcap + 255) / 256));
        hipLaunchKernelGGL((pic::k_adj_unpermute<R, D>), grid, dim3(256), 0, x->stream, p,
                           reinterpret_cast<const R *>(la), reinterpret_cast<const R *>(ua),
                           reinterpret_cast<R *>(lb), reinterpret_cast<R *>(ub), stride);
        HIP_OK(hipGetLastError());
        return PIC_OK;
    }

    // per-tile diagnostic partials into part [tiles][NPART] and the charge
    // blocks into rblk [tiles][(T+1)^D]
    static pic_status diag_partials(pic_ctx *x, double *part, double *rblk, int cont_valid)
    {
        Params<R> p = params<R>(x);
        const Layout &L = x->L;
        const double *mass = reinterpret_cast<const double *>(x->ws + L.off_mass);
        size_t lds = L.rblk_cells * sizeof(double);
        pic_status st = set_lds(pic::k_diag_tile<R, D>, lds);
        if (st) return st;
        dim3 g((unsigned)L.pub.tiles_total);
        hipLaunchKernelGGL((pic::k_diag_tile<R, D>), g, dim3(256), lds, x->stream, p, mass, part, rblk);
        double *rho_prev = reinterpret_cast<double *>(x->ws + L.off_rho_prev);
        hipLaunchKernelGGL((pic::k_diag_gauss<R, D>), g, dim3(256), 0, x->stream, p, part, rblk, rho_prev, cont_valid);
        HIP_OK(hipGetLastError());
        return PIC_OK;
    }

    // the diagnostics with the partials in the static scratch, reduced on
    // the device; no allocation of any kind
    static pic_status diag_static(pic_ctx *x, pic_diag *out)
    {
        const Layout &L = x->L;
        const uint64_t part_bytes = align256(L.pub.tiles_total * pic::NPART * sizeof(double));
        const uint64_t rblk_bytes = align256(L.pub.tiles_total * L.rblk_cells * sizeof(double));
        const uint64_t need = part_bytes + rblk_bytes + align256(sizeof(pic::DiagRec));
        if (need > STATIC_SCRATCH_BYTES)
            return fail(PIC_E_ARG, "pic_diagnostics_static needs %llu bytes of static scratch for %lld tiles; "
                                   "the limit is %llu bytes (use pic_diagnostics)",
                        (unsigned long long)need, (long long)L.pub.tiles_total,
                        (unsigned long long)STATIC_SCRATCH_BYTES);
        double *part = reinterpret_cast<double *>(x->scratch);
        double *rblk = reinterpret_cast<double *>(x->scratch + part_bytes);
        pic::DiagRec *rec = reinterpret_cast<pic::DiagRec *>(x->scratch + part_bytes + rblk_bytes);
        const int cont_valid = x->diag_step >= 0 && x->steps - x->diag_step == 1;
        pic_status st = diag_partials(x, part, rblk, cont_valid);
        if (st) return st;
        hipLaunchKernelGGL(pic::k_diag_reduce, dim3(1), dim3(64), 0, x->stream, part, L.pub.tiles_total, cont_valid,
                           rec);
        HIP_OK(hipGetLastError());
        pic::DiagRec h{};
        HIP_OK(hipMemcpyAsync(&h, rec, sizeof h, hipMemcpyDeviceToHost, x->stream));
        HIP_OK(hipStreamSynchronize(x->stream));
        memset(out, 0, sizeof *out);
        out->field_energy = h.field_energy;
        out->kinetic_energy = h.kinetic_energy;
        out->gauss_max = h.gauss_max;
        out->divb_max = h.divb_max;
        out->charge_total = h.charge_total;
        out->particles = h.particles;
        out->near_face = h.near_face;
        out->continuity_max = h.continuity_max;
        x->diag_step = x->steps;
        return PIC_OK;
    }

    static pic_status diag(pic_ctx *x, pic_diag *out, bool per_box)
    {
        const Layout &L = x->L;
        double *part = reinterpret_cast<double *>(x->ws + L.off_part);
        double *rblk = reinterpret_cast<double *>(x->ws + L.off_rblk);
        const int cont_valid = x->diag_step >= 0 && x->steps - x->diag_step == 1;
        pic_status st = diag_partials(x, part, rblk, cont_valid);
        if (st) return st;
        std::vector<double> h(L.pub.tiles_total * pic::NPART);
        HIP_OK(hipMemcpyAsync(h.data(), part, h.size() * sizeof(double), hipMemcpyDeviceToHost, x->stream));
        HIP_OK(hipStreamSynchronize(x->stream));
        const int nout = per_box ? x->nb : 1;
        memset(out, 0, nout * sizeof *out);
        for (int64_t t = 0; t < L.pub.tiles_total; ++t) {
            const double *o = &h[t * pic::NPART];
            pic_diag *d = per_box ? out + L.tiles[t].box : out;
            d->field_energy += o[0];
            d->divb_max = std::max(d->divb_max, o[1]);
            d->kinetic_energy += o[2];
            d->particles += (int64_t)o[3];
            d->gauss_max = std::max(d->gauss_max, o[4]);
            d->charge_total += o[5];
            d->near_face += (int64_t)o[7];
        }
        for (int k = 0; k < nout; ++k) out[k].continuity_max = cont_valid ? 0.0 : -1.0;
        if (cont_valid)
            for (int64_t t = 0; t < L.pub.tiles_total; ++t) {
                pic_diag *d = per_box ? out + L.tiles[t].box : out;
                d->continuity_max = std::max(d->continuity_max, h[t * pic::NPART + 6]);
            }
        x->diag_step = x->steps;
        return PIC_OK;
    }
};

#define PIC_DISPATCH(ctx, CALL)                                      \
    do {                                                             \
        if ((ctx)->prec == PIC_FP32) {                               \
            switch ((ctx)->D) {                                      \
            case 1: return Impl<float, 1>::CALL;                     \
            case 2: return Impl<float, 2>::CALL;                     \
            default: return Impl<float, 3>::CALL;                    \
            }                                                        \
        } else {                                                     \
            switch ((ctx)->D) {                                      \
            case 1: return Impl<double, 1>::CALL;                    \
            case 2: return Impl<double, 2>::CALL;                    \
            default: return Impl<double, 3>::CALL;                   \
            }                                                        \
        }                                                            \
    } while (0)

pic_status do_init(pic_ctx *x, const int64_t *counts, const pic_init_data *in) { PIC_DISPATCH(x, init(x, counts, in)); }
pic_status do_fdtd(pic_ctx *x, int phase) { PIC_DISPATCH(x, fdtd(x, phase)); }
pic_status do_push(pic_ctx *x, bool fused, bool halfb) { PIC_DISPATCH(x, push(x, fused, halfb)); }
pic_status do_deposit(pic_ctx *x, bool unfused, bool curl_e) { PIC_DISPATCH(x, deposit(x, unfused, curl_e)); }
pic_status do_migrate(pic_ctx *x, bool out, bool in, bool sort, int32_t *mc, int64_t *fl, int64_t fcap)
{
    PIC_DISPATCH(x, migrate(x, out, in, sort, mc, fl, fcap));
}
pic_status do_diag(pic_ctx *x, pic_diag *o, bool per_box) { PIC_DISPATCH(x, diag(x, o, per_box)); }
pic_status do_diag_static(pic_ctx *x, pic_diag *o) { PIC_DISPATCH(x, diag_static(x, o)); }
pic_status do_adjoint(pic_ctx *x, void *a, void *b, void *c, void *d) { PIC_DISPATCH(x, adjoint(x, a, b, c, d)); }
pic_status do_filter(pic_ctx *x, int passes) { PIC_DISPATCH(x, filter(x, passes)); }
pic_status do_inject(pic_ctx *x, int b, int s, int64_t n, const double *pos, const double *u)
{
    PIC_DISPATCH(x, inject(x, b, s, n, pos, u));
}
pic_status do_unpermute(pic_ctx *x, const void *a, const void *b, void *c, void *d, int64_t s)
{
    PIC_DISPATCH(x, unpermute(x, a, b, c, d, s));
}

template <typename R>
pic_status upload_tables(pic_ctx *x, const pic_config *cfg)
{
    const Layout &L = x->L;
    uint8_t *ws = x->ws;
    const int n = x->nb * x->ns;
    std::vector<R> ch(n), qm(n);
    for (int i = 0; i < n; ++i) {
        ch[i] = (R)cfg->charge[i];
        qm[i] = (R)cfg->qm[i];
    }
    x->mass.assign(cfg->mass, cfg->mass + n);
    HIP_OK(hipMemcpy(ws + L.off_charge, ch.data(), n * sizeof(R), hipMemcpyHostToDevice));
    HIP_OK(hipMemcpy(ws + L.off_qm, qm.data(), n * sizeof(R), hipMemcpyHostToDevice));
    return PIC_OK;
}

pic_status read_error(pic_ctx *x, int32_t *bits)
{
    int32_t *err = reinterpret_cast<int32_t *>(x->ws + x->L.pub.off_error);
    HIP_OK(hipMemcpyAsync(bits, err, sizeof(int32_t), hipMemcpyDeviceToHost, x->stream));
    HIP_OK(hipStreamSynchronize(x->stream));
    if (*bits) {
        pic_status st = fill<int32_t>(x, err, 1, 0);
        if (st) return st;
        HIP_OK(hipStreamSynchronize(x->stream));
    }
    return PIC_OK;
}

pic_status error_status(int32_t bits)
{
    pic_status st = 0;
    if (bits & pic::ERR_CAPACITY) st |= PIC_E_CAPACITY;
    if (bits & pic::ERR_CFL) st |= PIC_E_CFL;
    if (bits & pic::ERR_NONFINITE) st |= PIC_E_NONFINITE;
    if (bits & pic::ERR_OUT_OF_TILE) st |= PIC_E_OUT_OF_TILE;
    if (bits & pic::ERR_ADJ_MAP) st |= PIC_E_ADJ_MAP;
    if (st) fail(st, "device error bits 0x%x", bits);
    return st;
}

}  // namespace

extern "C" {

pic_status pic_query(const pic_config *cfg, const int64_t *counts, pic_layout *out)
{
    if (!out) return fail(PIC_E_ARG, "null output");
    Layout L;
    pic_status st = make_layout(cfg, counts, L);
    if (st) return st;
    *out = L.pub;
    return PIC_OK;
}

pic_status pic_init_tiles(const pic_config *cfg, const int64_t *counts, void *workspace, uint64_t workspace_bytes,
                          const pic_init_data *init, void *hip_stream, pic_ctx **out)
{
    if (!out || !init) return fail(PIC_E_ARG, "null argument");
    *out = nullptr;
    pic_ctx *x = new pic_ctx();
    pic_status st = make_layout(cfg, counts, x->L);
    if (st) {
        delete x;
        return st;
    }
    if (!workspace || workspace_bytes < x->L.pub.total_bytes || (reinterpret_cast<uintptr_t>(workspace) & 255)) {
        delete x;
        return fail(PIC_E_ARG, "workspace must be 256-byte aligned and hold %llu bytes",
                    (unsigned long long)x->L.pub.total_bytes);
    }
    x->D = cfg->dim;
    x->prec = cfg->precision;
    x->ns = cfg->n_species;
    x->nb = cfg->n_boxes;
    x->block = cfg->block ? cfg->block : 256;
    x->acc_working = (cfg->options & PIC_OPT_ACC_WORKING) != 0;
    x->persistent = (cfg->options & PIC_OPT_PERSISTENT) != 0;
    x->track = (cfg->options & PIC_OPT_TRACK) != 0;
    x->walls = false;
    x->pusher = cfg->pusher;
    x->filter_passes = cfg->filter_passes;
    x->order = cfg->fdtd_order == 4 ? 4 : 2;
    x->steps = 0;
    x->order_age = ORDER_EVERY;
    x->capturing = false;
    x->diag_step = -1;
    for (int b = 0; cfg->box_walls && b < cfg->n_boxes; ++b) x->walls = x->walls || (cfg->box_walls[b] & PIC_WALL_X);
    x->graph = nullptr;
    x->graph_steps = 0;
    {
        int dev = 0;
        hipDeviceProp_t prop;
        if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) {
            delete x;
            return fail(PIC_E_HIP, "cannot query the device");
        }
        x->n_cu = prop.multiProcessorCount;
    }
    for (int d = 0; d < 3; ++d) x->T[d] = cfg->tile[d];
    x->c = cfg->cfl;
    x->stream = reinterpret_cast<hipStream_t>(hip_stream);
    x->ws = reinterpret_cast<uint8_t *>(workspace);
    x->state = 0;
    x->all_species = (1u << x->ns) - 1u;
    x->pushed = 0;
    x->launch_mask = x->all_species;
    const Layout &L = x->L;
    auto cleanup = [&](pic_status s) {
        delete x;
        return s;
    };
#define INIT_HIP(expr)                                                                           \
    do {                                                                                         \
        hipError_t e_ = (expr);                                                                  \
        if (e_ != hipSuccess) return cleanup(fail(PIC_E_HIP, "%s: %s", #expr, hipGetErrorString(e_))); \
    } while (0)
    INIT_HIP(hipStreamSynchronize(x->stream));
    {
        void *sp = nullptr;
        if ((st = scratch_address(&sp))) return cleanup(st);
        x->scratch = reinterpret_cast<uint8_t *>(sp);
    }
    INIT_HIP(hipMemcpy(x->ws + L.off_tiles, L.tiles.data(), L.tiles.size() * sizeof(TileDesc), hipMemcpyHostToDevice));
    INIT_HIP(hipMemcpy(x->ws + L.pub.off_seg_offset, L.seg_off.data(), L.seg_off.size() * 8, hipMemcpyHostToDevice));
    INIT_HIP(hipMemcpy(x->ws + L.pub.off_seg_capacity, L.seg_cap.data(), L.seg_cap.size() * 4, hipMemcpyHostToDevice));
    INIT_HIP(hipMemcpy(x->ws + L.off_order, L.order.data(), L.order.size() * 4, hipMemcpyHostToDevice));
    INIT_HIP(hipMemcpy(x->ws + L.off_mass, cfg->mass, (size_t)x->nb * x->ns * 8, hipMemcpyHostToDevice));
    st = x->prec == PIC_FP32 ? upload_tables<float>(x, cfg) : upload_tables<double>(x, cfg);
    if (st) return cleanup(st);
    if ((st = fill<int32_t>(x, reinterpret_cast<int32_t *>(x->ws + L.pub.off_error), 1, 0))) return cleanup(st);
    if ((st = do_init(x, counts, init))) return cleanup(st);
    int32_t bits = 0;
    if ((st = read_error(x, &bits))) return cleanup(st);
    if (bits) return cleanup(error_status(bits));
#undef INIT_HIP
    *out = x;
    return PIC_OK;
}

pic_status pic_fdtd_step(pic_ctx *x, int32_t phase)
{
    if (!x) return fail(PIC_E_ARG, "null context");
    return do_fdtd(x, phase);
}

// species mask of a push or deposit call: PIC_ALL_SPECIES or a nonempty
// subset of the context's species
static pic_status species_of(pic_ctx *x, uint32_t mask, uint32_t *out)
{
    if (mask == PIC_ALL_SPECIES) mask = x->all_species;
    if (!mask || (mask & ~x->all_species))
        return fail(PIC_E_ARG, "species mask 0x%x: empty or beyond the %d species", mask, x->ns);
    if (x->track && mask != x->all_species)
        return fail(PIC_E_ARG, "origin tracking (PIC_OPT_TRACK) needs every species in one call");
    *out = mask;
    return PIC_OK;
}

pic_status pic_push_interp(pic_ctx *x, uint32_t species_mask, uint32_t flags)
{
    if (!x) return fail(PIC_E_ARG, "null context");
    uint32_t mask = 0;
    pic_status st = species_of(x, species_mask, &mask);
    if (st) return st;
    const bool fused = flags & PIC_FUSED;
    if (x->state >= 3) return fail(PIC_E_STATE, "push called after this step's deposit");
    if (x->state != 0 && (x->state == 2) != fused)
        return fail(PIC_E_STATE, "every push of a step must use the same PIC_FUSED setting");
    if (x->pushed & mask) return fail(PIC_E_STATE, "species 0x%x already pushed in this step", x->pushed & mask);
    if (x->order == 4 && (flags & PIC_PUSH_HALF_B))
        return fail(PIC_E_ARG, "PIC_PUSH_HALF_B applies the second-order half update; use pic_fdtd_step with FDTD4");
    if (x->track && !fused) return fail(PIC_E_ARG, "origin tracking records origins in the fused push only");
    if (x->walls && !fused) return fail(PIC_E_ARG, "boxes with walls need the fused push (PIC_FUSED)");
    x->launch_mask = mask;
    st = do_push(x, fused, (flags & PIC_PUSH_HALF_B) != 0);
    x->launch_mask = x->all_species;
    if (st) return st;
    x->pushed |= mask;
    x->state = fused ? 2 : 1;
    return PIC_OK;
}

pic_status pic_deposit_current(pic_ctx *x, uint32_t species_mask, uint32_t flags)
{
    if (!x) return fail(PIC_E_ARG, "null context");
    uint32_t mask = 0;
    pic_status st = species_of(x, species_mask, &mask);
    if (st) return st;
    const bool curl_e = flags & PIC_DEPOSIT_CURL_E;
    if (curl_e && x->order != 2) return fail(PIC_E_ARG, "PIC_DEPOSIT_CURL_E applies the second-order E update; use pic_fdtd_step with FDTD4");
    if (x->state != 1 && x->state != 2) return fail(PIC_E_STATE, "deposit needs a preceding push (once per step)");
    if (mask & ~x->pushed) return fail(PIC_E_STATE, "species 0x%x not pushed in this step", mask & ~x->pushed);
    x->launch_mask = mask;
    st = do_deposit(x, x->state == 1, curl_e);
    x->launch_mask = x->all_species;
    if (st) return st;
    x->state = 3 + (x->state == 2 ? 1 : 0);   // 3: unfused deposited, 4: fused deposited
    return PIC_OK;
}

pic_status pic_sort_migrate(pic_ctx *x, uint32_t flags, int32_t *migration_counts, int64_t *flagged,
                            int64_t flagged_capacity)
{
    if (!x) return fail(PIC_E_ARG, "null context");
    if (x->state == 1) return fail(PIC_E_STATE, "deposit the current of an unfused push before migrating");
    if (flagged_capacity < 0) return fail(PIC_E_ARG, "flagged_capacity must be >= 0");
    const bool sort = flags & PIC_SORT_CELLS;
    if (x->track && sort) return fail(PIC_E_ARG, "the cell sort does not record origins (PIC_OPT_TRACK)");
    const bool stepped = x->state != 0;
    if (migration_counts && !stepped) return fail(PIC_E_STATE, "migration counts need a preceding push");
    pic_status st;
    if (x->state == 3) st = do_migrate(x, true, true, sort, migration_counts, flagged, flagged_capacity);
    else if (stepped) st = do_migrate(x, false, true, sort, migration_counts, flagged, flagged_capacity);
    else st = do_migrate(x, false, false, sort, nullptr, flagged, flagged_capacity);   // nothing moved
    if (st) return st;
    x->state = 0;
    x->pushed = 0;
    if (stepped) ++x->steps;
    return PIC_OK;
}

// deposit (or fold), filter, E += c curl- B - J; with FDTD2 and no filter
// the fold and the E update are one pass.
static pic_status current_and_e(pic_ctx *x, uint32_t flags)
{
    pic_status st;
    if (!x->filter_passes && x->order == 2) return pic_deposit_current(x, PIC_ALL_SPECIES, flags | PIC_DEPOSIT_CURL_E);
    if ((st = pic_deposit_current(x, PIC_ALL_SPECIES, flags))) return st;
    if (x->filter_passes && (st = pic_filter_current(x, x->filter_passes))) return st;
    return pic_fdtd_step(x, PIC_CURL_E_ADD_J);
}

pic_status pic_step(pic_ctx *x, uint32_t flags)
{
    pic_status st;
    if (!x) return fail(PIC_E_ARG, "null context");
    if (x->order == 4) flags &= ~PIC_PUSH_HALF_B;   // the in-LDS half update is second order
    flags &= ~PIC_DEPOSIT_CURL_E;                    // chosen below
    if (flags & PIC_PUSH_HALF_B) {
        // push_half_b1 happens inside the push on its LDS copy of B; both
        // half updates are then applied to the stored B in one pass
        if ((st = pic_push_interp(x, PIC_ALL_SPECIES, flags))) return st;
        if ((st = pic_fdtd_step(x, PIC_TWO_HALF_B))) return st;
        if ((st = current_and_e(x, flags))) return st;
        return pic_sort_migrate(x, flags, nullptr, nullptr, 0);
    }
    if ((st = pic_fdtd_step(x, PIC_HALF_B))) return st;
    if ((st = pic_push_interp(x, PIC_ALL_SPECIES, flags))) return st;
    if ((st = pic_fdtd_step(x, PIC_HALF_B))) return st;
    if ((st = current_and_e(x, flags))) return st;
    return pic_sort_migrate(x, flags, nullptr, nullptr, 0);
}

pic_status pic_inject(pic_ctx *x, int32_t box, int32_t species, int64_t count, const double *pos, const double *u)
{
    if (!x) return fail(PIC_E_ARG, "null context");
    if (x->state != 0) return fail(PIC_E_STATE, "inject between steps");
    if (box < 0 || box >= x->nb || species < 0 || species >= x->ns) return fail(PIC_E_ARG, "box or species out of range");
    if (count < 0 || count > x->L.max_count)
        return fail(PIC_E_ARG, "a batch holds at most %lld particles (pic_config.inject_max)", (long long)x->L.max_count);
    if (count == 0) return PIC_OK;
    if (!pos || !u) return fail(PIC_E_ARG, "pos and u are required");
    x->order_age = ORDER_EVERY;   // counts changed: re-sort at the next push
    return do_inject(x, box, species, count, pos, u);
}

pic_status pic_filter_current(pic_ctx *x, int32_t passes)
{
    if (!x) return fail(PIC_E_ARG, "null context");
    if (passes < 0) return fail(PIC_E_ARG, "passes must be >= 0");
    if (x->walls) return fail(PIC_E_ARG, "the current filter covers periodic boxes only");
    if (passes == 0) return PIC_OK;
    return do_filter(x, passes);
}

pic_status pic_graph_capture(pic_ctx *x, int32_t nsteps, uint32_t flags)
{
    if (!x || nsteps < 1) return fail(PIC_E_ARG, "need a context and nsteps >= 1");
    if (x->state != 0) return fail(PIC_E_STATE, "capture must start between steps");
    if (!x->stream) return fail(PIC_E_ARG, "graph capture needs a context on a created (non-default) stream");
    if (x->graph) {
        HIP_OK(hipGraphExecDestroy(x->graph));
        x->graph = nullptr;
    }
    // one eager step sets the kernels' LDS attributes before capture
    pic_status st = pic_step(x, flags);
    if (st) return st;
    HIP_OK(hipStreamSynchronize(x->stream));
    const int64_t steps_before = x->steps;   // captured steps do not run now
    HIP_OK(hipStreamBeginCapture(x->stream, hipStreamCaptureModeThreadLocal));
    x->capturing = true;
    for (int k = 0; k < nsteps && !st; ++k) st = pic_step(x, flags);
    x->capturing = false;
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(x->stream, &g);
    x->steps = steps_before;
    if (st) {
        if (g) (void)hipGraphDestroy(g);
        return st;
    }
    if (e != hipSuccess) return fail(PIC_E_HIP, "hipStreamEndCapture: %s", hipGetErrorString(e));
    e = hipGraphInstantiate(&x->graph, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) {
        x->graph = nullptr;
        return fail(PIC_E_HIP, "hipGraphInstantiate: %s", hipGetErrorString(e));
    }
    x->graph_steps = nsteps;
    return PIC_OK;
}

pic_status pic_graph_launch(pic_ctx *x)
{
    if (!x || !x->graph) return fail(PIC_E_STATE, "no captured graph");
    HIP_OK(hipGraphLaunch(x->graph, x->stream));
    x->steps += x->graph_steps;
    return PIC_OK;
}

pic_status pic_error(pic_ctx *x)
{
    if (!x) return fail(PIC_E_ARG, "null context");
    int32_t bits = 0;
    pic_status st = read_error(x, &bits);
    if (st) return st;
    return error_status(bits);
}

pic_status pic_diagnostics(pic_ctx *x, pic_diag *out)
{
    if (!x || !out) return fail(PIC_E_ARG, "null argument");
    pic_status st = do_diag(x, out, false);
    if (st) return st;
    int32_t bits = 0;
    if ((st = read_error(x, &bits))) return st;
    out->error_bits = bits;
    return error_status(bits);
}

pic_status pic_diagnostics_static(pic_ctx *x, pic_diag *out)
{
    if (!x || !out) return fail(PIC_E_ARG, "null argument");
    pic_status st = do_diag_static(x, out);
    if (st) return st;
    int32_t bits = 0;
    if ((st = read_error(x, &bits))) return st;
    out->error_bits = bits;
    return error_status(bits);
}

pic_status pic_diagnostics_boxes(pic_ctx *x, pic_diag *out)
{
    if (!x || !out) return fail(PIC_E_ARG, "null argument");
    pic_status st = do_diag(x, out, true);
    if (st) return st;
    int32_t bits = 0;
    if ((st = read_error(x, &bits))) return st;
    for (int b = 0; b < x->nb; ++b) out[b].error_bits = bits;
    return error_status(bits);
}

pic_status pic_adjoint_unpermute(pic_ctx *x, const void *lpos_after, const void *lu_after, void *lpos_before,
                                 void *lu_before, int64_t before_stride)
{
    if (!x) return fail(PIC_E_ARG, "null context");
    if (!x->track) return fail(PIC_E_STATE, "the context was created without PIC_OPT_TRACK");
    if (!lpos_after || !lu_after || !lpos_before || !lu_before || before_stride < 1)
        return fail(PIC_E_ARG, "adjoint buffers and a positive before_stride are required");
    if (x->state != 0) return fail(PIC_E_STATE, "unpermute must run between steps");
    return do_unpermute(x, lpos_after, lu_after, lpos_before, lu_before, before_stride);
}

pic_status pic_adjoint_step(pic_ctx *x, void *lpos, void *lu, void *lE, void *lB)
{
    if (!x) return fail(PIC_E_ARG, "null context");
    if (!x->track) return fail(PIC_E_STATE, "the context was created without PIC_OPT_TRACK");
    if (x->walls) return fail(PIC_E_ARG, "the adjoint step covers periodic boxes only");
    if (x->pusher != PIC_PUSHER_BORIS || x->filter_passes || x->order != 2)
        return fail(PIC_E_ARG, "the adjoint step covers the Boris pusher and FDTD2 without current filter");
    if (!lpos || !lu || !lE || !lB) return fail(PIC_E_ARG, "adjoint buffers are required");
    if (x->state != 0) return fail(PIC_E_STATE, "the adjoint step must start between steps");
    return do_adjoint(x, lpos, lu, lE, lB);
}

pic_status pic_destroy(pic_ctx *x)
{
    if (x && x->graph) (void)hipGraphExecDestroy(x->graph);
    delete x;
    return PIC_OK;
}

const char *pic_last_error(void) { return g_last_error; }

}  // extern "C"
