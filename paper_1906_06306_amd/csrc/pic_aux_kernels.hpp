// Initialisation (binning) and FP64 diagnostic kernels.
#pragma once

#include "pic_kernels.hpp"

namespace pic {

// ---------------------------------------------------------------- generic

template <typename T>
__global__ void k_fill(T *p, int64_t n, T v)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

template <typename T>
__global__ void k_copy(T *__restrict__ dst, const T *__restrict__ src, int64_t n)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        dst[i] = src[i];
}

// FP64 box field [3][cells] -> working precision, into the global planes.
template <typename R>
__global__ void k_load_field(R *dst, int64_t cells_total, int64_t cell0, const double *src, int64_t cells)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < 3 * cells;
         i += (int64_t)gridDim.x * blockDim.x) {
        int64_t m = i / cells, k = i - m * cells;
        dst[m * cells_total + cell0 + k] = (R)src[i];
    }
}

// ------------------------------------------------------- dispatch order

// Visiting order of the (tile, species) segments for the push and deposit
// launches: decreasing particle count, so that the largest segments start
// first and the end of a launch is made of small ones (densities become
// very uneven as a plasma compresses).  Counting sort over the key
// count >> shift in one work-group of ORDER_BUCKETS threads; segments with
// equal keys come in no particular order, which the results do not depend
// on (every segment writes its own current block and counters).
constexpr int ORDER_BUCKETS = 1024;

__global__ void __launch_bounds__(ORDER_BUCKETS) k_order(const int32_t *cnt, int32_t n, int32_t shift, int32_t *order)
{
    __shared__ int hist[ORDER_BUCKETS];
    __shared__ int wsum[ORDER_BUCKETS / 64];
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    hist[tid] = 0;
    __syncthreads();
    for (int w = tid; w < n; w += ORDER_BUCKETS)
        atomicAdd(&hist[ORDER_BUCKETS - 1 - min(max(cnt[w], 0) >> shift, ORDER_BUCKETS - 1)], 1);
    __syncthreads();
    // exclusive prefix over the buckets: wave scans, then the wave totals
    const int v = hist[tid];
    int x = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int y = __shfl_up(x, o, 64);
        if (lane >= o) x += y;
    }
    if (lane == 63) wsum[wv] = x;
    __syncthreads();
    if (tid == 0) {
        int run = 0;
        for (int k = 0; k < ORDER_BUCKETS / 64; ++k) {
            const int t = wsum[k];
            wsum[k] = run;
            run += t;
        }
    }
    __syncthreads();
    hist[tid] = x - v + wsum[wv];
    __syncthreads();
    for (int w = tid; w < n; w += ORDER_BUCKETS) {
        const int pos = atomicAdd(&hist[ORDER_BUCKETS - 1 - min(max(cnt[w], 0) >> shift, ORDER_BUCKETS - 1)], 1);
        order[pos] = w;
    }
}

// -------------------------------------------------------------- binning

struct BinGeom {
    int32_t n[3], T[3], nt[3];
    int32_t ntb;          // tiles in the box
    int64_t count;        // particles of this (box, species)
    int32_t nchunks;
    int32_t chunk;        // particles per chunk
    int64_t id_base;      // origin id of input particle 0 of this (box, species)
    int32_t walls;        // the box has conducting walls at x = 0 and x = n0
    int32_t hist_lds;     // per-chunk tile histograms fit in LDS (else they stay in global memory)
};

// Tile key and tile-centre-relative position of every particle.
template <typename R, int D>
__global__ void k_bin_keys(BinGeom g, const double *pos, int32_t *key, R *xl, int32_t *err)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < g.count;
         i += (int64_t)gridDim.x * blockDim.x) {
        int tc[3] = {0, 0, 0};
        bool ok = true;
#pragma unroll
        for (int d = 0; d < D; ++d) {
            double x = pos[d * g.count + i];
            ok = ok && x >= 0.0 && x < (double)g.n[d];
            int t = (int)floor(x / g.T[d]);
            t = min(max(t, 0), g.nt[d] - 1);
            double centre = (double)t * g.T[d] + g.T[d] / 2;
            R loc = (R)(x - centre);
            const R half = R(g.T[d] / 2);
            if (loc >= half) {
                if (d == 0 && g.walls && t + 1 == g.nt[0]) {
                    loc = nextafter(half, R(0));   // stays below the wall at x = n0
                } else {
                    t = t + 1 == g.nt[d] ? 0 : t + 1;
                    loc = -half;
                }
            }
            tc[d] = t;
            xl[d * g.count + i] = loc;
        }
        if (!ok) {
            latch(err, ERR_OUT_OF_TILE);
            key[i] = -1;
        } else {
            key[i] = tc[0] + g.nt[0] * (tc[1] + g.nt[1] * tc[2]);
        }
    }
}

// Zero the wall planes (Ey, Ez, Bx at x = 0) of the tiles on a low-x wall.
template <typename R, int D>
__global__ void __launch_bounds__(256) k_hold_walls(Params<R> p)
{
    const TileDesc td = p.tiles[blockIdx.x];
    if (!(td.walls & 1)) return;
    const int T1 = D > 1 ? p.T[1] : 1, T2 = D > 2 ? p.T[2] : 1;
    const int64_t N = p.cells_total;
    for (int k = threadIdx.x; k < T1 * T2; k += blockDim.x) {
        const int gy = D > 1 ? td.tc[1] * T1 + k % T1 : 0;
        const int gz = D > 2 ? td.tc[2] * T2 + k / T1 : 0;
        const int64_t g = td.cell0 + (int64_t)td.n[0] * (gy + (int64_t)td.n[1] * gz);
        p.E[N + g] = R(0);
        p.E[2 * N + g] = R(0);
        p.B[g] = R(0);
    }
}

// Per-chunk tile histograms.
__global__ void k_bin_hist(BinGeom g, const int32_t *key, int32_t *hist)
{
    extern __shared__ int sh[];
    int32_t *row = hist + (int64_t)blockIdx.x * g.ntb;
    const int64_t lo = (int64_t)blockIdx.x * g.chunk, hi = min(g.count, lo + g.chunk);
    if (!g.hist_lds) {
        // too many tiles for LDS: count straight into the (zeroed) row
        for (int64_t i = lo + threadIdx.x; i < hi; i += blockDim.x) {
            const int k = key[i];
            if (k >= 0) atomicAdd(&row[k], 1);
        }
        return;
    }
    for (int k = threadIdx.x; k < g.ntb; k += blockDim.x) sh[k] = 0;
    __syncthreads();
    for (int64_t i = lo + threadIdx.x; i < hi; i += blockDim.x) {
        int k = key[i];
        if (k >= 0) atomicAdd(&sh[k], 1);
    }
    __syncthreads();
    for (int k = threadIdx.x; k < g.ntb; k += blockDim.x) row[k] = sh[k];
}

// Chunk start offsets per tile, in (tile, chunk) order, and segment counts.
__global__ void k_bin_scan(BinGeom g, int32_t *hist, int32_t *seg_cnt, const int32_t *seg_cap, int tile0,
                           int nspecies, int species, int32_t *err)
{
    for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < g.ntb; k += gridDim.x * blockDim.x) {
        const int ts = (tile0 + k) * nspecies + species;
        int run = seg_cnt[ts];
        for (int c = 0; c < g.nchunks; ++c) {
            int v = hist[(int64_t)c * g.ntb + k];
            hist[(int64_t)c * g.ntb + k] = run;
            run += v;
        }
        if (run > seg_cap[ts]) {
            latch(err, ERR_CAPACITY);
            run = seg_cap[ts];
        }
        seg_cnt[ts] = run;
    }
}

// Stable scatter: one wave per chunk walks its particles in order, 64 at a
// time; equal keys among the 64 lanes are ranked with ballots.
template <typename R, int D>
__global__ void __launch_bounds__(64) k_bin_scatter(BinGeom g, const int32_t *key, const R *xl, const double *u64,
                                                    const int32_t *hist, Params<R> p, int tile0, int species)
{
    extern __shared__ int sh[];
    // running slot of every tile for this chunk: in LDS, or, for boxes with
    // too many tiles, the chunk's own row of offsets in global memory (only
    // this wave touches it; updated with atomics, which keep their order)
    int32_t *grow = const_cast<int32_t *>(hist) + (int64_t)blockIdx.x * g.ntb;
    if (g.hist_lds) {
        for (int k = threadIdx.x; k < g.ntb; k += 64) sh[k] = grow[k];
        __syncthreads();
    }
    int nbits = 0;
    while ((1 << nbits) < g.ntb) ++nbits;
    const int64_t lo = (int64_t)blockIdx.x * g.chunk, hi = min(g.count, lo + g.chunk);
    const int lane = threadIdx.x;
    const int64_t cap = p.cap_total;
    for (int64_t base = lo; base < hi; base += 64) {
        const int64_t i = base + lane;
        const int k = i < hi ? key[i] : -1;
        const bool valid = k >= 0;
        unsigned long long m = __ballot(valid);
        for (int b = 0; b < nbits; ++b) {
            unsigned long long bb = __ballot((k >> b) & 1);
            m &= ((k >> b) & 1) ? bb : ~bb;
        }
        const int rank = lanes_below(m);
        const int lead = valid ? __ffsll((long long)m) - 1 : lane;
        int old = 0;
        if (valid && lane == lead) {
            if (g.hist_lds) {
                old = sh[k];
                sh[k] = old + __popcll(m);
            } else {
                old = atomicAdd(&grow[k], __popcll(m));
            }
        }
        old = __shfl(old, lead, 64);      // the lead lane of this lane's key
        if (valid) {
            const int ts = (tile0 + k) * p.nspecies + species;
            const int slot = old + rank;
            if (slot < p.seg_cap[ts]) {
                const int64_t dst = p.seg_off[ts] + slot;
#pragma unroll
                for (int d = 0; d < D; ++d) p.pos[d * cap + dst] = xl[d * g.count + i];
#pragma unroll
                for (int mm = 0; mm < 3; ++mm) p.u[mm * cap + dst] = (R)u64[mm * g.count + i];
                if (p.ids) p.ids[dst] = g.id_base < 0 ? -1 : (int32_t)(g.id_base + i);   // index in the concatenated input
            }
        }
    }
}

// ------------------------------------------------------------ diagnostics

__device__ __forceinline__ double wg_sum(double v, double *sh)
{
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
    __syncthreads();
    if (lane == 0) sh[wave] = v;
    __syncthreads();
    double s = 0;
    for (int w = 0; w < nw; ++w) s += sh[w];
    return s;
}

__device__ __forceinline__ double wg_max(double v, double *sh)
{
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o));
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
    __syncthreads();
    if (lane == 0) sh[wave] = v;
    __syncthreads();
    double s = 0;
    for (int w = 0; w < nw; ++w) s = fmax(s, sh[w]);
    return s;
}

constexpr int NPART = 8;   // partial values per tile

// Per tile: field energy, max |div+ B|, kinetic energy, particle count, the
// near-face count, and the cloud-in-cell charge block (nodes 0..T per
// dimension, FP64).
template <typename R, int D>
__global__ void __launch_bounds__(256) k_diag_tile(Params<R> p, const double *mass, double *part, double *rblk)
{
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ double red[MAX_WAVES];
    double *sR = reinterpret_cast<double *>(smem);
    const int t = blockIdx.x;
    const TileDesc td = p.tiles[t];
    const int T0 = p.T[0], T1 = D > 1 ? p.T[1] : 1, T2 = D > 2 ? p.T[2] : 1;
    const int r0 = T0 + 1, r1 = D > 1 ? T1 + 1 : 1, r2 = D > 2 ? T2 + 1 : 1;
    const int nr = r0 * r1 * r2;
    for (int k = threadIdx.x; k < nr; k += blockDim.x) sR[k] = 0.0;
    const int64_t N = p.cells_total;
    const int n0 = td.n[0], n1 = td.n[1], n2 = td.n[2];
    double ef = 0.0, divb = 0.0;
    const int ncell = T0 * T1 * T2;
    for (int k = threadIdx.x; k < ncell; k += blockDim.x) {
        const int gx = td.tc[0] * T0 + k % T0;
        const int gy = D > 1 ? td.tc[1] * T1 + (k / T0) % T1 : 0;
        const int gz = D > 2 ? td.tc[2] * T2 + k / (T0 * T1) : 0;
        auto at = [&](int x, int y, int z) -> int64_t {
            return td.cell0 + x + (int64_t)n0 * (y + (int64_t)n1 * z);
        };
        const int64_t g = at(gx, gy, gz);
        for (int m = 0; m < 3; ++m) {
            double e = p.E[m * N + g], b = p.B[m * N + g];
            ef += e * e + b * b;
        }
        const int64_t ip = at(gx + 1 == n0 ? 0 : gx + 1, gy, gz);
        const int64_t jp = at(gx, gy + 1 == n1 ? 0 : gy + 1, gz);
        const int64_t kp = at(gx, gy, gz + 1 == n2 ? 0 : gz + 1);
        double dv = ((double)p.B[ip] - (double)p.B[g]) + ((double)p.B[N + jp] - (double)p.B[N + g]) +
                    ((double)p.B[2 * N + kp] - (double)p.B[2 * N + g]);
        divb = fmax(divb, fabs(dv));
    }
    __syncthreads();
    double ek = 0.0, np_ = 0.0;
    const int64_t cap = p.cap_total;
    for (int s = 0; s < p.nspecies; ++s) {
        const int ts = t * p.nspecies + s;
        const int64_t so = p.seg_off[ts];
        const int cnt = p.seg_cnt[ts];
        const double q = (double)p.charge[td.box * p.nspecies + s];
        const double ms = mass[td.box * p.nspecies + s];
        if (threadIdx.x == 0) np_ += cnt;
        for (int i = threadIdx.x; i < cnt; i += blockDim.x) {
            double u0 = p.u[so + i], u1 = p.u[cap + so + i], u2 = p.u[2 * cap + so + i];
            ek += ms * (sqrt(1.0 + u0 * u0 + u1 * u1 + u2 * u2) - 1.0);
            int b[3] = {0, 0, 0};
            double w[3] = {0, 0, 0};
            bool ok = true;
#pragma unroll
            for (int d = 0; d < D; ++d) {
                double x = p.pos[d * cap + so + i];
                double fl = floor(x);
                b[d] = (int)fl + p.T[d] / 2;
                w[d] = x - fl;
                ok = ok && b[d] >= 0 && b[d] < p.T[d];
            }
            if (!ok) continue;
            for (int cn = 0; cn < (1 << D); ++cn) {
                int idx = 0, stride = 1;
                double wt = q;
#pragma unroll
                for (int d = 0; d < D; ++d) {
                    int bit = (cn >> d) & 1;
                    idx += (b[d] + bit) * stride;
                    stride *= p.T[d] + 1;
                    wt *= bit ? w[d] : 1.0 - w[d];
                }
                atomicAdd(&sR[idx], wt);
            }
        }
    }
    const double c2 = (double)p.c * (double)p.c;
    double s_ef = wg_sum(ef, red);
    double s_ek = wg_sum(ek, red);
    double m_db = wg_max(divb, red);
    double s_np = wg_sum(np_, red);
    if (threadIdx.x == 0) {
        double *o = part + (int64_t)t * NPART;
        o[0] = 0.5 * s_ef;
        o[1] = m_db;
        o[2] = c2 * s_ek;
        o[3] = s_np;
        double nf = 0;
        for (int s = 0; s < p.nspecies; ++s) nf += p.nf_seg[t * p.nspecies + s];
        o[7] = nf;
    }
    __syncthreads();
    double *blk = rblk + (int64_t)t * nr;
    for (int k = threadIdx.x; k < nr; k += blockDim.x) blk[k] = sR[k];
}

// Per tile: rho on nodes from the charge blocks of the tile and of its lower
// neighbours, Gauss residual max |div- E - rho| and total charge.
template <typename R, int D>
__global__ void __launch_bounds__(256) k_diag_gauss(Params<R> p, double *part, const double *rblk, double *rho_prev,
                                                    int cont_valid)
{
    __shared__ double red[MAX_WAVES];
    const int t = blockIdx.x;
    const TileDesc td = p.tiles[t];
    const int T0 = p.T[0], T1 = D > 1 ? p.T[1] : 1, T2 = D > 2 ? p.T[2] : 1;
    const int r0 = T0 + 1, r1 = D > 1 ? T1 + 1 : 1, r2 = D > 2 ? T2 + 1 : 1;
    const int nr = r0 * r1 * r2;
    (void)r2;
    const int64_t N = p.cells_total;
    const int n0 = td.n[0], n1 = td.n[1];
    double gmax = 0.0, qsum = 0.0, cmax = 0.0;
    const int ncell = T0 * T1 * T2;
    for (int k = threadIdx.x; k < ncell; k += blockDim.x) {
        const int l[3] = {k % T0, (k / T0) % T1, k / (T0 * T1)};
        double rho = 0.0;
        for (int oz = (D > 2 ? -1 : 0); oz <= 0; ++oz)
            for (int oy = (D > 1 ? -1 : 0); oy <= 0; ++oy)
                for (int ox = -1; ox <= 0; ++ox) {
                    const int o[3] = {ox, oy, oz};
                    int bi[3] = {0, 0, 0}, nc[3] = {0, 0, 0};
                    bool in = true;
                    for (int d = 0; d < 3; ++d) {
                        if (d < D) {
                            bi[d] = l[d] - o[d] * p.T[d];
                            in = in && bi[d] <= p.T[d];
                            nc[d] = wrapi(td.tc[d] + o[d], td.nt[d]);
                        }
                    }
                    if (!in) continue;
                    const int nid = td.tile0 + nc[0] + td.nt[0] * (nc[1] + td.nt[1] * nc[2]);
                    rho += rblk[(int64_t)nid * nr + bi[0] + r0 * (bi[1] + r1 * bi[2])];
                }
        const int gx = td.tc[0] * T0 + l[0];
        const int gy = D > 1 ? td.tc[1] * T1 + l[1] : 0;
        const int gz = D > 2 ? td.tc[2] * T2 + l[2] : 0;
        auto at = [&](int x, int y, int z) -> int64_t {
            return td.cell0 + x + (int64_t)n0 * (y + (int64_t)n1 * z);
        };
        const int64_t g = at(gx, gy, gz);
        const int64_t im = at(gx == 0 ? td.n[0] - 1 : gx - 1, gy, gz);
        const int64_t jm = at(gx, gy == 0 ? td.n[1] - 1 : gy - 1, gz);
        const int64_t km = at(gx, gy, gz == 0 ? td.n[2] - 1 : gz - 1);
        double dive = ((double)p.E[g] - (double)p.E[im]) + ((double)p.E[N + g] - (double)p.E[N + jm]) +
                      ((double)p.E[2 * N + g] - (double)p.E[2 * N + km]);
        // the wall plane carries the conductor's surface charge: no Gauss law there
        const bool wall = (td.walls & 1) && gx == 0;
        if (!wall) gmax = fmax(gmax, fabs(dive - rho));
        qsum += rho;
        // discrete continuity against the charge of the previous call
        if (cont_valid && !wall) {
            const double divj = ((double)p.J[g] - (double)p.J[im]) + ((double)p.J[N + g] - (double)p.J[N + jm]) +
                                ((double)p.J[2 * N + g] - (double)p.J[2 * N + km]);
            cmax = fmax(cmax, fabs(rho - rho_prev[g] + divj));
        }
        rho_prev[g] = rho;
    }
    double m = wg_max(gmax, red);
    double s = wg_sum(qsum, red);
    double cm = wg_max(cmax, red);
    if (threadIdx.x == 0) {
        part[(int64_t)t * NPART + 4] = m;
        part[(int64_t)t * NPART + 5] = s;
        part[(int64_t)t * NPART + 6] = cm;
    }
}

// The diagnostics of all tiles reduced into one record.
struct DiagRec {
    double field_energy, divb_max, kinetic_energy, gauss_max, charge_total, continuity_max;
    long long particles, near_face;
};

// Sum the per-tile partials of k_diag_tile / k_diag_gauss in tile order on
// one thread: the same order and arithmetic as a host loop over the tiles,
// so the record equals the host reduction of the same partials.
__global__ void k_diag_reduce(const double *part, int64_t ntiles, int cont_valid, DiagRec *rec)
{
    if (blockIdx.x != 0 || threadIdx.x != 0) return;
    DiagRec r{};
    r.continuity_max = cont_valid ? 0.0 : -1.0;
    for (int64_t t = 0; t < ntiles; ++t) {
        const double *o = part + t * NPART;
        r.field_energy += o[0];
        r.divb_max = fmax(r.divb_max, o[1]);
        r.kinetic_energy += o[2];
        r.particles += (long long)o[3];
        r.gauss_max = fmax(r.gauss_max, o[4]);
        r.charge_total += o[5];
        if (cont_valid) r.continuity_max = fmax(r.continuity_max, o[6]);
        r.near_face += (long long)o[7];
    }
    *rec = r;
}

}  // namespace pic
