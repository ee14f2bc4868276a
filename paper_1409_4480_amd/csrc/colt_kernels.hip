// HIP kernels of the Lyman-alpha transport library (gfx950).
//
//  k_cell_setup   per-cell line quantities from (n_HI, T, v, k_dust)
//  k_nonlocal     per-cell non-local a*tau estimate (six axis paths)
//  k_transport    persistent photon-pool transport: each lane carries one
//                 photon through emission, cell-by-cell ray tracing,
//                 scattering and the event-cell part of its next-event
//                 estimates; a lane whose photon has escaped or been absorbed
//                 takes the next photon from a shared queue (one atomic per
//                 wave per refill); a stopped launch suspends its photons
//  k_peel         persistent next-event marches beyond the event's cell
//  k_plan, k_advance   device-side slicing of jobs before and after a launch
//  k_voigt, k_sample   device checks of H(a,x) and of the samplers
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <mutex>

#include "colt_device.h"
#include "colt_internal.h"
#include "colt_launch.h"

#ifndef COLT_FP32_MIN_BLOCKS
#define COLT_FP32_MIN_BLOCKS 4
#endif
#ifndef COLT_FP64_MIN_BLOCKS
#define COLT_FP64_MIN_BLOCKS 2
#endif
// FP32 camera kernels: two workgroups per CU leave them ~185 VGPRs and no
// spill, measured faster than three with a few dozen bytes of spill per lane
#ifndef COLT_FP32_CAM_MIN_BLOCKS
#define COLT_FP32_CAM_MIN_BLOCKS 2
#endif
#ifndef COLT_PEEL_MIN_BLOCKS
#define COLT_PEEL_MIN_BLOCKS 4
#endif

namespace colt {

// ---------------------------------------------------------------------------
// Cell set-up (Sec. 2): T4 = T/1e4, v_th = 12.85 T4^1/2 km/s, a = 4.702e-4
// T4^-1/2, sigma0 = 5.898e-14 T4^-1/2 cm^2, recoil g = 2.536e-4 T4^-1/2; the
// core-wing crossover x_cw from its rational fit in ln a (Sec. 3.2.2); the
// Jeans estimate a tau_J = 6.428e4 T4^-1/2 n^1/2 (Sec. 3.2.4).
// Opacities are stored per grid unit (dx_cm), velocities in units of v_th.
// ---------------------------------------------------------------------------
__global__ void k_cell_setup(int64_t n, const double *__restrict__ n_HI,
                             const double *__restrict__ T, const double *__restrict__ v,
                             const double *__restrict__ k_dust,
                             const double *__restrict__ atau_nl, double dx_cm,
                             CellRec<double> *__restrict__ rd, CellAux<double> *__restrict__ ad,
                             CellRec<float> *__restrict__ rf, int rf_stride,
                             CellAux<float> *__restrict__ af)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double T4 = T[i] / 1.0e4;
    const double sq = ::sqrt(T4);
    const double vth = kVthRef * sq;
    const double a = 4.702e-4 / sq;
    const double sigma0 = 5.898e-14 / sq;
    const double k0 = n_HI[i] * sigma0;
    const double xcw = 6.9184721 + 81.766279 / (::log(a) - 14.651253);
    const double g = 2.536e-4 / sq;
    const double kd = k_dust ? k_dust[i] : 0.0;
    const double vx = v ? v[3 * i] : 0.0, vy = v ? v[3 * i + 1] : 0.0, vz = v ? v[3 * i + 2] : 0.0;
    CellRec<double> c;
    c.k0 = k0 * dx_cm;
    c.a = a;
    c.s = kVthRef / vth;
    c.kd = kd * dx_cm;
    c.ux = vx / vth;
    c.uy = vy / vth;
    c.uz = vz / vth;
    c.xcw = xcw;
    rd[i] = c;
    CellAux<double> x;
    x.g = g;
    x.atau_nl = atau_nl ? atau_nl[i] : 0.0;
    // a tau across one Jeans length of the cell's gas (Sec. 3.2.4, eq. atau0J)
    x.atau_j = 6.428e4 / sq * ::sqrt(n_HI[i]);
    x.pad = 0.0;
    ad[i] = x;
    CellRec<float> cf;
    cf.k0 = (float)c.k0; cf.a = (float)c.a; cf.s = (float)c.s; cf.kd = (float)c.kd;
    cf.ux = (float)c.ux; cf.uy = (float)c.uy; cf.uz = (float)c.uz; cf.xcw = (float)c.xcw;
    rf[i * rf_stride] = cf;
    CellAux<float> xf;
    xf.g = (float)x.g;
    xf.atau_nl = (float)x.atau_nl;
    xf.atau_j = (float)x.atau_j;
    xf.pad = 0.0f;
    af[i] = xf;
}

// ---------------------------------------------------------------------------
// Geometry.  Cells are half-open; a point on a face belongs to the cell the
// photon moves into.  Positions are in grid units from the lower box corner.
// ---------------------------------------------------------------------------
struct CellBox {
    double lo[3];
    double size;
    int32_t cell;
};

__device__ __forceinline__ int side_of(double r, double mid, double k)
{
    return (r > mid) ? 1 : ((r < mid) ? 0 : ((k < 0.0) ? 0 : 1));
}

// Finds the cell holding r for a photon moving along k; false if r is outside
// the domain (box or escape sphere).
__device__ __forceinline__ bool locate(const GridView &g, const double r[3], const double k[3], CellBox &c)
{
    int ib[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const double n = (double)g.n[d];
        if (r[d] < 0.0 || r[d] > n) return false;
        if (r[d] == n && k[d] >= 0.0) return false;
        if (r[d] == 0.0 && k[d] < 0.0) return false;
        const double f = ::floor(r[d]);
        int i = (int)f;
        if (r[d] == f && k[d] < 0.0) i -= 1;
        i = (i < 0) ? 0 : ((i >= g.n[d]) ? g.n[d] - 1 : i);
        ib[d] = i;
    }
    if (g.esc_r > 0.0) {
        double d2 = 0.0;
#pragma unroll
        for (int d = 0; d < 3; ++d) d2 += (r[d] - g.centre[d]) * (r[d] - g.centre[d]);
        if (d2 >= g.esc_r * g.esc_r) return false;
    }
    const int flat = (ib[2] * g.n[1] + ib[1]) * g.n[0] + ib[0];
    c.lo[0] = ib[0]; c.lo[1] = ib[1]; c.lo[2] = ib[2];
    c.size = 1.0;
    if (g.kind == 0) {
        c.cell = flat;
        return true;
    }
    int node = g.base[flat];
    int ch = g.child[node];
    double size = 1.0;
    while (ch >= 0) {
        const double half = 0.5 * size;
        int oct = 0;
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            const int b = side_of(r[d], c.lo[d] + half, k[d]);
            if (b) c.lo[d] += half;
            oct |= b << d;
        }
        node = ch + oct;
        size = half;
        ch = g.child[node];
    }
    c.size = size;
    c.cell = -ch - 1;
    return true;
}

// Distance to the exit of cell c along k (inverse components ik), nearest face
// first-axis on ties, or to the escape sphere (by_sphere) if nearer or equal.
__device__ __forceinline__ double exit_distance(const GridView &g, const CellBox &c,
                                                const double r[3], const double k[3],
                                                const double ik[3], int &axis, bool &by_sphere)
{
    double best = __builtin_inf();
    axis = 0;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        double t;
        if (k[d] > 0.0) t = (c.lo[d] + c.size - r[d]) * ik[d];
        else if (k[d] < 0.0) t = (c.lo[d] - r[d]) * ik[d];
        else continue;
        t = (t < 0.0) ? 0.0 : t;
        if (t < best) { best = t; axis = d; }
    }
    by_sphere = false;
    if (g.esc_r > 0.0) {
        double b = 0.0, rr = 0.0;
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            const double rc = r[d] - g.centre[d];
            b += rc * k[d];
            rr += rc * rc;
        }
        // The sphere lies at least esc_r - |rc| away and the cell exit at most
        // one cell diagonal (2 sizes bound it): skip the root when the sphere
        // cannot be the nearer exit (the result is the same either way).
        const double reach = g.esc_r - 2.0 * c.size;
        if (reach <= 0.0 || rr >= reach * reach) {
            const double disc = b * b - (rr - g.esc_r * g.esc_r);
            double t = (disc > 0.0) ? -b + ::sqrt(disc) : 0.0;
            t = (t < 0.0) ? 0.0 : t;
            if (t <= best) { best = t; by_sphere = true; }
        }
    }
    return best;
}

// Moves a photon on the exit face of `axis` into the next cell; false if it
// leaves the domain.  The axis is selected with explicit branches so that the
// position and cell arrays stay in registers.
__device__ __forceinline__ void snap_face(CellBox &c, double r[3], const double k[3], int axis,
                                          int &step)
{
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        if (d == axis) {
            step = (k[d] > 0.0) ? 1 : -1;
            r[d] = (k[d] > 0.0) ? c.lo[d] + c.size : c.lo[d];
        }
    }
}

// Octree crossing through the leaf's neighbour link: the leaf across the face
// (same level or coarser), read straight from the link, or the refined node
// across at the leaf's level, which is descended.  Where r lies on one of that
// cell's other faces and k points out of it, the tie rules of the search from
// the root could pick a diagonal cell, so that case, and links the set-up could
// not encode, use the search.  Either way the cell is the one locate() finds.
__device__ __forceinline__ bool cross_octree(const GridView &g, CellBox &c, const double r[3],
                                             const double k[3], int axis, int step)
{
    const uint32_t e = g.rope[(size_t)c.cell * g.rope_stride + 2 * axis + (step > 0 ? 1 : 0)];
    if (e == 0xFFFFFFFFu) return false;                  // the domain face
    if (e == 0xFFFFFFFEu) return locate(g, r, k, c);
    const bool leaf = (e >> 31) != 0u;
    const int up = (int)((e >> 27) & 15u);
    const int idx = (int)(e & 0x7FFFFFFu);
    const double size = c.size * (double)(1u << up);     // exact (powers of two)
    const double inv_size = 1.0 / size;                   // exact as well
    double lo[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const double x = (d == axis) ? ((step > 0) ? c.lo[d] + c.size : c.lo[d] - c.size)
                                     : c.lo[d];
        lo[d] = (up == 0) ? x : ::floor(x * inv_size) * size;   // exact: size is 2^k
    }
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        if (d == axis) continue;
        if ((r[d] == lo[d] && k[d] < 0.0) || (r[d] == lo[d] + size && !(k[d] < 0.0)))
            return locate(g, r, k, c);
    }
    if (g.esc_r > 0.0) {
        double d2 = 0.0;
#pragma unroll
        for (int d = 0; d < 3; ++d) d2 += (r[d] - g.centre[d]) * (r[d] - g.centre[d]);
        if (d2 >= g.esc_r * g.esc_r) return false;
    }
    c.lo[0] = lo[0]; c.lo[1] = lo[1]; c.lo[2] = lo[2];
    if (leaf) {
        c.size = size;
        c.cell = idx;
        return true;
    }
    double sz = size;
    int node = idx;
    int ch = g.child[node];
    while (ch >= 0) {
        const double half = 0.5 * sz;
        int oct = 0;
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            const int b = side_of(r[d], c.lo[d] + half, k[d]);
            if (b) c.lo[d] += half;
            oct |= b << d;
        }
        node = ch + oct;
        sz = half;
        ch = g.child[node];
    }
    c.size = sz;
    c.cell = -ch - 1;
    return true;
}

__device__ __forceinline__ bool cross(const GridView &g, CellBox &c, double r[3],
                                      const double k[3], int axis)
{
    int step = 0;
    snap_face(c, r, k, axis, step);
    if (g.kind == 0) {
        bool inside = true;
        int stride = 1;
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            if (d == axis) {
                const int i = (int)c.lo[d] + step;
                inside = (i >= 0) && (i < g.n[d]);
                c.lo[d] = (double)i;
                c.cell += step * stride;
            }
            stride *= g.n[d];
        }
        return inside;
    }
    if (g.rope) return cross_octree(g, c, r, k, axis, step);
    return locate(g, r, k, c);
}

__device__ __forceinline__ double min_face_distance(const CellBox &c, const double r[3])
{
    double m = __builtin_inf();
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const double lo = r[d] - c.lo[d], hi = c.lo[d] + c.size - r[d];
        m = (lo < m) ? lo : m;
        m = (hi < m) ? hi : m;
    }
    return (m < 0.0) ? 0.0 : m;
}

template <typename R>
__device__ __forceinline__ CellRec<R> load_cell(const GridView &g, int32_t i)
{
    return reinterpret_cast<const CellRec<R> *>(g.cells)[(size_t)i * g.rec_stride];
}

template <typename R>
__device__ __forceinline__ CellAux<R> load_aux(const GridView &g, int32_t i)
{
    return reinterpret_cast<const CellAux<R> *>(g.aux)[i];
}

__device__ __forceinline__ int bin_of(double x, double lo, double hi, int n)
{
    if (x < lo) return 0;
    const double t = (x - lo) / (hi - lo) * n;
    if (t >= n) return n + 1;
    return 1 + (int)t;
}

// Per-lane event counters.  They live in LDS (64-bit, one column per lane of
// the workgroup), so counting takes no registers and no wait: an event adds
// to the lane's own column, and the column is flushed to the job's spread
// counter slots when the lane changes job and at the end.
constexpr int kLaneCounters = 12;
constexpr int kMaxBlock = 256;

// C_ROUNDS (cooperative sampler rounds) and C_PASSES (wave-loop passes) are
// counted once per wave, by its first lane.
enum { C_EMITTED = 0, C_ESCAPED, C_ABSORBED, C_SCAT_HI, C_SCAT_DUST, C_CROSSINGS, C_PEELS,
       C_UPAR_TRIES, C_PEEL_CROSSINGS, C_CAPPED, C_ROUNDS, C_PASSES };

struct LaneCounters {
    unsigned long long *col;     // &counts[0][threadIdx.x] in the workgroup's LDS table
    __device__ __forceinline__ void add(int c, uint32_t by = 1u)
    {
        atomicAdd(col + c * kMaxBlock, (unsigned long long)by);
    }
};

__device__ __forceinline__ void flush_counters(const JobView *J, LaneCounters &lc, int slot)
{
    unsigned long long *dst = J->counters + (size_t)slot * kNumCounters;
#pragma unroll
    for (int i = 0; i < kLaneCounters; ++i) {
        const unsigned long long v = lc.col[i * kMaxBlock];
        if (v) atomicAdd(dst + i, v);
        lc.col[i * kMaxBlock] = 0ull;
    }
}

// End of a single-job launch: the wave sums its lanes' columns first, so the
// job's counters take one atomic per counter per wave.  All 64 lanes call it.
__device__ __forceinline__ void flush_counters_wave(const JobView *J, LaneCounters &lc, int slot)
{
    unsigned long long *dst = J->counters + (size_t)slot * kNumCounters;
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int i = 0; i < kLaneCounters; ++i) {
        unsigned long long v = lc.col[i * kMaxBlock];
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
        if (lane == 0 && v) atomicAdd(dst + i, v);
        lc.col[i * kMaxBlock] = 0ull;
    }
}

template <typename R>
struct Photon {
    double r[3];
    R kr[3];          // direction in the bulk precision
    double ik[3];     // FP64: 1 / k (FP32-bulk recomputes it where needed)
    R x;              // lab-frame frequency (Doppler widths at 1e4 K)
    double tau;       // optical depth left to the next interaction
    CellBox c;
    uint64_t events;
    int32_t nscat;
    int32_t status;   // 0 alive, 1 escaped, 2 absorbed, 3 capped
    Rng<R> rng;       // its counter space also carries the photon id
    __device__ __forceinline__ uint64_t id() const
    {
        return ((uint64_t)rng.key.id1 << 32) | rng.key.id0;
    }
};

template <typename R>
__device__ __forceinline__ void set_dir(Photon<R> &p, R kx, R ky, R kz)
{
    p.kr[0] = kx; p.kr[1] = ky; p.kr[2] = kz;
    if constexpr (sizeof(R) == 8) {
#pragma unroll
        for (int d = 0; d < 3; ++d) p.ik[d] = (p.kr[d] != 0.0) ? 1.0 / p.kr[d] : 0.0;
    }
}

// Direction and its inverse for the geometry, in double.  FP32-bulk takes
// 1/k from the single-precision reciprocal, as accurate as the FP32 direction
// itself; FP64 uses the exact quotients kept with the photon.
template <typename R>
__device__ __forceinline__ void geom_dir(const Photon<R> &p, double k[3], double ik[3])
{
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        k[d] = (double)p.kr[d];
        if constexpr (sizeof(R) == 8)
            ik[d] = p.ik[d];
        else
            ik[d] = (p.kr[d] != 0.0f) ? (double)__builtin_amdgcn_rcpf(p.kr[d]) : 0.0;
    }
}

template <typename R>
__device__ __forceinline__ void isotropic_dir(Photon<R> &p)
{
    using F = Fn<R>;
    const R mu = R(2) * p.rng.next() - R(1);
    const R Rphi = p.rng.next();
    R c, s;
    F::cossin2pi(Rphi, c, s);
    const R st = F::sqrt(R(1) - mu * mu);
    set_dir(p, st * c, st * s, mu);
}

// What an event contributes toward camera direction d: comoving frequency
// base + d.ua + g (k.d - 1) and phase weight (1 + rW (k.d)^2) / (1 + rW/3).
// Emission: base = x_nat, ua = atom velocity; dust: base = x, ua = 0; H I:
// base = x - u_par, ua = atom velocity, with recoil g and the event's rW.
template <typename R>
struct PeelSource {
    R base, grec, rW;
    R ua[3];
};

// W exp(-tau) of camera `cam` into its spectrum bin and image pixel (and the
// photon's record).
__device__ __forceinline__ void peel_tally(const JobView &J, int cam, int bin, int pix,
                                           uint64_t id, double w)
{
    if (J.record) atomicAdd(J.rec_peel + id * J.n_cams + cam, w);
    if (bin >= 1 && bin <= J.cam_nbins)
        atomicAdd(J.cam_spec + (size_t)cam * J.cam_nbins + (bin - 1), w);
    if (pix >= 0) atomicAdd(J.cam_img + (size_t)cam * J.npix * J.npix + pix, w);
}

// Image pixel of position r (grid units) for camera table entry cam:
// orthographic projection onto the camera's (u, v) axes about the box centre.
__device__ __forceinline__ int pixel_of(const JobView &J, const double *cam, const double r[3])
{
    if (J.npix <= 0) return -1;
    double pu = 0.0, pv = 0.0;
#pragma unroll
    for (int e = 0; e < 3; ++e) {
        const double rc = r[e] - J.g.centre[e];
        pu += rc * cam[6 + e];
        pv += rc * cam[9 + e];
    }
    pu = pu / J.fov + 0.5;
    pv = pv / J.fov + 0.5;
    if (!(pu >= 0.0 && pu < 1.0 && pv >= 0.0 && pv < 1.0)) return -1;
    int iu = (int)(pu * J.npix), iv = (int)(pv * J.npix);
    iu = (iu >= J.npix) ? J.npix - 1 : iu;
    iv = (iv >= J.npix) ? J.npix - 1 : iv;
    return iv * J.npix + iu;
}

// Camera spectrum bin and image pixel for the march kernel: the forms of
// bin_of and pixel_of with their divisions replaced by products with
// reciprocals taken once per launch (a bin or pixel can differ from the
// quotient form only where a value lies within a rounding of an edge).
struct BinPixScale {
    double bin_lo, bin_scale, inv_fov;
};

__device__ __forceinline__ int bin_scaled(double x, const BinPixScale &q, int n)
{
    if (x < q.bin_lo) return 0;
    const double t = (x - q.bin_lo) * q.bin_scale;
    if (t >= n) return n + 1;
    return 1 + (int)t;
}

__device__ __forceinline__ int pixel_scaled(const JobView &J, const BinPixScale &q,
                                            const double *cam, const double r[3])
{
    if (J.npix <= 0) return -1;
    double pu = 0.0, pv = 0.0;
#pragma unroll
    for (int e = 0; e < 3; ++e) {
        const double rc = r[e] - J.g.centre[e];
        pu += rc * cam[6 + e];
        pv += rc * cam[9 + e];
    }
    pu = pu * q.inv_fov + 0.5;
    pv = pv * q.inv_fov + 0.5;
    if (!(pu >= 0.0 && pu < 1.0 && pv >= 0.0 && pv < 1.0)) return -1;
    int iu = (int)(pu * J.npix), iv = (int)(pv * J.npix);
    iu = (iu >= J.npix) ? J.npix - 1 : iu;
    iv = (iv >= J.npix) ? J.npix - 1 : iv;
    return iv * J.npix + iu;
}

// Optical depth of the cell c from r along camera direction d (inverse id)
// to its exit, for lab frequency xl (the cell's line data in cr); the exit
// axis and whether it is the escape sphere are returned.
template <typename R>
__device__ __forceinline__ double peel_cell_tau(const JobView &J, const CellBox &c,
                                                const CellRec<R> &cr, const double r[3],
                                                const double d[3], const double id[3],
                                                const R dr[3], R xl, double &l, int &axis,
                                                bool &by_sphere)
{
    l = exit_distance(J.g, c, r, d, id, axis, by_sphere);
    const R xloc = xl * cr.s - (dr[0] * cr.ux + dr[1] * cr.uy + dr[2] * cr.uz);
    const R kt = cr.k0 * voigt_H<R>(cr.a, xloc) + cr.kd;
    return (double)kt * l;
}

// March-task slots a lane holds: it reserves kTaskChunk consecutive slots of
// its sub-buffer at a time (slot == end: none held).
struct TaskCursor {
    uint32_t slot, end;
};

// Marks the lane's unused reserved slots as empty (cam = -1).
__device__ __forceinline__ void close_tasks(const JobView &J, TaskCursor &tc)
{
    for (; tc.slot < tc.end; ++tc.slot) J.task.cam[tc.slot] = -1;
}

// The next-event estimate of one event (Sec. 6.1, eq. SB) for every camera:
// W(mu_c) and the frequency x_c the photon would have toward the camera, from
// the event's own atom velocity; then the optical depth across the rest of the
// event's cell.  Above the cut-off the contribution is nil; a march that leaves
// the domain through the escape sphere inside the cell is tallied at once; any
// other march is written as a task (event position, cell, frequency, weight)
// for the march kernel, which follows it to the domain edge.  A lane whose
// sub-buffer fills past the high-water mark asks the launch to stop.
template <typename R>
__device__ __forceinline__ void peel_event(const JobView &J, const double *cams,
                                           const Photon<R> &p, const CellRec<R> &cr,
                                           const PeelSource<R> &ps, const R kin[3],
                                           TaskCursor &tc, int sub, unsigned int *stop_dev,
                                           LaneCounters &lc)
{
    using F = Fn<R>;
    const R wn = R(1) + F::div(ps.rW, R(3));
    // every camera's estimate crosses at least the event's own cell
    lc.add(C_PEELS, (uint32_t)J.n_cams);
    lc.add(C_PEEL_CROSSINGS, (uint32_t)J.n_cams);
    for (int i = 0; i < J.n_cams; ++i) {
        const double *cam = cams + 12 * i;
        const double d[3] = {cam[0], cam[1], cam[2]};
        const double id[3] = {cam[3], cam[4], cam[5]};
        const R dr[3] = {(R)cam[0], (R)cam[1], (R)cam[2]};
        const R muc = kin[0] * dr[0] + kin[1] * dr[1] + kin[2] * dr[2];
        const R W = F::div(R(1) + ps.rW * muc * muc, wn);
        const R xc = ps.base + (dr[0] * ps.ua[0] + dr[1] * ps.ua[1] + dr[2] * ps.ua[2]) +
                     ps.grec * (muc - R(1));
        const R xl = F::div(xc + (dr[0] * cr.ux + dr[1] * cr.uy + dr[2] * cr.uz), cr.s);
        double l;
        int axis;
        bool by_sphere;
        const double tau = peel_cell_tau<R>(J, p.c, cr, p.r, d, id, dr, xl, l, axis, by_sphere);
        if (tau > J.tau_peel_max) continue;
        if (by_sphere) {
            peel_tally(J, i, bin_of((double)xl, J.cam_xmin, J.cam_xmax, J.cam_nbins),
                       pixel_of(J, cam, p.r), p.id(), (double)W * ::exp(-tau));
            continue;
        }
        if (tc.slot == tc.end) {
            const uint32_t b = atomicAdd(&J.ctl->tn[sub * 16], (unsigned int)kTaskChunk);
            if (b + kTaskChunk > J.task_hw) atomicOr(stop_dev, 1u);
            if (b + kTaskChunk > J.task_sub_cap) {
                // no room: the slots of this reservation that exist stay empty
                for (uint32_t e = b; e < J.task_sub_cap; ++e)
                    J.task.cam[(uint32_t)sub * J.task_sub_cap + e] = -1;
                atomicAdd(&J.ctl->overflow, 1u);
                continue;
            }
            tc.slot = (uint32_t)sub * J.task_sub_cap + b;
            tc.end = tc.slot + kTaskChunk;
        }
        const uint32_t t = tc.slot++;
        const TaskSoA &T = J.task;
        T.rx[t] = p.r[0];
        T.ry[t] = p.r[1];
        T.rz[t] = p.r[2];
        T.lox[t] = (float)p.c.lo[0];
        T.loy[t] = (float)p.c.lo[1];
        T.loz[t] = (float)p.c.lo[2];
        T.size[t] = (float)p.c.size;
        T.cell[t] = p.c.cell;
        T.cam[t] = i;
        reinterpret_cast<R *>(T.xl)[t] = xl;
        reinterpret_cast<R *>(T.W)[t] = W;
        T.id[t] = p.id();
    }
}

// Emission (Sec. 3.1.1): source position, isotropic direction, frequency,
// first optical depth; draw order [source][blob offset] mu phi [x_nat, atom
// velocity] tau.  cr receives the line data of the birth cell.
// A lane's state for next-event estimates in camera kernels.  An event
// (emission, dust or H I scattering) leaves its source and the photon's
// incoming direction here; the estimate itself is made once per pass, at one
// place in the wave loop, so its code is inlined only once.
template <typename R>
struct PeelCtx {
    const double *cams;       // the job's camera table (an LDS copy in one-job launches)
    TaskCursor tc;
    int sub;                  // the lane's task sub-buffer
    unsigned int *stop_dev;
    bool pend;                // an event waits for its estimate
    PeelSource<R> ps;
    R kin[3];
};

template <typename R, bool CAMS>
__device__ __forceinline__ void emit(const JobView &J, Photon<R> &p, uint64_t id,
                                     CellRec<R> &cr, PeelCtx<R> &pc, LaneCounters &lc)
{
    using F = Fn<R>;
    p.events = 0;
    p.nscat = 0;
    p.status = 0;
    p.rng.init(J.seed, id);
    int src = 0;
    if (J.n_src > 1) {
        const double Rs = (double)p.rng.next();
        while (src < J.n_src - 1 && Rs > J.src_cdf[src]) ++src;
    }
    p.r[0] = J.src_pos[3 * src];
    p.r[1] = J.src_pos[3 * src + 1];
    p.r[2] = J.src_pos[3 * src + 2];
    if (J.src_kind == 1) {
        const R R1 = p.rng.next(), R2 = p.rng.next(), R3 = p.rng.next(), R4 = p.rng.next();
        const R q1 = F::sqrt(R(-2) * F::log(R1)), q2 = F::sqrt(R(-2) * F::log(R3));
        R c2, s2, c4, s4;
        F::cossin2pi(R2, c2, s2);
        F::cossin2pi(R4, c4, s4);
        p.r[0] += J.sigma * (double)(q1 * c2);
        p.r[1] += J.sigma * (double)(q1 * s2);
        p.r[2] += J.sigma * (double)(q2 * c4);
    }
    isotropic_dir(p);
    lc.add(C_EMITTED);
    p.x = R(0);
    double k[3], ik[3];
    geom_dir(p, k, ik);
    if (!locate(J.g, p.r, k, p.c)) {           // born outside the domain
        p.status = 1;
        return;
    }
    cr = load_cell<R>(J.g, p.c.cell);
    R x = R(0);
    R ua[3] = {R(0), R(0), R(0)};
    R xnat = R(0);
    if (J.freq_mode == 1) {                    // eq. init_freq
        const R Rl = p.rng.next();
        if constexpr (sizeof(R) == 8) {
            xnat = cr.a * ::tan(kPi * (Rl - 0.5));
        } else {
            float c, s;
            F::cossin2pi(0.5f * Rl, c, s);
            xnat = -cr.a * F::div(c, s);
        }
        const R R1 = p.rng.next(), R2 = p.rng.next(), R3 = p.rng.next(), R4 = p.rng.next();
        const R q1 = F::sqrt(-F::log(R1)), q2 = F::sqrt(-F::log(R3));
        R c2, s2, c4, s4;
        F::cossin2pi(R2, c2, s2);
        F::cossin2pi(R4, c4, s4);
        ua[0] = q1 * c2;
        ua[1] = q1 * s2;
        ua[2] = q2 * c4;
        x = xnat + (p.kr[0] * ua[0] + p.kr[1] * ua[1] + p.kr[2] * ua[2]);
    }
    p.x = F::div(x + (p.kr[0] * cr.ux + p.kr[1] * cr.uy + p.kr[2] * cr.uz), cr.s);
    if constexpr (CAMS) {
        if (J.n_cams > 0) {
            pc.ps = {xnat, R(0), R(0), {ua[0], ua[1], ua[2]}};
            pc.pend = true;
        }
    }
    p.tau = -(double)F::log(p.rng.next());
}

// One step of the ray tracing (Sec. 3.1.2) in the photon's current cell,
// whose line data the caller holds in cr.  Returns kCrossed after moving the
// photon into the next cell (cr then holds that cell's data), kEvent with the
// photon at its interaction point (comoving frequency in xloc, total opacity
// in ktot), or kGone once it has left the domain or reached the event cap.
enum { kCrossed = 0, kEvent = 1, kGone = 2 };

template <typename R>
__device__ __forceinline__ int march_step(const JobView &J, Photon<R> &p, CellRec<R> &cr,
                                          R &xloc, double &ktot, LaneCounters &lc)
{
    int axis;
    bool by_sphere;
    double k[3], ik[3];
    geom_dir(p, k, ik);
    const double l_exit = exit_distance(J.g, p.c, p.r, k, ik, axis, by_sphere);
    xloc = p.x * cr.s - (p.kr[0] * cr.ux + p.kr[1] * cr.uy + p.kr[2] * cr.uz);
    const R kHI = cr.k0 * voigt_H<R>(cr.a, xloc);
    ktot = (double)(kHI + cr.kd);
    const double tau_cell = ktot * l_exit;
    if (p.tau > tau_cell) {
        p.tau -= tau_cell;
#pragma unroll
        for (int d = 0; d < 3; ++d) p.r[d] += l_exit * k[d];
        lc.add(C_CROSSINGS);
        if (++p.events >= J.max_events) { p.status = 3; return kGone; }
        if (by_sphere || !cross(J.g, p.c, p.r, k, axis)) { p.status = 1; return kGone; }
        cr = load_cell<R>(J.g, p.c.cell);
        return kCrossed;
    }
    // FP32: ktot holds single-precision opacities, so its reciprocal in
    // single precision loses nothing a double division would keep
    const double l = (sizeof(R) == 4) ? p.tau * (double)__builtin_amdgcn_rcpf((float)ktot)
                                      : p.tau / ktot;
#pragma unroll
    for (int d = 0; d < 3; ++d) p.r[d] += l * k[d];
    if (++p.events >= J.max_events || !(p.r[0] == p.r[0])) { p.status = 3; return kGone; }
    return kEvent;
}

// Interaction channel: grey dust with probability k_dust / k_tot (absorbed
// unless a second draw falls below the albedo, else isotropic scattering with
// the comoving frequency kept); otherwise an H I scattering (returns true).
template <typename R, bool CAMS>
__device__ __forceinline__ bool interact(const JobView &J, Photon<R> &p, const CellRec<R> &cr,
                                         R xloc, double ktot, PeelCtx<R> &pc, LaneCounters &lc)
{
    using F = Fn<R>;
    if (cr.kd > R(0) && p.rng.next() < F::div(cr.kd, (R)ktot)) {
        if (p.rng.next() >= (R)J.g.albedo) { p.status = 2; return false; }
        isotropic_dir(p);
        p.x = F::div(xloc + (p.kr[0] * cr.ux + p.kr[1] * cr.uy + p.kr[2] * cr.uz), cr.s);
        lc.add(C_SCAT_DUST);
        if constexpr (CAMS) {
            if (J.n_cams > 0) {
                pc.ps = {xloc, R(0), R(0), {R(0), R(0), R(0)}};
                pc.pend = true;
            }
        }
        p.tau = -(double)F::log(p.rng.next());
        return false;
    }
    return true;
}

// H I scattering after the parallel velocity is known (Sec. 3.1.3, 3.2.4):
// perpendicular velocity (truncated below x_crit when core-skipping applies),
// new direction from the phase function, redistributed frequency (eq. x_f),
// next-event tallies and the next optical depth.
template <typename R, bool CAMS>
__device__ __forceinline__ void scatter_finish(const JobView &J, Photon<R> &p,
                                               const CellRec<R> &cr, R xloc, R upar,
                                               PeelCtx<R> &pc, LaneCounters &lc)
{
    using F = Fn<R>;
    const R a = cr.a, xcw = cr.xcw;
    R xc = R(0);
    if (J.xcrit_mode == 1) {
        xc = (sizeof(R) == 4) ? (R)J.xcrit_global_f : (R)J.xcrit_global;
    } else if (J.xcrit_mode == 2) {
        const CellAux<R> ax = load_aux<R>(J.g, p.c.cell);
        const R atau = a * cr.k0 * (R)min_face_distance(p.c, p.r) + ax.atau_nl;
        xc = xcrit_of<R>(atau);
    } else if (J.xcrit_mode == 3) {
        xc = xcrit_of<R>(load_aux<R>(J.g, p.c.cell).atau_j);
    }
    const R axl = (xloc < R(0)) ? -xloc : xloc;
    if (axl >= xcw) xc = R(0);                 // already in the wing: no cut-off
    // the scattering's draws in stream order: u_perp (2), mu, phi, next tau;
    // FP32 takes all five at once (its two generator blocks overlap)
    R dw[5] = {R(0), R(0), R(0), R(0), R(0)};
    R u1, u2;
    if constexpr (sizeof(R) == 4) {
        p.rng.next5(dw);
        draw_uperp_from<R>(xc, dw[0], dw[1], u1, u2);
    } else {
        draw_uperp<R>(xc, p.rng, u1, u2);
    }
    R e1[3], e2[3];
    perp_basis<R>(p.kr, e1, e2);
    R ua[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) ua[d] = upar * p.kr[d] + u1 * e1[d] + u2 * e2[d];
    const R rW = J.isotropic ? R(0) : ((axl < xcw) ? R(3.0 / 11.0) : R(1));
    R mu, cph, sph;
    if constexpr (sizeof(R) == 4) {
        mu = draw_mu_from<R>(rW, dw[2]);
        F::cossin2pi(dw[3], cph, sph);
    } else {
        mu = draw_mu<R>(rW, p.rng);
        F::cossin2pi(p.rng.next(), cph, sph);
    }
    const R st = F::sqrt(R(1) - mu * mu);
    R kf[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) kf[d] = mu * p.kr[d] + st * (cph * e1[d] + sph * e2[d]);
    const R nk2 = kf[0] * kf[0] + kf[1] * kf[1] + kf[2] * kf[2];
    if constexpr (sizeof(R) == 4) {
        const R inv = F::rsqrt(nk2);
#pragma unroll
        for (int d = 0; d < 3; ++d) kf[d] *= inv;
    } else {
        const R nk = F::sqrt(nk2);
#pragma unroll
        for (int d = 0; d < 3; ++d) kf[d] = F::div(kf[d], nk);
    }
    R grec = R(0);
    if (J.recoil) grec = load_aux<R>(J.g, p.c.cell).g;
    const R xf = xloc - upar + (kf[0] * ua[0] + kf[1] * ua[1] + kf[2] * ua[2]) +
                 grec * (mu - R(1));              // eq. x_f
    ++p.nscat;
    lc.add(C_SCAT_HI);
    if constexpr (CAMS) {
        if (J.n_cams > 0) {
            pc.ps = {xloc - upar, grec, rW, {ua[0], ua[1], ua[2]}};
            pc.kin[0] = p.kr[0];
            pc.kin[1] = p.kr[1];
            pc.kin[2] = p.kr[2];
            pc.pend = true;
        }
    }
    set_dir(p, kf[0], kf[1], kf[2]);
    p.x = F::div(xf + (kf[0] * cr.ux + kf[1] * cr.uy + kf[2] * cr.uz), cr.s);
    p.tau = -(double)F::log((sizeof(R) == 4) ? dw[4] : p.rng.next());
}

template <typename R>
__device__ __forceinline__ void finish(const JobView &J, const Photon<R> &p, LaneCounters &lc)
{
    if (p.status == 1) {
        lc.add(C_ESCAPED);
        if (J.n_bins > 0) {
            const int b = bin_of((double)p.x, J.x_min, J.x_max, J.n_bins);
            atomicAdd(J.spectrum + b, 1ull);
        }
    } else if (p.status == 2) {
        lc.add(C_ABSORBED);
    } else {
        lc.add(C_CAPPED);
    }
    if (J.record) {
        const uint64_t id = p.id();
        J.rec_x[id] = (double)p.x;
        J.rec_nscat[id] = p.nscat;
        J.rec_status[id] = p.status;
#pragma unroll
        for (int d = 0; d < 3; ++d)        // one rounding in every kernel variant
            J.rec_pos[3 * id + d] = ::fma(p.r[d], J.dx_cm, J.box_min_cm[d]);
    }
}

// ---------------------------------------------------------------------------
// Cooperative u_par sampling.  The lanes of a wave that need a parallel atom
// velocity (two-part or core proposal) post their requests in LDS; in each
// round every lane of the wave evaluates one unit of candidates: lane L works
// for the (L mod m)-th open request (m open requests), on its unit number
// base + L / m.  A unit is one candidate in FP64 and the two candidates that
// share a generator block in FP32.  The smallest accepted candidate number of
// a request is its sequential result, so the outcome equals the one-lane loop
// exactly while all 64 lanes stay busy until the last request of the wave is
// served.
// ---------------------------------------------------------------------------
// A request in LDS.  KU: the generator key is the same for every lane (one
// job), so the slot need not hold it.
template <typename R, bool KU>
struct UparSlot;

template <bool KU>
struct UparSlot<double, KU> {
    double X, a, u0, p, th0;
    int32_t regime;
    uint32_t key0, key1, id0, id1, b0lo, b0hi;
    uint32_t base;
    __device__ __forceinline__ void put(const UparReq<double> &q, const RngKey &k)
    {
        X = q.X; a = q.a; u0 = q.u0; p = q.p; th0 = q.th0; regime = q.regime;
        key0 = k.key0; key1 = k.key1; id0 = k.id0; id1 = k.id1;
    }
    __device__ __forceinline__ UparReq<double> req() const
    {
        UparReq<double> q;
        q.X = X; q.a = a; q.u0 = u0; q.p = p; q.th0 = th0; q.regime = regime;
        q.wp = 0u; q.inv_lo = 0.0f; q.inv_hi = 0.0f;
        return q;
    }
    __device__ __forceinline__ RngKey key(const RngKey &uniform) const
    {
        RngKey k;
        k.key0 = KU ? uniform.key0 : key0;
        k.key1 = KU ? uniform.key1 : key1;
        k.id0 = id0; k.id1 = id1;
        return k;
    }
};

// FP32 candidates need no regime and no p: the word split point and the
// reciprocal part widths stand in for them.  Twelve words per request; with
// a per-lane key the reciprocals give way to the key and are recomputed.
template <>
struct UparSlot<float, true> {
    float X, a, u0, th0, inv_lo, inv_hi;
    uint32_t wp, id0, id1, b0lo, b0hi;
    uint32_t base;
    __device__ __forceinline__ void put(const UparReq<float> &q, const RngKey &k)
    {
        X = q.X; a = q.a; u0 = q.u0; th0 = q.th0; inv_lo = q.inv_lo; inv_hi = q.inv_hi;
        wp = q.wp; id0 = k.id0; id1 = k.id1;
    }
    __device__ __forceinline__ UparReq<float> req() const
    {
        UparReq<float> q;
        q.X = X; q.a = a; q.u0 = u0; q.p = 0.0f; q.th0 = th0; q.regime = UPAR_SPLIT;
        q.wp = wp; q.inv_lo = inv_lo; q.inv_hi = inv_hi;
        return q;
    }
    __device__ __forceinline__ RngKey key(const RngKey &uniform) const
    {
        RngKey k;
        k.key0 = uniform.key0; k.key1 = uniform.key1; k.id0 = id0; k.id1 = id1;
        return k;
    }
};

template <>
struct UparSlot<float, false> {
    float X, a, u0, th0;
    uint32_t wp, key0, key1, id0, id1, b0lo, b0hi;
    uint32_t base;
    __device__ __forceinline__ void put(const UparReq<float> &q, const RngKey &k)
    {
        X = q.X; a = q.a; u0 = q.u0; th0 = q.th0; wp = q.wp;
        key0 = k.key0; key1 = k.key1; id0 = k.id0; id1 = k.id1;
    }
    __device__ __forceinline__ UparReq<float> req() const
    {
        UparReq<float> q;
        q.X = X; q.a = a; q.u0 = u0; q.p = 0.0f; q.th0 = th0; q.regime = UPAR_SPLIT;
        q.wp = wp;
        q.inv_lo = __builtin_amdgcn_rcpf((float)wp);
        q.inv_hi = __builtin_amdgcn_rcpf((float)(0u - wp));
        return q;
    }
    __device__ __forceinline__ RngKey key(const RngKey &) const
    {
        RngKey k;
        k.key0 = key0; k.key1 = key1; k.id0 = id0; k.id1 = id1;
        return k;
    }
};

__device__ __forceinline__ void wave_lds_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

constexpr uint32_t kMaxUparRounds = 1u << 22;   // bound on rounds; never reached in practice

// n / m for 0 <= n < 256 and 1 <= m <= 64 through the reciprocal of m:
// (n + 1/2) / m stays at least 1/(2m) from an integer, far more than the
// rounding of the product, so the truncation is exact.
__device__ __forceinline__ uint32_t small_div(uint32_t n, float inv_m)
{
    return (uint32_t)(((float)n + 0.5f) * inv_m);
}

// All 64 lanes of the wave must call this together.  On return, lanes with
// `need` hold the unsigned |u_par| in u and the accepted candidate number in t
// (ok = false only if the round bound was hit).  KEY_UNIFORM: every lane's
// generator key (the job seed) is the same wave-uniform value.
template <typename R, bool KEY_UNIFORM>
__device__ __forceinline__ uint32_t coop_upar(bool need, const UparReq<R> &q, const RngKey &key,
                                              uint64_t B0, R &u, uint32_t &t, bool &ok,
                                              UparSlot<R, KEY_UNIFORM> *slots, int32_t *table,
                                              uint32_t *first)
{
    const int lane = threadIdx.x & 63;
    ok = true;
    uint32_t base = 0;
    uint32_t rounds = 0;
    if (need) {
        UparSlot<R, KEY_UNIFORM> s;
        s.put(q, key);
        s.b0lo = (uint32_t)B0; s.b0hi = (uint32_t)(B0 >> 32);
        s.base = 0;
        slots[lane] = s;
    }
    for (uint32_t round = 0;; ++round) {
        const uint64_t S = __ballot(need);
        if (S == 0) break;
        ++rounds;
        const int m = __popcll(S);
        const float inv_m = __builtin_amdgcn_rcpf((float)m);
        const int rank = __popcll(S & ((lane == 0) ? 0ull : (~0ull >> (64 - lane))));
        if (need) {
            table[rank] = lane;
            first[rank] = 64u;
        }
        wave_lds_sync();
        const uint32_t ss = small_div((uint32_t)lane, inv_m);
        const int rr = lane - (int)ss * m;
        const UparSlot<R, KEY_UNIFORM> s = slots[table[rr]];
        const UparReq<R> qq = s.req();
        const RngKey kk = s.key(key);
        const uint64_t b0 = ((uint64_t)s.b0hi << 32) | s.b0lo;
        R uc;
        uint32_t half = 0;
        bool acc;
        if constexpr (sizeof(R) == 8)
            acc = upar_candidate<R>(qq, kk, b0, s.base + ss, uc);
        else
            acc = upar_pair_fp32(qq, kk, b0, s.base + ss, uc, half);
        if (acc) atomicMin(&first[rr], (uint32_t)lane);
        wave_lds_sync();
        uint32_t f = 64u;
        if (need) f = first[rank];
        const int src = (need && f < 64u) ? (int)f : lane;
        R got;
        uint32_t got_half = 0;
        if constexpr (sizeof(R) == 8) {
            const uint64_t bits = __double_as_longlong(uc);
            const uint32_t lo = __shfl((uint32_t)bits, src), hi = __shfl((uint32_t)(bits >> 32), src);
            got = __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
        } else {
            got = __shfl(uc, src);
            got_half = __shfl(half, src);
        }
        if (need) {
            if (f < 64u) {
                u = got;
                const uint32_t unit = base + small_div(f, inv_m);
                t = (sizeof(R) == 8) ? unit : 2u * unit + got_half;
                need = false;
            } else {
                base += small_div((uint32_t)(64 - rank + m - 1), inv_m);
                slots[lane].base = base;
                if (round >= kMaxUparRounds) { need = false; ok = false; u = R(0); t = base; }
            }
        }
        wave_lds_sync();
    }
    return rounds;
}

__device__ __forceinline__ int find_job(const LaunchView &L, uint64_t g)
{
    int lo = 0, hi = L.n_jobs - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (L.prefix[mid] <= g) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}
__device__ __forceinline__ int find_rjob(const LaunchView &L, uint32_t r)
{
    int lo = 0, hi = L.n_jobs - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (L.rprefix[mid] <= r) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// ---------------------------------------------------------------------------
// Preemption.  At the end of a pass every live photon is in flight with its
// optical depth to go, so its whole state fits a SuspRec; a stopped launch
// writes its photons to the job's other suspend array, and the next launch
// resumes them (before new photons) with bit-identical continuations.
// ---------------------------------------------------------------------------
template <typename R>
__device__ __forceinline__ void suspend(const JobView &J, const Photon<R> &p)
{
    const unsigned int cur = J.ctl->cur;
    const unsigned int i = atomicAdd(&J.ctl->n_out, 1u);
    if (i >= J.susp_cap) {
        atomicAdd(&J.ctl->overflow, 1u);
        return;
    }
    SuspRec *s = (cur ? J.susp[0] : J.susp[1]) + i;   // the array not being resumed from
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        s->r[d] = p.r[d];
        s->lo[d] = p.c.lo[d];
        s->k[d] = (double)p.kr[d];
    }
    s->tau = p.tau;
    s->size = p.c.size;
    s->x = (double)p.x;
    s->events = p.events;
    s->id = p.id();
    s->rng_k = p.rng.k;
    s->cell = p.c.cell;
    s->nscat = p.nscat;
}

template <typename R>
__device__ __forceinline__ void resume(const JobView &J, Photon<R> &p, uint32_t i,
                                       CellRec<R> &cr)
{
    const SuspRec *s = (J.ctl->cur ? J.susp[1] : J.susp[0]) + i;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        p.r[d] = s->r[d];
        p.c.lo[d] = s->lo[d];
    }
    p.c.size = s->size;
    p.c.cell = s->cell;
    set_dir(p, (R)s->k[0], (R)s->k[1], (R)s->k[2]);
    p.x = (R)s->x;
    p.tau = s->tau;
    p.events = s->events;
    p.nscat = s->nscat;
    p.status = 0;
    p.rng.init(J.seed, s->id);
    p.rng.restore(s->rng_k);
    cr = load_cell<R>(J.g, p.c.cell);
}

// A stopped launch hands the resumes no lane has taken to the next launch.
__device__ __forceinline__ void carry_over(const JobView &J, uint32_t i)
{
    const unsigned int cur = J.ctl->cur;
    const unsigned int o = atomicAdd(&J.ctl->n_out, 1u);
    if (o >= J.susp_cap) {
        atomicAdd(&J.ctl->overflow, 1u);
        return;
    }
    const SuspRec *in = cur ? J.susp[1] : J.susp[0];
    SuspRec *out = cur ? J.susp[0] : J.susp[1];
    out[o] = in[i];
}

// Host stop words are read every kHostPoll passes (each read crosses PCIe).
constexpr uint32_t kHostPoll = 32;

// Persistent photon pool.  Each pass of the wave loop: idle lanes take
// suspended photons to resume, then new photons, from the launch's queues
// (one atomic per wave for each); the photons in flight take ray-tracing
// steps, the wave stepping on while at least L.march_min of its lanes are
// still in flight (the rest resume in the next pass, so one long flight does
// not hold the whole wave); the wave then serves all parallel-velocity draws
// cooperatively and completes the scatterings.  At the end of a pass the wave
// checks for a stop request (or, under the tail rule, whether it holds fewer
// than L.tail_live photons once both queues are empty); a stopped wave
// suspends its photons and leaves.
// A photon's history does not depend on where passes cut its flights or on
// where the launch was stopped.
// SINGLE launches carry one job.  The FP32 kernels take it by value as J1:
// its parameters are then kernel arguments, read through the scalar cache
// (the job table in global memory is re-read with vector loads on every use).
// The FP64 kernels, whose vector registers are full, keep reading the table:
// scalar copies of the parameters push part of their photon state to scratch.
// Resident workgroups of 256 lanes per CU the register allocation aims for.
template <typename R, bool CAMS>
constexpr int transport_min_blocks()
{
    return CAMS ? ((sizeof(R) == 4) ? COLT_FP32_CAM_MIN_BLOCKS : 1)
                : ((sizeof(R) == 4) ? COLT_FP32_MIN_BLOCKS : COLT_FP64_MIN_BLOCKS);
}

template <typename R, bool CAMS, bool SINGLE, int GK>
__global__ __launch_bounds__(256, (transport_min_blocks<R, CAMS>())) void k_transport(LaunchView L, JobView J1)
{
    __shared__ UparSlot<R, SINGLE> s_slots[4][64];
    __shared__ int32_t s_table[4][64];
    __shared__ uint32_t s_first[4][64];
    __shared__ unsigned long long s_counts[kLaneCounters][kMaxBlock];
    __shared__ double s_cam[(CAMS && SINGLE) ? 12 * kMaxCams : 1];
    const int wave = threadIdx.x >> 6;
    const int lane = threadIdx.x & 63;
    const uint64_t lane_lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    const int slot = (int)((blockIdx.x * (blockDim.x >> 6) + wave) & (kCounterSlots - 1));
    PeelCtx<R> pc;
    pc.pend = false;
    pc.cams = nullptr;
    pc.tc.slot = pc.tc.end = 0;
    pc.sub = (int)((blockIdx.x * blockDim.x + threadIdx.x) & (kTaskSubs - 1));
    pc.stop_dev = L.stop_dev;
    if constexpr (CAMS && SINGLE) {
        // the job's camera table, read at every next-event estimate, kept in LDS
        for (int i = threadIdx.x; i < 12 * J1.n_cams; i += blockDim.x) s_cam[i] = J1.cam[i];
        pc.cams = s_cam;
        __syncthreads();
    }
    Photon<R> p;
    p.status = 0;
    CellRec<R> cr;                 // line data of the photon's cell while it lives
    LaneCounters lc;
    lc.col = &s_counts[0][threadIdx.x];
#pragma unroll
    for (int i = 0; i < kLaneCounters; ++i) s_counts[i][threadIdx.x] = 0ull;
    // GK fixes the grid kind of a one-job FP32 launch at compile time, so a
    // Cartesian launch carries no octree code (0 Cartesian, 1 octree, -1 any)
    JobView Jk = J1;
    if constexpr (GK == 0) {
        Jk.g.kind = 0;
        Jk.g.rope = nullptr;
        Jk.g.rec_stride = 1;
    } else if constexpr (GK == 1) {
        Jk.g.kind = 1;
        Jk.g.rec_stride = (sizeof(R) == 4) ? 2 : 1;
        Jk.g.rope_stride = (sizeof(R) == 4) ? 16 : 6;
    }
    const JobView *const J_single = (sizeof(R) == 4) ? &Jk : L.jobs;
    const JobView *J = SINGLE ? J_single : nullptr;
    const uint64_t total = L.prefix[L.n_jobs];
    const uint32_t rtotal = L.rprefix[L.n_jobs];
    const int march_min = L.march_min;
    bool res_left = rtotal > 0, new_left = total > 0;
    bool have = false, moving = false, stopping = false;   // stopping: a stop was seen
    // the tail rule: with every photon handed out, a wave holding fewer than
    // tail_live photons suspends them for a later launch (not in a launch
    // that started small, which therefore always runs to the end)
    const int tail_live = (total + rtotal >= kTailMinWork) ? L.tail_live : 0;
    uint32_t pass = 0;
    for (;;) {
        // a stop request set before or during this pass is acted on at its end;
        // only camera launches can set the device word (a task buffer near full)
        int stop_word = 0;
        if (lane == 0) {
            if constexpr (CAMS)
                stop_word = (int)__hip_atomic_load(L.stop_dev, __ATOMIC_RELAXED,
                                                   __HIP_MEMORY_SCOPE_AGENT);
            if (L.stop_host && (pass % kHostPoll) == 0)
                stop_word |= __hip_atomic_load(L.stop_host, __ATOMIC_RELAXED,
                                               __HIP_MEMORY_SCOPE_SYSTEM);
        }
        if (res_left || new_left) {
            const uint64_t need = __ballot(!have);
            if (need) {
                const int n_need = __popcll(need);
                const int leader = __ffsll((unsigned long long)need) - 1;
                const int rank = __popcll(need & lane_lt);
                int n_res = 0;
                uint32_t rbase = 0;
                if (res_left) {
                    uint32_t b = 0;
                    if (lane == leader) b = (uint32_t)atomicAdd(L.rqueue, (unsigned long long)n_need);
                    b = __shfl(b, leader);
                    if (b < rtotal) n_res = (rtotal - b < (uint32_t)n_need) ? (int)(rtotal - b) : n_need;
                    if (b + (uint32_t)n_need >= rtotal) res_left = false;
                    rbase = b;
                }
                unsigned long long qbase = 0;
                const int n_new = n_need - n_res;
                bool take_new = false;
                if (n_new > 0 && new_left) {
                    if (lane == leader) qbase = atomicAdd(L.queue, (unsigned long long)n_new);
                    const uint32_t blo = __shfl((uint32_t)qbase, leader);
                    const uint32_t bhi = __shfl((uint32_t)(qbase >> 32), leader);
                    qbase = ((unsigned long long)bhi << 32) | blo;
                    if (qbase + n_new >= total) new_left = false;
                    take_new = true;
                }
                if (!have) {
                    int j = -1;
                    uint64_t id = 0;
                    uint32_t ri = 0;
                    const bool res = rank < n_res;
                    if (res) {
                        ri = rbase + (uint32_t)rank;
                        j = SINGLE ? 0 : find_rjob(L, ri);
                    } else if (take_new) {
                        const uint64_t g = qbase + (uint64_t)(rank - n_res);
                        if (g < total) {
                            j = SINGLE ? 0 : find_job(L, g);
                            id = L.first_id[j] + (g - L.prefix[j]);
                        }
                    }
                    if (j >= 0) {
                        if constexpr (!SINGLE) {
                            const JobView *Jn = &L.jobs[j];
                            if (Jn != J) {
                                if (J) {
                                    flush_counters(J, lc, slot);
                                    if constexpr (CAMS) close_tasks(*J, pc.tc);
                                }
                                J = Jn;
                                pc.cams = J->cam;
                            }
                        }
                        have = true;
                        moving = true;
                        if (res) {
                            resume<R>(*J, p, ri - L.rprefix[j], cr);
                        } else {
                            emit<R, CAMS>(*J, p, id, cr, pc, lc);
                            if (p.status != 0) {
                                finish<R>(*J, p, lc);
                                have = false;
                                moving = false;
                            } else if (CAMS && pc.pend) {
                                // the emission's estimate is made this pass,
                                // from the birth point; the flight starts next
                                moving = false;
                                pc.kin[0] = p.kr[0];
                                pc.kin[1] = p.kr[1];
                                pc.kin[2] = p.kr[2];
                            }
                        }
                    }
                }
            }
        }
        const bool any_have = __any(have);
        if (any_have) {
            if constexpr (SINGLE) {
                // one job: its seed, the generator key, is wave-uniform
                p.rng.key.key0 = (uint32_t)J->seed;
                p.rng.key.key1 = (uint32_t)(J->seed >> 32);
            }
            bool event = false;
            R xloc = R(0);
            double ktot = 0.0;
            // with few photons left in the wave a pass need not wait for many
            // flights: the threshold shrinks with the number of live lanes
            const int live = __popcll(__ballot(have));
            const int quarter = (live + 3) >> 2;
            const int stop_below = (march_min < quarter) ? march_min : quarter;
            for (;;) {
                if (moving) {
                    const int st = march_step<R>(*J, p, cr, xloc, ktot, lc);
                    if (st != kCrossed) {
                        moving = false;
                        event = st == kEvent;
                    }
                }
                const int in_flight = __popcll(__ballot(moving));
                if (in_flight == 0 || in_flight < stop_below) break;
            }
            bool hi = false;
            UparReq<R> q;
            q.regime = UPAR_GAUSS;
            uint64_t B0 = 0;
            if (event) {
                if (interact<R, CAMS>(*J, p, cr, xloc, ktot, pc, lc)) {
                    hi = true;
                    q = upar_setup<R>(cr.a, xloc, cr.xcw);
                    B0 = p.rng.align();
                } else if (p.status == 0) {
                    moving = true;                    // dust scattering: a new flight
                }
            }
            R u = R(0);
            uint32_t tacc = 0;
            bool ok = true;
            const uint32_t rounds = coop_upar<R, SINGLE>(hi && q.regime != UPAR_GAUSS, q, p.rng.key, B0, u,
                                                 tacc, ok, s_slots[wave], s_table[wave],
                                                 s_first[wave]);
            if (lane == 0 && J) {
                lc.add(C_ROUNDS, rounds);
                lc.add(C_PASSES);
            }
            if (hi) {
                if (q.regime == UPAR_GAUSS) {
                    u = upar_gauss<R>(q, p.rng.key, B0);
                    p.rng.k += Rng<R>::kPerBlock;
                } else {
                    lc.add(C_UPAR_TRIES, tacc + 1);
                    p.rng.k += upar_advance<R>(q.regime, tacc);
                    if (!ok) p.status = 3;
                }
                if (p.status == 0) {
                    scatter_finish<R, CAMS>(*J, p, cr, xloc, (xloc < R(0)) ? -u : u, pc, lc);
                    moving = true;
                }
            }
            if constexpr (CAMS) {
                if (pc.pend) {
                    peel_event<R>(*J, pc.cams, p, cr, pc.ps, pc.kin, pc.tc, pc.sub, pc.stop_dev,
                                  lc);
                    pc.pend = false;
                    moving = true;
                }
            }
            if (have && p.status != 0) {
                finish<R>(*J, p, lc);
                have = false;
                moving = false;
            }
        }
        ++pass;
        if (__builtin_amdgcn_readfirstlane(stop_word) != 0) {   // lane 0: all lanes are active here
            stopping = true;
            break;
        }
        if (!any_have && !res_left && !new_left) break;
        if (tail_live > 0 && !res_left && !new_left && __popcll(__ballot(have)) < tail_live) {
            stopping = true;
            break;
        }
    }
    if (stopping) {
        // suspend the wave's photons (all in flight at the end of a pass) and
        // hand on the resumes no lane has taken
        if (have) suspend<R>(*J, p);
        while (res_left) {
            uint32_t b = 0;
            if (lane == 0) b = (uint32_t)atomicAdd(L.rqueue, 64ull);
            b = __shfl(b, 0);
            if (b + 64u >= rtotal) res_left = false;
            const uint32_t ri = b + (uint32_t)lane;
            if (ri < rtotal) {
                const int j = SINGLE ? 0 : find_rjob(L, ri);
                carry_over(SINGLE ? *J_single : L.jobs[j], ri - L.rprefix[j]);
            }
        }
    }
    if constexpr (CAMS) {
        if (J) close_tasks(*J, pc.tc);
    }
    if constexpr (SINGLE)
        flush_counters_wave(J, lc, slot);
    else if (J)
        flush_counters(J, lc, slot);
}

// ---------------------------------------------------------------------------
// Launch planning on the device, from the jobs' control blocks, so eager
// launches and graph replays work the same way and a stopped launch's state is
// picked up by the next one.  k_plan reserves each job's next slice of new
// photons (cursor += take, so launches of a job on several streams take
// disjoint slices) and lays out the resume and new-photon index ranges;
// k_advance gives back the part of a slice a stopped launch did not reach,
// swaps the suspend arrays and empties the march-task buffers.  One
// workgroup of 256 threads each, any number of jobs.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_plan(LaunchView L)
{
    __shared__ unsigned long long s_a[256];
    __shared__ unsigned int s_b[256];
    const int t = threadIdx.x;
    unsigned long long carry_a = 0;
    unsigned int carry_b = 0;
    for (int base = 0; base < L.n_jobs; base += 256) {
        const int j = base + t;
        unsigned long long a = 0;
        unsigned int b = 0;
        if (j < L.n_jobs) {
            // reserve [cursor, cursor + a) atomically: launches of one job on
            // different streams may plan at the same time
            JobCtl *c = L.jobs[j].ctl;
            const unsigned long long n = L.jobs[j].n_photons;
            unsigned long long cur = __hip_atomic_load(&c->cursor, __ATOMIC_RELAXED,
                                                       __HIP_MEMORY_SCOPE_AGENT);
            for (;;) {
                const unsigned long long left = n - cur;
                a = (L.quota && L.quota < left) ? L.quota : left;
                const unsigned long long seen = atomicCAS(&c->cursor, cur, cur + a);
                if (seen == cur) break;
                cur = seen;
            }
            b = c->n_in;
            L.first_id[j] = cur;
            c->n_out = 0;
        }
        s_a[t] = a;
        s_b[t] = b;
        __syncthreads();
        for (int o = 1; o < 256; o <<= 1) {          // inclusive scans
            const unsigned long long ya = (t >= o) ? s_a[t - o] : 0ull;
            const unsigned int yb = (t >= o) ? s_b[t - o] : 0u;
            __syncthreads();
            s_a[t] += ya;
            s_b[t] += yb;
            __syncthreads();
        }
        if (j < L.n_jobs) {
            L.prefix[j + 1] = carry_a + s_a[t];
            L.rprefix[j + 1] = carry_b + s_b[t];
        }
        carry_a += s_a[255];
        carry_b += s_b[255];
        __syncthreads();
    }
    if (t == 0) {
        L.prefix[0] = 0;
        L.rprefix[0] = 0;
        *L.queue = 0ull;
        *L.rqueue = 0ull;
        *L.stop_dev = 0u;
    }
    for (int j = t; j < L.n_jobs; j += 256) L.peel_work[j] = 0ull;
}

__global__ __launch_bounds__(256) void k_advance(LaunchView L)
{
    const unsigned long long n = L.prefix[L.n_jobs];
    const unsigned long long q = (*L.queue < n) ? *L.queue : n;
    for (int j = threadIdx.x; j < L.n_jobs; j += 256) {
        JobCtl *c = L.jobs[j].ctl;
        const unsigned long long lo = L.prefix[j], hi = L.prefix[j + 1];
        const unsigned long long used = (q <= lo) ? 0ull : ((q >= hi) ? hi - lo : q - lo);
        if (used < hi - lo) atomicAdd(&c->cursor, (unsigned long long)(used - (hi - lo)));
        if (c->n_in != 0u || c->n_out != 0u) {
            c->cur ^= 1u;
            // n_out counts suspension attempts; beyond the array they failed
            // (and were counted as overflow)
            c->n_in = (c->n_out < L.jobs[j].susp_cap) ? c->n_out : L.jobs[j].susp_cap;
            c->n_out = 0u;
        }
        if (L.jobs[j].task_sub_cap)
            for (int b = 0; b < kTaskSubs; ++b) c->tn[b * 16] = 0u;
    }
}

// ---------------------------------------------------------------------------
// Deferred next-event marches (Sec. 6.1): each task follows one camera's ray
// from an event to the domain edge, adding the optical depth of every cell
// (H I at the Doppler-shifted frequency of that cell, and dust), and tallies
// W exp(-tau) unless the cut-off is passed first.  A lean persistent kernel in
// which lanes step marches at every iteration: lanes whose marches end take
// the next tasks they hold as soon as a few of them wait, so that this set-up
// is shared by several lanes even where marches are long.  Next tasks are
// loaded ahead, once a quarter of the wave needs one (or a lane would idle),
// from a chunk of task slots the wave claims with one atomic; a chunk lies
// inside one sub-buffer, so a lane's slot is the chunk start plus its rank.
// The first step repeats the event cell that the transport kernel already
// found below the cut-off (it is not counted again).
// ---------------------------------------------------------------------------
constexpr uint32_t kPeelChunk = 256;     // task slots a wave claims at a time
constexpr int kPeelTake = 8;             // ended marches that start the next tasks

template <typename R, int GK>
__global__ __launch_bounds__(256, COLT_PEEL_MIN_BLOCKS) void k_peel(JobView J, unsigned long long *work)
{
    __shared__ double s_cam[12 * kMaxCams];
    // chunks before each sub-buffer's first, and its task count
    __shared__ uint32_t s_chunk[kTaskSubs + 1], s_n[kTaskSubs];
    for (int i = threadIdx.x; i < 12 * J.n_cams; i += blockDim.x) s_cam[i] = J.cam[i];
    if (threadIdx.x == 0) {
        uint32_t acc = 0;
        for (int b = 0; b < kTaskSubs; ++b) {
            const uint32_t nb = J.ctl->tn[b * 16];
            s_n[b] = (nb < J.task_sub_cap) ? nb : J.task_sub_cap;
            s_chunk[b] = acc;
            acc += (s_n[b] + kPeelChunk - 1) / kPeelChunk;
        }
        s_chunk[kTaskSubs] = acc;
    }
    __syncthreads();
    if constexpr (GK == 0) {
        J.g.kind = 0;
        J.g.rope = nullptr;
        J.g.rec_stride = 1;
    } else if constexpr (GK == 1) {
        J.g.kind = 1;
        J.g.rec_stride = (sizeof(R) == 4) ? 2 : 1;
        J.g.rope_stride = (sizeof(R) == 4) ? 16 : 6;
    }
    const int lane = threadIdx.x & 63;
    const uint64_t lane_lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    const uint32_t n_chunks = s_chunk[kTaskSubs];
    const BinPixScale q = {J.cam_xmin, (double)J.cam_nbins / (J.cam_xmax - J.cam_xmin),
                           (J.npix > 0) ? 1.0 / J.fov : 0.0};
    // the wave's claimed task slots [wlo, whi) (wave-uniform)
    uint32_t wlo = 0, whi = 0;
    bool drained = n_chunks == 0;
    // the march being stepped
    bool have = false, first = false;
    CellBox c;
    double r[3] = {0.0, 0.0, 0.0}, tau = 0.0;
    R xl = R(0), W = R(0);
    int cam = 0, bin = 0, pix = -1;
    unsigned long long id = 0, steps = 0;
    // the next task, loaded ahead
    bool nv = false;
    double nr[3] = {0.0, 0.0, 0.0};
    float nlo[3] = {0.0f, 0.0f, 0.0f}, nsize = 0.0f;
    int32_t ncell = 0, ncam = -1;
    R nxl = R(0), nW = R(0);
    unsigned long long nid = 0;
    for (;;) {
        // lanes whose marches have ended take the tasks they hold, once
        // kPeelTake of them wait (or the wave has no march left)
        const uint64_t ready = __ballot(!have && nv);
        if (ready && (__popcll(ready) >= kPeelTake || !__any(have)) && !have && nv) {
            r[0] = nr[0];
            r[1] = nr[1];
            r[2] = nr[2];
            c.lo[0] = (double)nlo[0];
            c.lo[1] = (double)nlo[1];
            c.lo[2] = (double)nlo[2];
            c.size = (double)nsize;
            c.cell = ncell;
            cam = ncam;
            xl = nxl;
            W = nW;
            id = nid;
            bin = bin_scaled((double)xl, q, J.cam_nbins);
            pix = pixel_scaled(J, q, s_cam + 12 * cam, r);
            tau = 0.0;
            first = true;
            have = true;
            nv = false;
        }
        // lanes without a next task load one from the wave's chunk
        if (!drained) {
            const uint64_t need = __ballot(!nv);
            if (__popcll(need) >= 16 || __ballot(!nv && !have)) {
                if (wlo >= whi) {
                    uint32_t k = 0;
                    if (lane == 0) k = (uint32_t)atomicAdd(work, 1ull);
                    k = __builtin_amdgcn_readfirstlane(k);
                    if (k >= n_chunks) {
                        drained = true;
                    } else {
                        int b = 0;
#pragma unroll
                        for (int h = kTaskSubs / 2; h > 0; h >>= 1)
                            if (s_chunk[b + h] <= k) b += h;
                        const uint32_t off = (k - s_chunk[b]) * kPeelChunk;
                        const uint32_t n = (s_n[b] - off < kPeelChunk) ? s_n[b] - off : kPeelChunk;
                        wlo = (uint32_t)b * J.task_sub_cap + off;
                        whi = wlo + n;
                    }
                }
                if (!drained) {
                    const uint32_t t = wlo + (uint32_t)__popcll(need & lane_lt);
                    if (!nv && t < whi) {
                        const TaskSoA &T = J.task;
                        ncam = T.cam[t];
                        nr[0] = T.rx[t];
                        nr[1] = T.ry[t];
                        nr[2] = T.rz[t];
                        nlo[0] = T.lox[t];
                        nlo[1] = T.loy[t];
                        nlo[2] = T.loz[t];
                        nsize = T.size[t];
                        ncell = T.cell[t];
                        nxl = reinterpret_cast<const R *>(T.xl)[t];
                        nW = reinterpret_cast<const R *>(T.W)[t];
                        nid = T.id[t];
                        // empty slots (cam = -1) are skipped
                        nv = ncam >= 0 && ncam < J.n_cams;
                    }
                    const uint32_t took = (uint32_t)__popcll(need);
                    wlo = (wlo + took < whi) ? wlo + took : whi;
                }
            }
        }
        if (!__any(have || nv)) {
            if (drained) break;
            continue;
        }
        if (have) {
            const double *cm = s_cam + 12 * cam;
            const double d[3] = {cm[0], cm[1], cm[2]};
            const double idv[3] = {cm[3], cm[4], cm[5]};
            const R dr[3] = {(R)cm[0], (R)cm[1], (R)cm[2]};
            const CellRec<R> cr = load_cell<R>(J.g, c.cell);
            double l;
            int axis;
            bool by_sphere;
            tau += peel_cell_tau<R>(J, c, cr, r, d, idv, dr, xl, l, axis, by_sphere);
            if (!first) ++steps;
            first = false;
            int st = 0;
            if (tau > J.tau_peel_max) {
                st = 2;
            } else if (by_sphere) {
                st = 1;
            } else {
#pragma unroll
                for (int e = 0; e < 3; ++e) r[e] += l * d[e];
                if (!cross(J.g, c, r, d, axis)) st = 1;
            }
            if (st) {
                have = false;
                if (st == 1) peel_tally(J, cam, bin, pix, id, (double)W * ::exp(-tau));
            }
        }
    }
    // crossings of the marches beyond the event cell, one atomic per wave
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) steps += __shfl_xor(steps, o);
    if (lane == 0 && steps) {
        const int slot = (int)((blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6)) &
                               (kCounterSlots - 1));
        atomicAdd(J.counters + (size_t)slot * kNumCounters + C_PEEL_CROSSINGS, steps);
    }
}

// ---------------------------------------------------------------------------
// Non-local a*tau (Sec. 3.2.4, eq. atauNL): per cell, six axis paths from the
// centres of its faces outward, summing a k0 l over the cells crossed while
// the density stays within f_NL of the starting cell's; the minimum of the six
// sums.  One thread per cell; paths end at the domain edge.
// ---------------------------------------------------------------------------
__global__ void k_nonlocal(GridView g, const double *__restrict__ n_HI,
                           const double *__restrict__ leaf_boxes, int64_t n, double f_nl,
                           CellAux<double> *__restrict__ ad, CellAux<float> *__restrict__ af)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double lo[3], size;
    if (g.kind == 0) {
        lo[0] = (double)(i % g.n[0]);
        lo[1] = (double)((i / g.n[0]) % g.n[1]);
        lo[2] = (double)(i / ((int64_t)g.n[0] * g.n[1]));
        size = 1.0;
    } else {
        lo[0] = leaf_boxes[4 * i];
        lo[1] = leaf_boxes[4 * i + 1];
        lo[2] = leaf_boxes[4 * i + 2];
        size = leaf_boxes[4 * i + 3];
    }
    const double n_start = n_HI[i];
    double best = __builtin_inf();
#pragma unroll 1
    for (int dir = 0; dir < 6; ++dir) {
        const int d = dir >> 1;
        const double sgn = (dir & 1) ? -1.0 : 1.0;
        double p[3], k[3], ik[3];
#pragma unroll
        for (int e = 0; e < 3; ++e) {
            p[e] = lo[e] + 0.5 * size;
            k[e] = (e == d) ? sgn : 0.0;
            ik[e] = k[e];
            if (e == d) p[e] = (sgn > 0.0) ? lo[e] + size : lo[e];
        }
        double sum = 0.0;
        CellBox c;
        if (locate(g, p, k, c)) {
            for (;;) {
                const double nn = n_HI[c.cell];
                if (!(::fabs(nn - n_start) < f_nl * n_start)) break;
                const CellRec<double> cr = load_cell<double>(g, c.cell);
                int axis;
                bool by_sphere;
                const double l = exit_distance(g, c, p, k, ik, axis, by_sphere);
                sum += cr.a * cr.k0 * l;
                if (by_sphere) break;
#pragma unroll
                for (int e = 0; e < 3; ++e) p[e] += l * k[e];
                if (!cross(g, c, p, k, axis)) break;
            }
        }
        best = (sum < best) ? sum : best;
    }
    ad[i].atau_nl = best;
    af[i].atau_nl = (float)best;
}

// ---------------------------------------------------------------------------
// Device checks.
// ---------------------------------------------------------------------------
template <typename R>
__global__ void k_voigt(int64_t n, const double *a, const double *x, double *out)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = (double)voigt_H<R>((R)a[i], (R)x[i]);
}

// what 0: u_par with the cooperative sampler (x = p1); what 4: the same with
// x varying across lanes, x_i = p1 + 0.41 (i mod 23) (-1)^i; what 5 and 6:
// the same two with the one-lane sequential sampler.
template <typename R>
__global__ __launch_bounds__(256) void k_sample(int what, double p0, double p1, double p2,
                                                uint64_t seed, int64_t n, double *out,
                                                int32_t *draws)
{
    __shared__ UparSlot<R, false> s_slots[4][64];
    __shared__ int32_t s_table[4][64];
    __shared__ uint32_t s_first[4][64];
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int wave = threadIdx.x >> 6;
    const bool live = i < n;
    Rng<R> rng;
    rng.init(seed, (uint64_t)(live ? i : 0));
    if (what == 0 || what == 4) {
        R x = (R)p1;
        if (what == 4) x = (R)(p1 + 0.41 * (double)(i % 23) * ((i & 1) ? -1.0 : 1.0));
        const UparReq<R> q = upar_setup<R>((R)p0, x, (R)p2);
        const uint64_t B0 = rng.align();
        R u = R(0);
        uint32_t t = 0;
        bool ok = true;
        coop_upar<R, false>(live && q.regime != UPAR_GAUSS, q, rng.key, B0, u, t, ok, s_slots[wave],
                     s_table[wave], s_first[wave]);
        if (!live) return;
        if (q.regime == UPAR_GAUSS) {
            u = upar_gauss<R>(q, rng.key, B0);
            rng.k += Rng<R>::kPerBlock;
        } else {
            rng.k += upar_advance<R>(q.regime, t);
        }
        out[i] = (double)((x < R(0)) ? -u : u);
        draws[i] = ok ? (int32_t)rng.k : -1;
        return;
    }
    if (!live) return;
    if (what == 1) {
        R u1, u2;
        draw_uperp<R>((R)p0, rng, u1, u2);
        out[2 * i] = (double)u1;
        out[2 * i + 1] = (double)u2;
    } else if (what == 2) {
        out[i] = (double)draw_mu<R>((R)p0, rng);
    } else if (what == 5 || what == 6) {
        R x = (R)p1;
        if (what == 6) x = (R)(p1 + 0.41 * (double)(i % 23) * ((i & 1) ? -1.0 : 1.0));
        uint32_t tries = 0;
        out[i] = (double)draw_upar<R>((R)p0, x, (R)p2, rng, tries);
        draws[i] = (int32_t)rng.k;
    } else if (what == 7) {
        const int64_t skip = (int64_t)p0;
        for (int64_t j = 0; j < skip; ++j) (void)rng.next();
        R d[5];
        if constexpr (sizeof(R) == 4) {
            rng.next5(d);
        } else {
#pragma unroll
            for (int j = 0; j < 5; ++j) d[j] = rng.next();
        }
#pragma unroll
        for (int j = 0; j < 5; ++j) out[5 * i + j] = (double)d[j];
    } else {
        const int64_t m = (int64_t)p0;
        for (int64_t j = 0; j < m; ++j) out[i * m + j] = (double)rng.next();
    }
}

// ---------------------------------------------------------------------------
// Launch table of the allocation-free entry point (colt_transport_static):
// one fixed device array, `scratch`, held by every GPU the library runs on
// until the process ends.  Job views reach it through k_put_views, whose
// kernel arguments carry them (no host staging buffer, no copy from pageable
// memory); k_plan fills the rest.  Host code addresses the array only through
// the pointer hipGetSymbolAddress gives on each device (the array's name is a
// host-side stand-in, not a device address).
// ---------------------------------------------------------------------------
static __device__ __align__(256) unsigned char scratch[kStaticTableBytes];

constexpr int kViewsPerPut = 7;
struct ViewChunk {
    JobView v[kViewsPerPut];
    int32_t n, first;
};
static_assert(sizeof(ViewChunk) + sizeof(void *) <= 4096, "kernel arguments fit 4 KB");

__global__ void k_put_views(ViewChunk c, JobView *dst)
{
    const int i = threadIdx.x;
    if (i < c.n) dst[c.first + i] = c.v[i];
}

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void *g_scratch_ptr[kMaxDevices];

hipError_t static_table(void **ptr)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_ptr[dev] = p;
    }
    *ptr = g_scratch_ptr[dev];
    return hipSuccess;
}

hipError_t put_views(const JobView *views, int n, JobView *dst, hipStream_t s)
{
    for (int first = 0; first < n; first += kViewsPerPut) {
        ViewChunk c{};
        c.n = (n - first < kViewsPerPut) ? n - first : kViewsPerPut;
        c.first = first;
        for (int i = 0; i < c.n; ++i) c.v[i] = views[first + i];
        hipLaunchKernelGGL(k_put_views, dim3(1), dim3(64), 0, s, c, dst);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

// ---------------------------------------------------------------------------
// Host-side launchers.
// ---------------------------------------------------------------------------
hipError_t launch_cell_setup(int64_t n, const double *n_HI, const double *T, const double *v,
                             const double *k_dust, const double *atau_nl, double dx_cm,
                             void *rd, void *ad, void *rf, int rf_stride, void *af, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    const int block = 256;
    const int64_t grid = (n + block - 1) / block;
    hipLaunchKernelGGL(k_cell_setup, dim3((unsigned)grid), dim3(block), 0, s, n, n_HI, T, v,
                       k_dust, atau_nl, dx_cm, (CellRec<double> *)rd, (CellAux<double> *)ad,
                       (CellRec<float> *)rf, rf_stride, (CellAux<float> *)af);
    return hipGetLastError();
}

template <typename R, bool CAMS, bool SINGLE, int GK = -1>
static hipError_t launch_t(const LaunchView &L, const JobView &J1, int grid, int block,
                           hipStream_t s)
{
    hipLaunchKernelGGL((k_transport<R, CAMS, SINGLE, GK>), dim3(grid), dim3(block), 0, s, L, J1);
    return hipGetLastError();
}

template <typename R, bool CAMS, bool SINGLE, int GK = -1>
static hipError_t occupancy_t(int block, int *blocks_per_cu)
{
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu,
                                                        k_transport<R, CAMS, SINGLE, GK>, block, 0);
}

hipError_t launch_transport(int precision, bool cams, const LaunchView &L, const JobView &J1,
                            int grid, int block, hipStream_t s)
{
    const bool single = L.n_jobs == 1;
    if (precision == 0) {
        if (cams) return single ? launch_t<double, true, true>(L, J1, grid, block, s)
                                : launch_t<double, true, false>(L, J1, grid, block, s);
        return single ? launch_t<double, false, true>(L, J1, grid, block, s)
                      : launch_t<double, false, false>(L, J1, grid, block, s);
    }
    if (!single)
        return cams ? launch_t<float, true, false>(L, J1, grid, block, s)
                    : launch_t<float, false, false>(L, J1, grid, block, s);
    if (J1.g.kind == 0)
        return cams ? launch_t<float, true, true, 0>(L, J1, grid, block, s)
                    : launch_t<float, false, true, 0>(L, J1, grid, block, s);
    return cams ? launch_t<float, true, true, 1>(L, J1, grid, block, s)
                : launch_t<float, false, true, 1>(L, J1, grid, block, s);
}

hipError_t transport_occupancy(int precision, bool cams, bool single, int grid_kind, int block,
                               int *blocks_per_cu)
{
    if (precision == 0) {
        if (cams) return single ? occupancy_t<double, true, true>(block, blocks_per_cu)
                                : occupancy_t<double, true, false>(block, blocks_per_cu);
        return single ? occupancy_t<double, false, true>(block, blocks_per_cu)
                      : occupancy_t<double, false, false>(block, blocks_per_cu);
    }
    if (!single)
        return cams ? occupancy_t<float, true, false>(block, blocks_per_cu)
                    : occupancy_t<float, false, false>(block, blocks_per_cu);
    if (grid_kind == 0)
        return cams ? occupancy_t<float, true, true, 0>(block, blocks_per_cu)
                    : occupancy_t<float, false, true, 0>(block, blocks_per_cu);
    return cams ? occupancy_t<float, true, true, 1>(block, blocks_per_cu)
                : occupancy_t<float, false, true, 1>(block, blocks_per_cu);
}

hipError_t launch_plan(const LaunchView &L, bool advance, hipStream_t s)
{
    if (advance) hipLaunchKernelGGL(k_advance, dim3(1), dim3(256), 0, s, L);
    else hipLaunchKernelGGL(k_plan, dim3(1), dim3(256), 0, s, L);
    return hipGetLastError();
}

template <typename R, int GK>
static hipError_t peel_t(const JobView &J, unsigned long long *work, int grid, hipStream_t s)
{
    hipLaunchKernelGGL((k_peel<R, GK>), dim3(grid), dim3(256), 0, s, J, work);
    return hipGetLastError();
}

hipError_t launch_peel(int precision, const JobView &J, unsigned long long *work, int grid,
                       hipStream_t s)
{
    if (precision == 0)
        return J.g.kind == 0 ? peel_t<double, 0>(J, work, grid, s)
                             : peel_t<double, 1>(J, work, grid, s);
    return J.g.kind == 0 ? peel_t<float, 0>(J, work, grid, s)
                         : peel_t<float, 1>(J, work, grid, s);
}

hipError_t peel_occupancy(int precision, int grid_kind, int *blocks_per_cu)
{
    if (precision == 0)
        return grid_kind == 0
                   ? hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, k_peel<double, 0>, 256, 0)
                   : hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, k_peel<double, 1>, 256, 0);
    return grid_kind == 0
               ? hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, k_peel<float, 0>, 256, 0)
               : hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, k_peel<float, 1>, 256, 0);
}

hipError_t launch_nonlocal(const GridView &g, const double *n_HI, const double *leaf_boxes,
                           int64_t n, double f_nl, void *ad, void *af, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    const int block = 128;
    const unsigned grid = (unsigned)((n + block - 1) / block);
    GridView gd = g;          // FP64 records
    hipLaunchKernelGGL(k_nonlocal, dim3(grid), dim3(block), 0, s, gd, n_HI, leaf_boxes, n, f_nl,
                       (CellAux<double> *)ad, (CellAux<float> *)af);
    return hipGetLastError();
}

hipError_t launch_voigt(int precision, int64_t n, const double *a, const double *x, double *out,
                        hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    const int block = 256;
    const unsigned grid = (unsigned)((n + block - 1) / block);
    if (precision == 0)
        hipLaunchKernelGGL(k_voigt<double>, dim3(grid), dim3(block), 0, s, n, a, x, out);
    else
        hipLaunchKernelGGL(k_voigt<float>, dim3(grid), dim3(block), 0, s, n, a, x, out);
    return hipGetLastError();
}

hipError_t launch_sample(int precision, int what, double p0, double p1, double p2,
                         uint64_t seed, int64_t n, double *out, int32_t *draws, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    const int block = 256;   // k_sample keeps per-wave LDS for four waves
    const unsigned grid = (unsigned)((n + block - 1) / block);
    if (precision == 0)
        hipLaunchKernelGGL(k_sample<double>, dim3(grid), dim3(block), 0, s, what, p0, p1, p2,
                           seed, n, out, draws);
    else
        hipLaunchKernelGGL(k_sample<float>, dim3(grid), dim3(block), 0, s, what, p0, p1, p2,
                           seed, n, out, draws);
    return hipGetLastError();
}

}  // namespace colt

