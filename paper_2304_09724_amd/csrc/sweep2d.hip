// sweep2d.hip -- one 2D ADER-SHWENO time step for a batch of rectangles:
// an x-sweep and a y-sweep kernel (unsplit: both read the state at t_n), the
// CFL reduction, and the small kernels that run the per-instance time loop on
// the device (step size, time, ping-pong parity, done and non-physical
// flags), so a sequence of steps can be replayed as one HIP graph.
//
// A sweep kernel works on tiles of L lines x 60 cells (L = 1, 2 or 4, the
// tile variant the autotuner picks): one wave per line
// (a row for the x-sweep, a column for the y-sweep), one lane per cell.  Lane
// l holds cell c0 + l - 2.  Every lane does stage 1 of its cell (transverse
// reconstruction, sec. 3.2); lanes 1..62 do stage 2 at each of the four
// Gauss-Lobatto edge nodes, getting the neighbours' stage-1 node values by
// wave shuffles; lanes 2..62 solve the GRP at their cell's lower interface
// node by node (sec. 3.1) and accumulate the flux of eq. (fx2d); lanes 2..61
// update their cell (sec. 3, the 2D form of eq. (cons), eqs. (derave2d)).
// The y-sweep runs the same code on the state seen with x and y exchanged.
#include "lanes.h"
#include "shw_kernels.h"
#include "sweep2d_math.h"

namespace shw {

namespace {

constexpr int WAVE = 64;
constexpr int BLOCK = 256;
constexpr int LINES = BLOCK / WAVE;
constexpr int CHUNK = WAVE - 4;

// a value the same in every lane, moved to a scalar register
__device__ __forceinline__ double uniform(double x)
{
    const long long b = __double_as_longlong(x);
    const int lo = __builtin_amdgcn_readfirstlane((int)(b & 0xffffffff));
    const int hi = __builtin_amdgcn_readfirstlane((int)(b >> 32));
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

// A double parked in two accumulation registers until it is needed: the GRP
// seeds of an edge node wait there for its Lax-Wendroff series, written once
// and read once, so the architectural registers keep the stage-2 working set.
struct Parked {
    unsigned lo, hi;
};

__device__ __forceinline__ Parked park(double x)
{
    const unsigned long long b = (unsigned long long)__double_as_longlong(x);
    Parked p;
    asm("v_accvgpr_write_b32 %0, %1" : "=a"(p.lo) : "v"((unsigned)b));
    asm("v_accvgpr_write_b32 %0, %1" : "=a"(p.hi) : "v"((unsigned)(b >> 32)));
    return p;
}

__device__ __forceinline__ double unpark(Parked p)
{
    unsigned lo, hi;
    asm("v_accvgpr_read_b32 %0, %1" : "=v"(lo) : "a"(p.lo));
    asm("v_accvgpr_read_b32 %0, %1" : "=v"(hi) : "a"(p.hi));
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// source index of a (possibly ghost) index j of an axis of n cells
__device__ __forceinline__ int map_index(int j, int n, int bc_lo, int bc_hi, int &kind)
{
    kind = -1;
    if (j >= 0 && j < n) return j;
    kind = j < 0 ? bc_lo : bc_hi;
    if (kind == BC_PERIODIC) return j < 0 ? j + n : j - n;
    if (kind == BC_TRANSMISSIVE) return j < 0 ? 0 : n - 1;
    return j < 0 ? -1 - j : 2 * n - 1 - j;
}

// The four averages of the cell at sweep index s, transverse index t, seen in
// the frame of sweep direction DIR (for DIR = 1: x <-> y, V <-> Y, momenta
// swapped).  Ghost cells by the boundary conditions of each axis: periodic
// wrap; transmissive copies with every average containing the normal
// derivative set to zero; reflective mirrors with odd quantities negated.
template <int EQ, int M, int DIR>
__device__ __forceinline__ long long load_cell2d(const double *__restrict__ base, const Inst2D &d,
                                                 int s, int t, double W[M], double V[M],
                                                 double Y[M], double Z[M])
{
    const int i = DIR == 0 ? s : t, j = DIR == 0 ? t : s;
    int kx, ky;
    const int si = map_index(i, d.nx, d.bc[0], d.bc[1], kx);
    const int sj = map_index(j, d.ny, d.bc[2], d.bc[3], ky);
    const long long plane = (long long)d.nx * d.ny;
    const long long o = (long long)sj * d.nx + si;
    double q[4][M];
#pragma unroll
    for (int k = 0; k < 4; ++k)
#pragma unroll
        for (int c = 0; c < M; ++c) q[k][c] = base[(k * M + c) * plane + o];
    if (kx == BC_TRANSMISSIVE) {
#pragma unroll
        for (int c = 0; c < M; ++c) { q[1][c] = 0.0; q[3][c] = 0.0; }
    } else if (kx == BC_REFLECTIVE) {
#pragma unroll
        for (int c = 0; c < M; ++c) {
            const double par = (EQ == EULER && c == 1) ? -1.0 : 1.0;
            q[0][c] *= par; q[1][c] *= -par; q[2][c] *= par; q[3][c] *= -par;
        }
    }
    if (ky == BC_TRANSMISSIVE) {
#pragma unroll
        for (int c = 0; c < M; ++c) { q[2][c] = 0.0; q[3][c] = 0.0; }
    } else if (ky == BC_REFLECTIVE) {
#pragma unroll
        for (int c = 0; c < M; ++c) {
            const double par = (EQ == EULER && c == 2) ? -1.0 : 1.0;
            q[0][c] *= par; q[1][c] *= par; q[2][c] *= -par; q[3][c] *= -par;
        }
    }
#pragma unroll
    for (int c = 0; c < M; ++c) {
        const int cc = (DIR == 1 && EQ == EULER && (c == 1 || c == 2)) ? 3 - c : c;
        W[c] = q[0][cc];
        V[c] = DIR == 0 ? q[1][cc] : q[2][cc];
        Y[c] = DIR == 0 ? q[2][cc] : q[1][cc];
        Z[c] = q[3][cc];
    }
    return o;
}

__device__ __forceinline__ int find_instance(const int *__restrict__ off, int n, int b)
{
    int lo = 0, hi = n;          // off[lo] <= b < off[hi]
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (off[mid] <= b) lo = mid; else hi = mid;
    }
    return lo;
}

// Workgroups go to the eight XCDs in turn (workgroup b to XCD b mod 8), each
// XCD with its own L2.  Tile numbers are dealt so that every XCD takes a
// contiguous run of them (XCD x the x-th of eight near-equal runs, in order):
// neighbouring tiles, which share cache lines (a y-sweep's adjacent columns,
// an x-sweep's transverse stencil rows), then fill one L2 instead of eight.
// A bijection of [0, nblocks) onto itself for any nblocks.
__device__ __forceinline__ int xcd_tile(int b, int nblocks)
{
    constexpr int XCDS = 8;
    const int q = nblocks / XCDS, r = nblocks % XCDS;
    const int x = b % XCDS;
    return x * q + min(x, r) + b / XCDS;
}

// The running tiles of a step (those of the instances still advancing,
// numbered consecutively by compact2d_kernel) go to the grid's first
// workgroups, dealt over the XCDs as above: as instances finish, the tiles
// left still spread over all eight XCDs.  The grid is sized for every
// instance's tiles; a workgroup past the running ones gets -1 and returns.
__device__ __forceinline__ int xcd_running_tile(int b, int running)
{
    return b < running ? xcd_tile(b, running) : -1;
}

// Positivity safeguard records (Euler): record q of a face, q < 4 the flux
// averaged over the step and the edge, 4 + 4g + c component c of the value at
// t_{n+1} at edge node g; components in the (x, y) frame.  An instance's
// x-faces (row j, face f = 0..nx between cells f-1 and f) come first, then its
// y-faces (column i, face f = 0..ny).
constexpr int REC = 20;

__device__ __forceinline__ long long xface_rec(const Inst2D &d, int q, int j, int f)
{
    return d.face_off + ((long long)q * d.ny + j) * (d.nx + 1) + f;
}

__device__ __forceinline__ long long yface_rec(const Inst2D &d, int q, int i, int f)
{
    return d.face_off + (long long)REC * d.ny * (d.nx + 1) + ((long long)q * (d.ny + 1) + f) * d.nx + i;
}

// FULL: every cell takes the nonlinear weights (the paper's scheme): the
// per-cell choice and its branches compile away.  CHAR (Euler): launched
// only with the characteristic path on (P.charwise), which compiles away
// the componentwise path's weights, and with FULL the whole componentwise
// path (see stage1).
template <int EQ, int DIR, int L, bool FULL, bool CHAR>
__global__ void __launch_bounds__(64 * L) sweep2d_kernel(Step2D S, DevParams P)
{
    constexpr int NB = 64 * L;
    constexpr int M = NComp<EQ, 2>::M;
    const int bid = xcd_running_tile(blockIdx.x, S.act_n[1 + DIR]);
    if (bid < 0) return;
    const int k = find_instance(S.act_off[DIR], S.act_n[0], bid);
    const int inst = S.act_inst[k];
    const double dt = S.dt[inst];
    const Inst2D d = S.inst[inst];
    const int ns = DIR == 0 ? d.nx : d.ny, nt = DIR == 0 ? d.ny : d.nx;
    const double dS = DIR == 0 ? d.dx : d.dy, dT = DIR == 0 ? d.dy : d.dx;
    const double as = DIR == 0 ? P.adv_a : P.adv_b, at = DIR == 0 ? P.adv_b : P.adv_a;
    const int tiles_s = (ns + CHUNK - 1) / CHUNK, tiles_t = (nt + L - 1) / L;
    const int tile = bid - S.act_off[DIR][k];
    const int lane = threadIdx.x % WAVE, wave = threadIdx.x / WAVE;
    // consecutive tiles: along the lines for the x-sweep (a row band at a
    // time), across them for the y-sweep (a band of rows over all columns),
    // so tiles running together read the same cache lines (a line holds 16
    // neighbouring columns of a row)
    const int tile_s = DIR == 0 ? tile % tiles_s : tile / tiles_t;
    const int tile_t = DIR == 0 ? tile / tiles_s : tile % tiles_t;
    const int t = tile_t * L + wave;
    if (t >= nt) return;
    const int s = tile_s * CHUNK + lane - 2;
    const bool live = s <= ns + 1;
    const int par = S.parity[inst];
    const double *src = (par ? S.alt : S.state) + d.off;
    double *dst = (par ? S.state : S.alt) + d.off;

    // ---- stage 1 of this lane's cell -------------------------------------
    // The stage-1 polynomials are parked in LDS for the node loop: a 256-lane
    // block of this kernel fills a CU's register file on its own, so the LDS
    // is free; the layout [coefficient][lane] keeps accesses conflict-free.
    __shared__ double s_poly[2][M][5][NB];
    double Wc[M];
    bool full = FULL || P.weights == W_NONLINEAR;
    bool charpath;
    {
        double PW[M][5], PV[M][5];
        double W[3][M], V[3][M], Y[3][M], Z[3][M];
        if (live) {
            long long o = 0;
#pragma unroll
            for (int l = 0; l < 3; ++l) {
                const long long ol = load_cell2d<EQ, M, DIR>(src, d, s, t - 1 + l, W[l], V[l], Y[l], Z[l]);
                if (l == 1) o = ol;
            }
            if constexpr (!FULL)
                if (P.weights == W_GATED || P.weights == W_LEARNED) full = S.flags[d.cell_off + o] != 0;
        }
        // one reconstruction path per wave: characteristic if any lane needs
        // the nonlinear weights
        charpath = FULL || __any(full);
        if (live) {
            stage1<M, EQ, CHAR, FULL>(W, V, Y, Z, dT, full, charpath, P, PW, PV);
#pragma unroll
            for (int c = 0; c < M; ++c) Wc[c] = W[1][c];
        } else {
#pragma unroll
            for (int c = 0; c < M; ++c) {
                Wc[c] = 1.0;
#pragma unroll
                for (int k = 0; k < 5; ++k) { PW[c][k] = 0.0; PV[c][k] = 0.0; }
            }
            Wc[M - 1] = 3.0;
        }
#pragma unroll
        for (int c = 0; c < M; ++c)
#pragma unroll
            for (int k = 0; k < 5; ++k) {
                s_poly[0][c][k][threadIdx.x] = PW[c][k];
                s_poly[1][c][k][threadIdx.x] = PV[c][k];
            }
    }
    // the scalings 1/dt^n and 1/(a! ds^a) are the same for the whole block:
    // held in scalar registers (an operand of the vector instructions), not
    // in vector ones.  The node values are taken as Taylor coefficients in
    // t (taylor_at) and the edge jets scaled by 1/a!, so the jets are
    // d^{a+n}W/ds^a dt^n / (a! n!), the seeds of the series the GRP builds
    // (both stages and the derivative Riemann problems are linear in them,
    // the weights coming from order 0)
    const double iT = uniform(1.0 / dT), iS = uniform(1.0 / dS);
    const double sct[5] = {1.0, iT, uniform(iT * iT), uniform(iT * iT * iT),
                           uniform(iT * iT * iT * iT)};
    const double scs[5] = {1.0, iS, uniform(0.5 * iS * iS), uniform((1.0 / 6.0) * iS * iS * iS),
                           uniform((1.0 / 24.0) * iS * iS * iS * iS)};
    const double node[4] = {-0.5, -LOB_H, LOB_H, 0.5};
    const double nw[4] = {LOB_W0, LOB_W1, LOB_W1, LOB_W0};

    // the faces' values at t_{n+1} wait in LDS for the update (NB + 1 slots:
    // the update reads its own lane's and the next lane's)
    __shared__ double s_we[4][M][NB + 1];
    double Fh[M];
#pragma unroll
    for (int c = 0; c < M; ++c) Fh[c] = 0.0;
    const bool face = lane >= 2 && lane <= 62 && s >= 0 && s <= ns;
#pragma unroll 1
    for (int g = 0; g < 4; ++g) {
        // characteristic fields of the sweep Jacobian at the cell average
        // (read by stage 2 on characteristic waves only)
        CharX<double> Em{};
        if constexpr (EQ == EULER) {
            if (charpath && P.charwise) char_x(Wc, P.gamma, Em);
        }
        // Stage 2 order by order; each order's jets move to the lane above at
        // once and become the GRP's series seeds there, so only one order of
        // jets is ever held (each lane reads back only its own LDS slots).
        double w[M][3];
        Parked pseed[M][5][5];
        Leading2D<M, EQ, double> G;
#pragma unroll
        for (int n = 0; n <= 4; ++n) {
            double am[M], a0[M], ap[M], bm[M], bp[M];
            // a compiler barrier at each node's first order: the node reads
            // the coefficients from the LDS afresh instead of holding them in
            // registers from the previous node (across the CK series); within
            // the node the compiler may keep or re-read them
            if (n == 0) asm volatile("" ::: "memory");
#pragma unroll
            for (int c = 0; c < M; ++c) {
                double pw[5], pv[5];
#pragma unroll
                for (int k = 0; k < 5; ++k) {
                    pw[k] = s_poly[0][c][k][threadIdx.x];
                    pv[k] = s_poly[1][c][k][threadIdx.x];
                }
                const double A = taylor_at(pw, node[g], n, sct[n]);
                const double B = taylor_at(pv, node[g], n, sct[n]);
                a0[c] = A;
                am[c] = from_lane_below(A);
                ap[c] = from_lane_above(A);
                bm[c] = from_lane_below(B);
                bp[c] = from_lane_above(B);
            }
            // every lane reconstructs: only lanes 1..62 feed a face, but the
            // others (lanes 0 and 63; lanes past the line's end, on zero
            // polynomials and a unit state) work on finite data too, and
            // leaving them out would cost a branch that clears their jets
            double lo[5][M], hi[5][M];
            stage2_order<M, EQ, CHAR, FULL>(n, am, a0, ap, bm, bp, Em, dS, scs, full, charpath, P,
                                            w, lo, hi);
#pragma unroll
            for (int a = 0; a + n <= 4; ++a) {
                double JL[M];
#pragma unroll
                for (int c = 0; c < M; ++c) JL[c] = from_lane_below(hi[a][c]);
                if (face) {
                    if (a + n == 0) {
                        grp2d_leading<M, EQ>(JL, lo[0], P, as, G);
#pragma unroll
                        for (int c = 0; c < M; ++c) pseed[c][0][0] = park(G.Ws[c]);
                    } else {
                        double o[M];
                        grp2d_seed<M, EQ>(JL, lo[a], G, o);
#pragma unroll
                        for (int c = 0; c < M; ++c) pseed[c][a][n] = park(o[c]);
                    }
                }
            }
        }
        if (face) {
            double wt[M][5], Fg[M], Wg[M];
            double seed[M][5][5];
#pragma unroll
            for (int c = 0; c < M; ++c)
#pragma unroll
                for (int a = 0; a < 5; ++a)
#pragma unroll
                    for (int b = 0; a + b < 5; ++b) seed[c][a][b] = unpark(pseed[c][a][b]);
            if constexpr (EQ == EULER) ck2d_euler(seed, P.gamma, wt);
            else ck2d_adv(seed[0], as, at, wt[0]);
            node_flux<M, EQ>(wt, dt, P, as, Fg, Wg);
#pragma unroll
            for (int c = 0; c < M; ++c) {
                Fh[c] += nw[g] * Fg[c];
                s_we[g][c][threadIdx.x] = Wg[c];
            }
        } else {
#pragma unroll
            for (int c = 0; c < M; ++c) s_we[g][c][threadIdx.x] = 0.0;
        }
    }
    // ---- update (this lane's cell; upper interface from lane + 1) ----------
    __syncthreads();            // every lane's face values are in s_we
    double Fu[M], We[4][M], Wu[4][M];
#pragma unroll
    for (int c = 0; c < M; ++c) {
        Fu[c] = from_lane_above(Fh[c]);
#pragma unroll
        for (int g = 0; g < 4; ++g) {
            We[g][c] = s_we[g][c][threadIdx.x];
            Wu[g][c] = s_we[g][c][threadIdx.x + 1];
        }
    }
    if constexpr (EQ == EULER) {
        // the safeguard's record of this lane's lower face (each face once:
        // lanes 2..61, and the last face of the line from lane 62)
        if (S.faces && face && (lane <= 61 || s == ns)) {
#pragma unroll
            for (int c = 0; c < M; ++c) {
                const int cc = (DIR == 1 && (c == 1 || c == 2)) ? 3 - c : c;
                const long long r0 = DIR == 0 ? xface_rec(d, cc, t, s) : yface_rec(d, cc, t, s);
                const long long stride = DIR == 0 ? (long long)d.ny * (d.nx + 1)
                                                  : (long long)(d.ny + 1) * d.nx;
                S.faces[r0] = Fh[c];
#pragma unroll
                for (int g = 0; g < 4; ++g) S.faces[r0 + (long long)(M + M * g) * stride] = We[g][c];
            }
        }
    }
    // lanes 2..61 own the cells of the tile; in the y-sweep every lane stays
    // for the wave's reduction of the non-physical flag and the speed
    const bool own = lane >= 2 && lane <= 61 && s >= 0 && s < ns;
    if (DIR == 0 && !own) return;
    const int i = DIR == 0 ? s : t, j = DIR == 0 ? t : s;
    const long long plane = (long long)d.nx * d.ny;
    const long long o = (long long)j * d.nx + i;
    const double r = dt / dS, iSS = 1.0 / (d.dx * d.dy);
    // the y-sweep adds to what the x-sweep wrote: every value it reads is
    // read before the first store (the stores could alias later reads, so
    // reads after them would each wait for the previous one's round trip)
    double Wx[M], Zx[M];
    if constexpr (DIR == 1) {
#pragma unroll
        for (int c = 0; c < M; ++c) { Wx[c] = 1.0; Zx[c] = 0.0; }
        if (own) {
#pragma unroll
            for (int c = 0; c < M; ++c) {
                Wx[c] = dst[c * plane + o];
                Zx[c] = dst[(3 * M + c) * plane + o];
            }
        }
    }
    double Wn[M];
#pragma unroll
    for (int c = 0; c < M; ++c) {
        const int cc = (DIR == 1 && EQ == EULER && (c == 1 || c == 2)) ? 3 - c : c;
        double dv = 0.0;
#pragma unroll
        for (int g = 0; g < 4; ++g) dv += nw[g] * (Wu[g][c] - We[g][c]);
        const double zc = 0.5 * (Wu[3][c] - We[3][c] - Wu[0][c] + We[0][c]) * iSS;
        if constexpr (DIR == 0) {
            Wn[cc] = src[cc * plane + o] - r * (Fu[c] - Fh[c]);
            dst[cc * plane + o] = Wn[cc];
            dst[(M + cc) * plane + o] = dv * iS;
            dst[(3 * M + cc) * plane + o] = zc;
        } else {
            Wn[cc] = Wx[cc] - r * (Fu[c] - Fh[c]);
            if (own) {
                dst[cc * plane + o] = Wn[cc];
                dst[(2 * M + cc) * plane + o] = dv * iS;
                dst[(3 * M + cc) * plane + o] = Zx[cc] + zc;
            }
        }
    }
    if constexpr (DIR == 1) {
        // non-physical check and the wave speed for the next step's CFL
        bool bad = false;
        double spd = 0.0;
        if (own) {
#pragma unroll
            for (int c = 0; c < M; ++c) bad |= !isfinite(Wn[c]);
            if constexpr (EQ == EULER) {
                const double ir = 1.0 / Wn[0];
                const double u = Wn[1] * ir, v = Wn[2] * ir;
                const double p = (P.gamma - 1.0) * (Wn[3] - 0.5 * Wn[0] * (u * u + v * v));
                bad |= !(Wn[0] > 0.0) || !(p > 0.0);
                if (!bad) {
                    const double c = sqrt(P.gamma * p * ir);
                    spd = (fabs(u) + c) / d.dx + (fabs(v) + c) / d.dy;
                }
            } else {
                spd = fabs(P.adv_a) / d.dx + fabs(P.adv_b) / d.dy;
            }
        }
        // one atomic of each kind per wave (speeds are >= 0, and such doubles
        // order like their bit patterns)
        const bool any_bad = __any(bad);
#pragma unroll
        for (int m = 32; m > 0; m >>= 1) spd = fmax(spd, __shfl_xor(spd, m, WAVE));
        if (lane == 0) {
            if (any_bad) atomicOr(&S.bad[inst], 1);
            atomicMax(reinterpret_cast<unsigned long long *>(&S.smax[inst]),
                      (unsigned long long)__double_as_longlong(spd));
        }
    }
}

// The learned gate of one 2D Euler step: for every cell of the instances
// that step, the network scores the cell along x and along y (features of the
// line through the cell in that direction, its normal components; the
// network is the 1D one) and the cell takes the nonlinear weights if either
// score reaches the threshold.  Both sweeps of the step read the flags.
// Tiles as for the x-sweep: L rows x 60 cells, one wave per row, lane l on
// cell c0 + l - 2 (every lane evaluates; lanes 2..61 store).
// A lane's slice of the packed network (256 bytes) read straight from
// global memory: the 16 KB network stays in the caches, and each wave of the
// gate kernel reads it once for all its tiles.
__device__ __forceinline__ GateLane gate_lane_global(const GateLane *g, int lane)
{
    GateLane G;
    const u32x4 *src = reinterpret_cast<const u32x4 *>(g + lane);
    u32x4 *dst = reinterpret_cast<u32x4 *>(&G);
#pragma unroll
    for (int w = 0; w < 16; ++w) dst[w] = src[w];
    return G;
}

template <int L>
__global__ void __launch_bounds__(64 * L) __attribute__((amdgpu_waves_per_eu(4)))
gate2d_kernel(Step2D S, DevParams P)
{
    constexpr int M = 4;
    // The grid holds as many workgroups as the device runs at once (a
    // multiple of 8); each walks the running tiles with the grid's stride
    // (tile numbers v = blockIdx.x + k gridDim.x stay on this workgroup's
    // XCD, v mod 8), with the network in registers throughout.  No LDS, so
    // the registers alone bound the waves per SIMD.
    const int lane = threadIdx.x % WAVE, wave = threadIdx.x / WAVE;
    const GateLane G = gate_lane_global(S.gate, lane);
    const int running = S.act_n[1];
    for (int v = blockIdx.x; v < running; v += gridDim.x) {
        const int bid = xcd_tile(v, running);
        const int k = find_instance(S.act_off[0], S.act_n[0], bid);
        const int inst = S.act_inst[k];
        const Inst2D d = S.inst[inst];
        const int tiles_s = (d.nx + CHUNK - 1) / CHUNK;
        const int tile = bid - S.act_off[0][k];
        const int t = (tile / tiles_s) * L + wave;
        if (t >= d.ny) continue;                  // the whole wave: past the last row
        const int s = (tile % tiles_s) * CHUNK + lane - 2;
        const int sc = s < 0 ? 0 : (s >= d.nx ? d.nx - 1 : s);   // lanes off the row: any cell
        const double *src = (S.parity[inst] ? S.alt : S.state) + d.off;
        float z[2];
        {
            double Wm[M], W0[M], Wp[M], Vm[M], V0[M], Vp[M], Y[M], Z[M];
            load_cell2d<EULER, M, 0>(src, d, sc - 1, t, Wm, Vm, Y, Z);
            load_cell2d<EULER, M, 0>(src, d, sc, t, W0, V0, Y, Z);
            load_cell2d<EULER, M, 0>(src, d, sc + 1, t, Wp, Vp, Y, Z);
            float f[GATE_NF];
            gate_features<M>(Wm, W0, Wp, Vm, Vp, d.dx, P.gamma, f);
            z[0] = gate_wave_logit(f, G);
        }
        {
            double Wm[M], W0[M], Wp[M], Vm[M], V0[M], Vp[M], Y[M], Z[M];
            load_cell2d<EULER, M, 1>(src, d, t - 1, sc, Wm, Vm, Y, Z);
            load_cell2d<EULER, M, 1>(src, d, t, sc, W0, V0, Y, Z);
            load_cell2d<EULER, M, 1>(src, d, t + 1, sc, Wp, Vp, Y, Z);
            float f[GATE_NF];
            gate_features<M>(Wm, W0, Wp, Vm, Vp, d.dy, P.gamma, f);
            z[1] = gate_wave_logit(f, G);
        }
        if (lane >= 2 && lane <= 61 && s < d.nx)
            S.flags[d.cell_off + (long long)t * d.nx + s] =
                (uint8_t)(fmaxf(z[0], z[1]) >= S.gate_logit_min);
    }
}

// max over the cells of (|u|+c)/dx + (|v|+c)/dy: SPEED_SPLIT blocks per
// instance (grid SPEED_SPLIT x instances), each over every SPEED_SPLIT-th
// stretch of BLOCK cells, combined by an atomic max into the cleared slot
constexpr int SPEED_SPLIT = 64;

__global__ void clear_smax2d_kernel(Step2D S)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < S.n_inst) S.smax[i] = 0.0;
}

// which: 0 the caller's buffer, 1 the current state (by parity), 2 the output
// of the step in flight (the other buffer); only: if set, the instances whose
// entry is non-zero
template <int EQ>
__global__ void __launch_bounds__(BLOCK) speed2d_kernel(Step2D S, DevParams P, int which,
                                                        const int *only)
{
    constexpr int M = NComp<EQ, 2>::M;
    __shared__ double red[LINES];
    const int inst = blockIdx.y;
    if (only && !only[inst]) return;
    const Inst2D d = S.inst[inst];
    const bool alt = which == 1 ? S.parity[inst] != 0 : which == 2 ? S.parity[inst] == 0 : false;
    const double *src = (alt ? S.alt : S.state) + d.off;
    const long long plane = (long long)d.nx * d.ny;
    double m = 0.0;
    bool bad = false;
    for (long long o = (long long)blockIdx.x * BLOCK + threadIdx.x; o < plane;
         o += (long long)SPEED_SPLIT * BLOCK) {
        double W[M];
#pragma unroll
        for (int c = 0; c < M; ++c) W[c] = src[c * plane + o];
        if constexpr (EQ == EULER) {
            const double ir = 1.0 / W[0];
            const double u = W[1] * ir, v = W[2] * ir;
            const double p = (P.gamma - 1.0) * (W[3] - 0.5 * W[0] * (u * u + v * v));
            const bool b = !isfinite(W[0]) || !isfinite(W[1]) || !isfinite(W[2]) ||
                           !isfinite(W[3]) || !(W[0] > 0.0) || !(p > 0.0);
            bad |= b;
            if (!b) {
                const double c = sqrt(P.gamma * p * ir);
                m = fmax(m, (fabs(u) + c) / d.dx + (fabs(v) + c) / d.dy);
            }
        } else {
            bad |= !isfinite(W[0]);
            m = fmax(m, fabs(P.adv_a) / d.dx + fabs(P.adv_b) / d.dy);
        }
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) m = fmax(m, __shfl_xor(m, o, WAVE));
    if (threadIdx.x % WAVE == 0) red[threadIdx.x / WAVE] = m;
    const int any_bad = __syncthreads_or(bad);
    if (threadIdx.x == 0) {
        double r = red[0];
        for (int w = 1; w < LINES; ++w) r = fmax(r, red[w]);
        // positive doubles order like their bit patterns
        atomicMax(reinterpret_cast<unsigned long long *>(&S.smax[inst]),
                  (unsigned long long)__double_as_longlong(r));
        if (any_bad) atomicOr(&S.bad[inst], 1);
    }
}

// ---- positivity safeguard (an addition to the paper's scheme; Euler) -----
// After the sweeps of a step that left a non-physical average: cells whose
// new average is non-physical are troubled (the test written as p = (g-1)(E -
// (mx^2 + my^2)/(2 rho)) > 0, so the decision rounds as a plain evaluation of
// that formula does); every x- and y-face next to a troubled cell takes the
// first-order HLLE flux of the two averages at t_n, its state at x/t = 0
// standing for the face value at all four edge nodes, and the cells on both
// sides are updated again from the sweeps' records of their other faces
// (conservative).  One round: a cell still non-physical stops its instance.
__device__ __forceinline__ bool troubled2d(const double W[4], const DevParams &P)
{
    if (!isfinite(W[0]) || !isfinite(W[1]) || !isfinite(W[2]) || !isfinite(W[3]) ||
        !(W[0] > 0.0))
        return true;
    double ke = 0.5 * W[1] * W[1] / W[0];
    ke += 0.5 * W[2] * W[2] / W[0];
    return !((P.gamma - 1.0) * (W[3] - ke) > 0.0);
}

__device__ __forceinline__ bool repairing(const Step2D &S, int inst)
{
    return S.bad[inst] != 0 && S.dt[inst] > 0.0;
}

__global__ void __launch_bounds__(BLOCK) guard_mark2d_kernel(Step2D S, DevParams P)
{
    const int inst = blockIdx.y;
    if (!repairing(S, inst)) return;
    const Inst2D d = S.inst[inst];
    const double *out = (S.parity[inst] ? S.state : S.alt) + d.off;
    const long long plane = (long long)d.nx * d.ny;
    for (long long o = (long long)blockIdx.x * BLOCK + threadIdx.x; o < plane;
         o += (long long)SPEED_SPLIT * BLOCK) {
        const double W[4] = {out[o], out[plane + o], out[2 * plane + o], out[3 * plane + o]};
        S.trouble[d.cell_off + o] = (uint8_t)troubled2d(W, P);
    }
}

// HLLE face between two cells loaded from the state at t_n (ghosts by the
// boundary conditions); dir 1: a y-face, solved with x and y exchanged
__device__ void hlle2d(const Inst2D &d, const double *src, int i0, int j0, int i1, int j1,
                       int dir, const DevParams &P, double F[4], double Ws[4])
{
    double WL[4], WR[4], V[4], Y[4], Z[4];
    load_cell2d<EULER, 4, 0>(src, d, i0, j0, WL, V, Y, Z);
    load_cell2d<EULER, 4, 0>(src, d, i1, j1, WR, V, Y, Z);
    if (dir == 0) {
        hlle_face<2>(WL, WR, P, F, Ws);
        return;
    }
    const double RL[4] = {WL[0], WL[2], WL[1], WL[3]}, RR[4] = {WR[0], WR[2], WR[1], WR[3]};
    double Fr[4], Sr[4];
    hlle_face<2>(RL, RR, P, Fr, Sr);
    F[0] = Fr[0]; F[1] = Fr[2]; F[2] = Fr[1]; F[3] = Fr[3];
    Ws[0] = Sr[0]; Ws[1] = Sr[2]; Ws[2] = Sr[1]; Ws[3] = Sr[3];
}

__global__ void __launch_bounds__(BLOCK) guard_fix2d_kernel(Step2D S, DevParams P)
{
    constexpr int M = 4;
    const int inst = blockIdx.y;
    if (!repairing(S, inst)) return;
    const Inst2D d = S.inst[inst];
    const double *src = (S.parity[inst] ? S.alt : S.state) + d.off;
    double *out = (S.parity[inst] ? S.state : S.alt) + d.off;
    const uint8_t *tr = S.trouble + d.cell_off;
    const long long plane = (long long)d.nx * d.ny;
    const double dt = S.dt[inst];
    const double nw[4] = {LOB_W0, LOB_W1, LOB_W1, LOB_W0};
    const long long sx = (long long)d.ny * (d.nx + 1), sy = (long long)(d.ny + 1) * d.nx;
    for (long long o = (long long)blockIdx.x * BLOCK + threadIdx.x; o < plane;
         o += (long long)SPEED_SPLIT * BLOCK) {
        const int i = (int)(o % d.nx), j = (int)(o / d.nx);
        int k;
        const int il = map_index(i - 1, d.nx, d.bc[0], d.bc[1], k);
        const int ir = map_index(i + 1, d.nx, d.bc[0], d.bc[1], k);
        const int jb = map_index(j - 1, d.ny, d.bc[2], d.bc[3], k);
        const int jt = map_index(j + 1, d.ny, d.bc[2], d.bc[3], k);
        const bool tc = tr[o] != 0;
        const bool xl = tc || tr[(long long)j * d.nx + il] != 0;
        const bool xr = tc || tr[(long long)j * d.nx + ir] != 0;
        const bool yb = tc || tr[(long long)jb * d.nx + i] != 0;
        const bool yt = tc || tr[(long long)jt * d.nx + i] != 0;
        if (!(xl || xr || yb || yt)) continue;
        // faces: flux and values at t_{n+1} at the four edge nodes
        double F[4][M], E[4][4][M];          // [left, right, bottom, top]
        const bool repl[4] = {xl, xr, yb, yt};
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            if (repl[e]) {
                double Fe[M], Ws[M];
                if (e == 0) hlle2d(d, src, i - 1, j, i, j, 0, P, Fe, Ws);
                else if (e == 1) hlle2d(d, src, i, j, i + 1, j, 0, P, Fe, Ws);
                else if (e == 2) hlle2d(d, src, i, j - 1, i, j, 1, P, Fe, Ws);
                else hlle2d(d, src, i, j, i, j + 1, 1, P, Fe, Ws);
#pragma unroll
                for (int c = 0; c < M; ++c) {
                    F[e][c] = Fe[c];
#pragma unroll
                    for (int g = 0; g < 4; ++g) E[e][g][c] = Ws[c];
                }
            } else {
                const long long r0 = e == 0 ? xface_rec(d, 0, j, i) : e == 1 ? xface_rec(d, 0, j, i + 1)
                                   : e == 2 ? yface_rec(d, 0, i, j) : yface_rec(d, 0, i, j + 1);
                const long long st = e < 2 ? sx : sy;
#pragma unroll
                for (int c = 0; c < M; ++c) {
                    F[e][c] = S.faces[r0 + c * st];
#pragma unroll
                    for (int g = 0; g < 4; ++g) E[e][g][c] = S.faces[r0 + (M + M * g + c) * st];
                }
            }
        }
        const double rx = dt / d.dx, ry = dt / d.dy, iSS = 1.0 / (d.dx * d.dy);
#pragma unroll
        for (int c = 0; c < M; ++c) {
            double V = 0.0, Y = 0.0;
#pragma unroll
            for (int g = 0; g < 4; ++g) {
                V += nw[g] * (E[1][g][c] - E[0][g][c]);
                Y += nw[g] * (E[3][g][c] - E[2][g][c]);
            }
            const double zx = E[1][3][c] - E[0][3][c] - E[1][0][c] + E[0][0][c];
            const double zy = E[3][3][c] - E[2][3][c] - E[3][0][c] + E[2][0][c];
            out[c * plane + o] = src[c * plane + o] - rx * (F[1][c] - F[0][c]) - ry * (F[3][c] - F[2][c]);
            out[(M + c) * plane + o] = V / d.dx;
            out[(2 * M + c) * plane + o] = Y / d.dy;
            out[(3 * M + c) * plane + o] = 0.5 * (zx + zy) * iSS;
        }
    }
}

// per instance: a repaired instance gets its flag and CFL speed anew
__global__ void guard_reset2d_kernel(Step2D S)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= S.n_inst) return;
    const int g = repairing(S, i) ? 1 : 0;
    S.guard[i] = g;
    if (g) {
        S.bad[i] = 0;
        S.smax[i] = 0.0;
    }
}

// per instance, before a step: dt from the CFL condition (or the fixed dt),
// clamped to the end time; 0 for instances that are done or non-physical
__global__ void prepare2d_kernel(Step2D S, DevParams P, int fixed)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i == 0) *S.active = 0;
    if (i >= S.n_inst) return;
    InstState st = S.ist[i];
    double dt = 0.0;
    int last = 0;
    if (S.bad[i] != 0 || st.code != 0) {
        st.code = 1;
    } else if (fixed) {
        dt = S.dt_fixed[i] > 0.0 ? S.dt_fixed[i] : 0.0;
    } else if (st.t < S.t_end[i] && S.steps_left[i] > 0) {
        dt = P.cfl / S.smax[i];
        if (dt >= S.t_end[i] - st.t) { dt = S.t_end[i] - st.t; last = 1; }
    }
    S.dt[i] = dt;
    S.last[i] = last;
    S.smax[i] = 0.0;
    S.ist[i] = st;
}

// The running instances of this step (step size > 0) in order, and per sweep
// direction the first tile of each in a consecutive numbering of their tiles
// (one block: each thread counts a run of instances, a scan over the block
// places the runs, each thread then writes its own).
constexpr int COMPACT_THREADS = 1024;

__global__ void __launch_bounds__(COMPACT_THREADS) compact2d_kernel(Step2D S)
{
    __shared__ int s_cnt[3][COMPACT_THREADS];
    const int n = S.n_inst, tid = threadIdx.x;
    const int per = (n + COMPACT_THREADS - 1) / COMPACT_THREADS;
    const int i0 = min(tid * per, n), i1 = min(i0 + per, n);
    int cnt = 0, tx = 0, ty = 0;
    for (int i = i0; i < i1; ++i)
        if (S.dt[i] > 0.0) {
            ++cnt;
            tx += S.tile_off[0][i + 1] - S.tile_off[0][i];
            ty += S.tile_off[1][i + 1] - S.tile_off[1][i];
        }
    s_cnt[0][tid] = cnt;
    s_cnt[1][tid] = tx;
    s_cnt[2][tid] = ty;
    __syncthreads();
    // exclusive scan of the three counts over the block (Hillis-Steele on the
    // inclusive sums, then shifted)
    for (int o = 1; o < COMPACT_THREADS; o <<= 1) {
        int v[3];
#pragma unroll
        for (int q = 0; q < 3; ++q) v[q] = tid >= o ? s_cnt[q][tid - o] : 0;
        __syncthreads();
#pragma unroll
        for (int q = 0; q < 3; ++q) s_cnt[q][tid] += v[q];
        __syncthreads();
    }
    int k = s_cnt[0][tid] - cnt, ox = s_cnt[1][tid] - tx, oy = s_cnt[2][tid] - ty;
    for (int i = i0; i < i1; ++i)
        if (S.dt[i] > 0.0) {
            S.act_inst[k] = i;
            S.act_off[0][k] = ox;
            S.act_off[1][k] = oy;
            ++k;
            ox += S.tile_off[0][i + 1] - S.tile_off[0][i];
            oy += S.tile_off[1][i + 1] - S.tile_off[1][i];
        }
    if (tid == COMPACT_THREADS - 1) {
        S.act_off[0][k] = ox;
        S.act_off[1][k] = oy;
        S.act_n[0] = k;
        S.act_n[1] = ox;
        S.act_n[2] = oy;
    }
}

// per instance, after a step: time, step count, parity, budget, activity
__global__ void finish2d_kernel(Step2D S)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= S.n_inst) return;
    const double dt = S.dt[i];
    if (!(dt > 0.0)) return;
    InstState st = S.ist[i];
    st.t = S.last[i] ? S.t_end[i] : st.t + dt;
    st.steps += 1;
    if (S.bad[i] != 0) st.code = 1;
    S.ist[i] = st;
    S.parity[i] ^= 1;
    S.steps_left[i] -= 1;
    if (st.code == 0 && st.t < S.t_end[i] && S.steps_left[i] > 0) atomicAdd(S.active, 1);
}

// copy instances whose current state sits in the ping-pong buffer back to
// the caller's buffer (one block per instance)
__global__ void settle2d_kernel(Step2D S, int m)
{
    const int inst = blockIdx.y;
    if (S.parity[inst] == 0) return;
    const Inst2D d = S.inst[inst];
    const long long n = 4LL * m * d.nx * d.ny;
    for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < n;
         e += (long long)gridDim.x * blockDim.x)
        S.state[d.off + e] = S.alt[d.off + e];
}

__global__ void clear_parity2d_kernel(Step2D S)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < S.n_inst) S.parity[i] = 0;
}

} // namespace

int sweep2d_tiles(int n_sweep, int n_trans, int lines)
{
    return ((n_sweep + CHUNK - 1) / CHUNK) * ((n_trans + lines - 1) / lines);
}

hipError_t launch_speed2d(int eq, const Step2D &S, const DevParams &P, int use_parity,
                          hipStream_t st)
{
    clear_smax2d_kernel<<<(S.n_inst + 255) / 256, 256, 0, st>>>(S);
    const dim3 grid(SPEED_SPLIT, S.n_inst);
    if (eq == EULER) speed2d_kernel<EULER><<<grid, BLOCK, 0, st>>>(S, P, use_parity, nullptr);
    else speed2d_kernel<ADV><<<grid, BLOCK, 0, st>>>(S, P, use_parity, nullptr);
    return hipGetLastError();
}

// Workgroups of the gate kernel: as many as the device holds at once (so no
// second round of workgroups trails the first), a multiple of 8 (so a
// workgroup's tiles stay on its XCD), fewer when there are fewer tiles; each
// walks the running tiles with the grid's stride.
template <int L>
static int gate2d_grid(int tiles)
{
    constexpr int MAX_DEVICES = 64;
    static int resident[MAX_DEVICES];          // per device, found on first use
    int dev = 0;
    (void)hipGetDevice(&dev);
    int &r = resident[dev >= 0 && dev < MAX_DEVICES ? dev : 0];
    if (r == 0) {
        int per_cu = 0, cus = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, gate2d_kernel<L>, 64 * L, 0) !=
                hipSuccess || per_cu < 1)
            per_cu = 1;
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
            cus < 1)
            cus = 1;
        const int g = per_cu * cus / 8 * 8;
        r = g < 8 ? 8 : g;
    }
    const int g = (tiles + 7) / 8 * 8;
    return g < r ? (g < 8 ? 8 : g) : r;
}

template <int L>
static void sweeps2d(int eq, const Step2D &S, const DevParams &P, const int total_tiles[2],
                     hipStream_t st)
{
    if (eq == EULER && P.weights == W_LEARNED)
        gate2d_kernel<L><<<gate2d_grid<L>(total_tiles[0]), 64 * L, 0, st>>>(S, P);
    const bool full = P.weights == W_NONLINEAR;
    if (eq == EULER && full && P.charwise) {
        sweep2d_kernel<EULER, 0, L, true, true><<<total_tiles[0], 64 * L, 0, st>>>(S, P);
        sweep2d_kernel<EULER, 1, L, true, true><<<total_tiles[1], 64 * L, 0, st>>>(S, P);
    } else if (eq == EULER && full) {
        sweep2d_kernel<EULER, 0, L, true, false><<<total_tiles[0], 64 * L, 0, st>>>(S, P);
        sweep2d_kernel<EULER, 1, L, true, false><<<total_tiles[1], 64 * L, 0, st>>>(S, P);
    } else if (eq == EULER && P.charwise) {
        sweep2d_kernel<EULER, 0, L, false, true><<<total_tiles[0], 64 * L, 0, st>>>(S, P);
        sweep2d_kernel<EULER, 1, L, false, true><<<total_tiles[1], 64 * L, 0, st>>>(S, P);
    } else if (eq == EULER) {
        sweep2d_kernel<EULER, 0, L, false, false><<<total_tiles[0], 64 * L, 0, st>>>(S, P);
        sweep2d_kernel<EULER, 1, L, false, false><<<total_tiles[1], 64 * L, 0, st>>>(S, P);
    } else {
        sweep2d_kernel<ADV, 0, L, false, false><<<total_tiles[0], 64 * L, 0, st>>>(S, P);
        sweep2d_kernel<ADV, 1, L, false, false><<<total_tiles[1], 64 * L, 0, st>>>(S, P);
    }
}

hipError_t launch_step2d(int eq, const Step2D &S, const DevParams &P, int fixed,
                         const int total_tiles[2], int lines, hipStream_t st)
{
    const int nb = (S.n_inst + 255) / 256;
    prepare2d_kernel<<<nb, 256, 0, st>>>(S, P, fixed);
    compact2d_kernel<<<1, COMPACT_THREADS, 0, st>>>(S);
    if (lines == 1) sweeps2d<1>(eq, S, P, total_tiles, st);
    else if (lines == 2) sweeps2d<2>(eq, S, P, total_tiles, st);
    else sweeps2d<4>(eq, S, P, total_tiles, st);
    if (eq == EULER && S.faces) {
        // the positivity safeguard: every kernel returns at once for the
        // instances whose step left no non-physical average
        const dim3 grid(SPEED_SPLIT, S.n_inst);
        guard_mark2d_kernel<<<grid, BLOCK, 0, st>>>(S, P);
        guard_fix2d_kernel<<<grid, BLOCK, 0, st>>>(S, P);
        guard_reset2d_kernel<<<nb, 256, 0, st>>>(S);
        speed2d_kernel<EULER><<<grid, BLOCK, 0, st>>>(S, P, 2, S.guard);
    }
    finish2d_kernel<<<nb, 256, 0, st>>>(S);
    return hipGetLastError();
}

hipError_t launch_settle2d(const Step2D &S, int m, hipStream_t st)
{
    settle2d_kernel<<<dim3(64, S.n_inst), 256, 0, st>>>(S, m);
    clear_parity2d_kernel<<<(S.n_inst + 255) / 256, 256, 0, st>>>(S);
    return hipGetLastError();
}

} // namespace shw
