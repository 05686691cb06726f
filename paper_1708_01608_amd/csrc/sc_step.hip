// sc_step.hip -- the fused Shan-Chen time step and the state kernels of libsc (gfx950).
//
// Storage: SoA populations f[i][idx] holding the post-collision value of the previous step, so a
// node pulls f_i(x, t) = stored_i(x - e_i) (pull streaming, periodic).  Stored values are
// deviations f_i - w_i rho_ref in FP32 / FP16 / BF16; the arithmetic type A is FP64 or FP32 (FP32
// only on 16-bit storage).  Loaded values stay in FP32 registers (exact for every storage type).
//
// One kernel per time step does, for every node (Sec. 3.1 and Fig. 1 step 6):
//   rho = sum_i f_i, j = sum_i f_i e_i, psi = 1 - exp(-rho)                  (pseudopotential)
//   F = -G psi(x) sum_{i != 0} w_i psi(x + e_i) e_i                        (Shan-Chen force)
//   u_eq = j/rho + tau F/rho;  f_i* = f_i - (f_i - f_i^eq(rho, u_eq))/tau   (forced BGK)
//   store f_i* at x (the next step pulls it from x + e_i)                  (streaming)
// psi of the neighbours needs their densities at the same time level.  A block owns a tile of
// one plane (a row segment in 2D, an x-y tile in 3D) and marches along the remaining axis; the
// psi of three planes (tile + a one-node ring) live in LDS.  Each plane is loaded once: the
// tile's own populations stay in registers for the collision one iteration later, the ring
// nodes' populations are loaded only to form their psi.  Four LDS plane slots let one barrier
// per plane separate writers from readers.
#include <algorithm>
#include <type_traits>

#include "sc_device.hpp"
#include "sc_internal.hpp"
#include "sc_stepcore.hpp"

namespace sc {

size_t storage_bytes(int storage) { return storage == SC_STORE_F32 ? 4 : 2; }

// ------------------------------------------------------------------------------------------
// D2Q9: a block owns TX nodes of a row and marches `planes` rows in y.
// ------------------------------------------------------------------------------------------
template <typename S, typename A, int TX, bool NT = false, bool EXT = false>
__global__ void __launch_bounds__(TX) k_step2d(const S* __restrict__ src, S* __restrict__ dst,
                                               StepArgs a, StepGrid grid)
{
    using L = lat<9>;
    __shared__ A ps[4][TX + 2];
    const Coef<A> c = coef_of(a, A());
    const int nx = a.nx, ny = a.ny;
    const int64_t N = a.N;
    const int lb = logical_block(grid);
    const int bx = lb % grid.gx, by = lb / grid.gx;
    const int tx = threadIdx.x;
    const int x0 = bx * TX;
    const int wx = min(TX, nx - x0);
    const int y0 = by * a.planes;
    const int ye = min(y0 + a.planes, ny);
    const bool own = tx < wx;
    const int x = x0 + (own ? tx : 0);
    const int xm = wrap_once(x - 1, nx), xp = wrap_once(x + 1, nx);
    // the two ring nodes of a row tile: x0 - 1 (thread 0) and x0 + wx (thread 1)
    const bool ring = tx < 2;
    const int hx = tx == 0 ? wrap_once(x0 - 1, nx) : wrap_once(x0 + wx, nx);
    const int hxm = wrap_once(hx - 1, nx), hxp = wrap_once(hx + 1, nx);
    const int hl = tx == 0 ? 0 : wx + 1;

    float cur[9], nxt[9];
    A dcur = (A)0, dnxt = (A)0;

    // prologue: rows y0 - 1 (psi only), y0 and y0 + 1 (psi, populations kept); the three rows'
    // loads are issued together, so the block waits out one memory latency for them
    {
        const int ya = wrap_once(y0 - 1, ny), yb = y0, yc = wrap_once(y0 + 1, ny);
        float g[9], h[3][9];
        if (own) {
            pull_node<9>(src, N, nx, ny, x, xm, xp, ya, wrap_once(ya - 1, ny), wrap_once(ya + 1, ny),
                         0, 0, 0, g);
            pull_node<9>(src, N, nx, ny, x, xm, xp, yb, wrap_once(yb - 1, ny), wrap_once(yb + 1, ny),
                         0, 0, 0, cur);
            pull_node<9>(src, N, nx, ny, x, xm, xp, yc, wrap_once(yc - 1, ny), wrap_once(yc + 1, ny),
                         0, 0, 0, nxt);
        }
        if (ring) {
            const int yy[3] = {ya, yb, yc};
#pragma unroll
            for (int r = 0; r < 3; ++r)
                pull_node<9>(src, N, nx, ny, hx, hxm, hxp, yy[r], wrap_once(yy[r] - 1, ny),
                             wrap_once(yy[r] + 1, ny), 0, 0, 0, h[r]);
        }
        if (own) {
            ps[0][tx + 1] = psi_f(c.rho_ref + sum_dev<9, A>(g));
            dcur = sum_dev<9, A>(cur);
            ps[1][tx + 1] = psi_f(c.rho_ref + dcur);
            dnxt = sum_dev<9, A>(nxt);
            ps[2][tx + 1] = psi_f(c.rho_ref + dnxt);
        }
        if (ring) {
#pragma unroll
            for (int r = 0; r < 3; ++r) ps[r][hl] = psi_f(c.rho_ref + sum_dev<9, A>(h[r]));
        }
    }

    for (int y = y0; y < ye; ++y) {
        const int s = (y - y0 + 1) & 3;
        const int sn = (s + 1) & 3, sp = (s + 3) & 3;
        if (y > y0) {  // row y0 + 1 came with the prologue
            const int yn = wrap_once(y + 1, ny);
            const int ym = wrap_once(yn - 1, ny), yp = wrap_once(yn + 1, ny);
            if (own) {
                pull_node<9>(src, N, nx, ny, x, xm, xp, yn, ym, yp, 0, 0, 0, nxt);
                dnxt = sum_dev<9, A>(nxt);
                ps[sn][tx + 1] = psi_f(c.rho_ref + dnxt);
            }
            if (ring) {
                float h[9];
                pull_node<9>(src, N, nx, ny, hx, hxm, hxp, yn, ym, yp, 0, 0, 0, h);
                ps[sn][hl] = psi_f(c.rho_ref + sum_dev<9, A>(h));
            }
        }
        __syncthreads();
        if (own) {
            const A pc = ps[s][tx + 1];
            A fx, fy, fz;
            interaction_sum<9, A>(
                [&](int i) {
                    const int slot = L::ey[i] > 0 ? sn : (L::ey[i] < 0 ? sp : s);
                    return ps[slot][tx + 1 + L::ex[i]];
                },
                fx, fy, fz);
            const A gp = -c.G * pc;
            collide_store<9, A, S, NT, EXT>(dst, N, (uint32_t)(x + nx * y), cur, dcur, gp * fx,
                                       gp * fy, (A)0, c);
        }
#pragma unroll
        for (int i = 0; i < 9; ++i) cur[i] = nxt[i];
        dcur = dnxt;
    }
}

// Ring cell (hlx, hly) of thread t in the psi tile of a wx x wy tile: the rows below and above
// (wx + 2 cells each, corners included), then the left and right columns (wy cells each).
__device__ __forceinline__ void ring_cell(int t, int wx, int wy, int& hlx, int& hly)
{
    if (t < wx + 2) {
        hlx = t; hly = 0;
    } else if (t < 2 * (wx + 2)) {
        hlx = t - (wx + 2); hly = wy + 1;
    } else if (t < 2 * (wx + 2) + wy) {
        hlx = 0; hly = 1 + t - 2 * (wx + 2);
    } else {
        hlx = wx + 1; hly = 1 + t - 2 * (wx + 2) - wy;
    }
}

// ------------------------------------------------------------------------------------------
// D3Q19: a block owns a TX x TY tile of an x-y plane and marches `planes` planes in z.
// ------------------------------------------------------------------------------------------
template <typename S, typename A, int TX, int TY, bool NT = false, bool EXT = false>
__global__ void __launch_bounds__(TX* TY) k_step3d(const S* __restrict__ src, S* __restrict__ dst,
                                                   StepArgs a, StepGrid grid)
{
    using L = lat<19>;
    __shared__ A ps[4][TY + 2][TX + 2];
    const Coef<A> c = coef_of(a, A());
    const int nx = a.nx, ny = a.ny, nz = a.nz;
    const int64_t N = a.N;
    const int lb = logical_block(grid);
    const int bx = lb % grid.gx;
    const int by = (lb / grid.gx) % grid.gy;
    const int bz = lb / (grid.gx * grid.gy);
    const int t = threadIdx.x;
    const int tx = t % TX, ty = t / TX;
    const int x0 = bx * TX, y0 = by * TY, z0 = bz * a.planes;
    const int wx = min(TX, nx - x0), wy = min(TY, ny - y0);
    const int ze = min(z0 + a.planes, nz);
    const bool own = tx < wx && ty < wy;
    const int x = x0 + (own ? tx : 0), y = y0 + (own ? ty : 0);
    const int xm = wrap_once(x - 1, nx), xp = wrap_once(x + 1, nx);
    const int ym = wrap_once(y - 1, ny), yp = wrap_once(y + 1, ny);

    // ring node of this thread (at most one: the host checks 2 (TX + 2) + 2 TY <= TX TY)
    const int nring = 2 * (wx + 2) + 2 * wy;
    const bool ring = t < nring;
    int hlx, hly;
    if (t < wx + 2) {
        hlx = t; hly = 0;
    } else if (t < 2 * (wx + 2)) {
        hlx = t - (wx + 2); hly = wy + 1;
    } else if (t < 2 * (wx + 2) + wy) {
        hlx = 0; hly = 1 + t - 2 * (wx + 2);
    } else {
        hlx = wx + 1; hly = 1 + t - 2 * (wx + 2) - wy;
    }
    const int hx = wrap_once(x0 - 1 + (ring ? hlx : 1), nx);
    const int hy = wrap_once(y0 - 1 + (ring ? hly : 1), ny);
    const int hxm = wrap_once(hx - 1, nx), hxp = wrap_once(hx + 1, nx);
    const int hym = wrap_once(hy - 1, ny), hyp = wrap_once(hy + 1, ny);

    float cur[19], nxt[19];
    A dcur = (A)0, dnxt = (A)0;

    {
        const int z = wrap_once(z0 - 1, nz);
        const int zm = wrap_once(z - 1, nz), zp = wrap_once(z + 1, nz);
        if (own) {
            float g[19];
            pull_node<19>(src, N, nx, ny, x, xm, xp, y, ym, yp, z, zm, zp, g);
            ps[0][ty + 1][tx + 1] = psi_f(c.rho_ref + sum_dev<19, A>(g));
        }
        if (ring) {
            float h[19];
            pull_node<19>(src, N, nx, ny, hx, hxm, hxp, hy, hym, hyp, z, zm, zp, h);
            ps[0][hly][hlx] = psi_f(c.rho_ref + sum_dev<19, A>(h));
        }
    }
    {
        const int z = z0;
        const int zm = wrap_once(z - 1, nz), zp = wrap_once(z + 1, nz);
        if (own) {
            pull_node<19>(src, N, nx, ny, x, xm, xp, y, ym, yp, z, zm, zp, cur);
            dcur = sum_dev<19, A>(cur);
            ps[1][ty + 1][tx + 1] = psi_f(c.rho_ref + dcur);
        }
        if (ring) {
            float h[19];
            pull_node<19>(src, N, nx, ny, hx, hxm, hxp, hy, hym, hyp, z, zm, zp, h);
            ps[1][hly][hlx] = psi_f(c.rho_ref + sum_dev<19, A>(h));
        }
    }

    // FP32 arithmetic: one plane per call, loading plane z+1 into `ld` and colliding plane z from
    // `co`; two calls per iteration with the arrays' roles swapped, so no plane is copied
    auto plane = [&](int z, float (&co)[19], float (&ld)[19], A& dco, A& dld) {
        const int s = (z - z0 + 1) & 3;
        const int sn = (s + 1) & 3, sp = (s + 3) & 3;
        {
            const int zn = wrap_once(z + 1, nz);
            const int zm = wrap_once(zn - 1, nz), zp = wrap_once(zn + 1, nz);
            if (own) {
                pull_node<19>(src, N, nx, ny, x, xm, xp, y, ym, yp, zn, zm, zp, ld);
                dld = sum_dev<19, A>(ld);
                ps[sn][ty + 1][tx + 1] = psi_f(c.rho_ref + dld);
            }
            if (ring) {
                float h[19];
                pull_node<19>(src, N, nx, ny, hx, hxm, hxp, hy, hym, hyp, zn, zm, zp, h);
                ps[sn][hly][hlx] = psi_f(c.rho_ref + sum_dev<19, A>(h));
            }
        }
        __syncthreads();
        if (own) {
            const A pc = ps[s][ty + 1][tx + 1];
            A fx, fy, fz;
            interaction_sum<19, A>(
                [&](int i) {
                    const int slot = L::ez[i] > 0 ? sn : (L::ez[i] < 0 ? sp : s);
                    return ps[slot][ty + 1 + L::ey[i]][tx + 1 + L::ex[i]];
                },
                fx, fy, fz);
            const A gp = -c.G * pc;
            collide_store<19, A, S, NT, EXT>(dst, N, (uint32_t)(x + nx * (y + ny * z)), co, dco,
                                            gp * fx, gp * fy, gp * fz, c);
        }
    };
    if constexpr (!std::is_same<A, double>::value) {
        for (int z = z0; z < ze; z += 2) {
            plane(z, cur, nxt, dcur, dnxt);
            if (z + 1 < ze) plane(z + 1, nxt, cur, dnxt, dcur);
        }
    } else {
    for (int z = z0; z < ze; ++z) {
        const int s = (z - z0 + 1) & 3;
        const int sn = (s + 1) & 3, sp = (s + 3) & 3;
        {
            // FP64 arithmetic fills the 128 VGPRs of a 1024-thread block, so the loop is shaped
            // for registers: every lane loads plane z+1 (a lane outside a ragged tile its clamped
            // in-box node, harmlessly) and the ring's loads and sum form one block, so both sets
            // of loads are in flight together and none is left pending past the sums (a pending
            // load would make the copy into cur wait for every store of the plane); coordinates
            // are derived from the thread index where they are used rather than held across
            // the loop (held, they spill, and each reload waits for all loads in flight)
            {
                const int zn = wrap_once(z + 1, nz);
                const int zm = wrap_once(zn - 1, nz), zp = wrap_once(zn + 1, nz);
                const int tt = opaque(t);
                const int ltx = tt % TX, lty = tt / TX;
                {
                    const int ox = x0 + min(ltx, wx - 1), oy = y0 + min(lty, wy - 1);
                    pull_node<19>(src, N, nx, ny, ox, wrap_once(ox - 1, nx),
                                  wrap_once(ox + 1, nx), oy, wrap_once(oy - 1, ny),
                                  wrap_once(oy + 1, ny), zn, zm, zp, nxt);
                }
                if (ring) {
                    int rlx, rly;
                    ring_cell(tt, wx, wy, rlx, rly);
                    const int ox = wrap_once(x0 - 1 + rlx, nx), oy = wrap_once(y0 - 1 + rly, ny);
                    float h[19];
                    pull_node<19>(src, N, nx, ny, ox, wrap_once(ox - 1, nx),
                                  wrap_once(ox + 1, nx), oy, wrap_once(oy - 1, ny),
                                  wrap_once(oy + 1, ny), zn, zm, zp, h);
                    ps[sn][rly][rlx] = psi_f(c.rho_ref + sum_dev<19, A>(h));
                }
                dnxt = sum_dev<19, A>(nxt);
                if (own) ps[sn][lty + 1][ltx + 1] = psi_f(c.rho_ref + dnxt);
            }
            __syncthreads();
            if (own) {
                const int tt = opaque(t);
                const int ltx = tt % TX, lty = tt / TX;
                const A pc = ps[s][lty + 1][ltx + 1];
                A fx, fy, fz;
                interaction_sum<19, A>(
                    [&](int i) {
                        const int slot = L::ez[i] > 0 ? sn : (L::ez[i] < 0 ? sp : s);
                        return ps[slot][lty + 1 + L::ey[i]][ltx + 1 + L::ex[i]];
                    },
                    fx, fy, fz);
                const A gp = -c.G * pc;
                const int ox = x0 + ltx, oy = y0 + lty;
                collide_store<19, A, S, NT, EXT, true>(dst, N, (uint32_t)(ox + nx * (oy + ny * z)),
                                                      cur, dcur, gp * fx, gp * fy, gp * fz, c);
            }
        }
#pragma unroll
        for (int i = 0; i < 19; ++i) cur[i] = nxt[i];
        dcur = dnxt;
    }
    }
}
// ------------------------------------------------------------------------------------------
// D3Q19, software-pipelined: the loads of plane z+2 are issued before plane z is collided, so a
// wave keeps a plane of loads in flight through its collision and stores.  Ring nodes go to the
// first threads of the block, as in k_step3d: a wave executes the ring's loads whether one lane
// or all 64 need them, so packing the ring into as few waves as possible keeps the instruction
// count down.  Iteration z reads psi slots of planes z-1, z, z+1 and writes plane z+2's slot
// after its collision; the one barrier at the end of the iteration separates writers from readers
// (plane z-2's slot, overwritten now, was last read before the previous barrier).  Stores are
// non-temporal.
// ------------------------------------------------------------------------------------------
template <typename S, typename A, int TX, int TY>
__global__ void __launch_bounds__(TX* TY) k_step3d_pipe(const S* __restrict__ src,
                                                        S* __restrict__ dst, StepArgs a,
                                                        StepGrid grid)
{
    using L = lat<19>;
    __shared__ A ps[4][TY + 2][TX + 2];
    const Coef<A> c = coef_of(a, A());
    const int nx = a.nx, ny = a.ny, nz = a.nz;
    const int64_t N = a.N;
    const int lb = logical_block(grid);
    const int bx = lb % grid.gx;
    const int by = (lb / grid.gx) % grid.gy;
    const int bz = lb / (grid.gx * grid.gy);
    const int t = threadIdx.x;
    const int tx = t % TX, ty = t / TX;
    const int x0 = bx * TX, y0 = by * TY, z0 = bz * a.planes;
    const int wx = min(TX, nx - x0), wy = min(TY, ny - y0);
    const int ze = min(z0 + a.planes, nz);
    const bool own = tx < wx && ty < wy;
    const int x = x0 + (own ? tx : 0), y = y0 + (own ? ty : 0);
    const int xm = wrap_once(x - 1, nx), xp = wrap_once(x + 1, nx);
    const int ym = wrap_once(y - 1, ny), yp = wrap_once(y + 1, ny);

    const int nring = 2 * (wx + 2) + 2 * wy;
    const int r = t;
    const bool ring = r < nring;
    int hlx, hly;
    if (r < wx + 2) {
        hlx = r; hly = 0;
    } else if (r < 2 * (wx + 2)) {
        hlx = r - (wx + 2); hly = wy + 1;
    } else if (r < 2 * (wx + 2) + wy) {
        hlx = 0; hly = 1 + r - 2 * (wx + 2);
    } else {
        hlx = wx + 1; hly = 1 + r - 2 * (wx + 2) - wy;
    }
    const int hx = wrap_once(x0 - 1 + (ring ? hlx : 1), nx);
    const int hy = wrap_once(y0 - 1 + (ring ? hly : 1), ny);
    const int hxm = wrap_once(hx - 1, nx), hxp = wrap_once(hx + 1, nx);
    const int hym = wrap_once(hy - 1, ny), hyp = wrap_once(hy + 1, ny);

    float cur[19], nxt[19], pre[19], hpre[19];
    A dcur = (A)0, dnxt = (A)0, dpre = (A)0;

    // planes z0-1 (psi), z0 (psi + cur), z0+1 (psi + nxt)
#pragma unroll 1
    for (int k = 0; k < 3; ++k) {
        const int z = wrap_once(z0 - 1 + k, nz);
        const int zm = wrap_once(z - 1, nz), zp = wrap_once(z + 1, nz);
        if (own) {
            pull_node<19>(src, N, nx, ny, x, xm, xp, y, ym, yp, z, zm, zp, pre);
            const A d = sum_dev<19, A>(pre);
            ps[k][ty + 1][tx + 1] = psi_f(c.rho_ref + d);
            if (k == 1) {
#pragma unroll
                for (int i = 0; i < 19; ++i) cur[i] = pre[i];
                dcur = d;
            } else if (k == 2) {
#pragma unroll
                for (int i = 0; i < 19; ++i) nxt[i] = pre[i];
                dnxt = d;
            }
        }
        if (ring) {
            pull_node<19>(src, N, nx, ny, hx, hxm, hxp, hy, hym, hyp, z, zm, zp, hpre);
            ps[k][hly][hlx] = psi_f(c.rho_ref + sum_dev<19, A>(hpre));
        }
    }
    __syncthreads();

    // one plane per call: plane z+2's loads into `pf`, plane z collided from `co`, plane z+1
    // waiting in `nx1`; three calls per iteration with the arrays' roles rotated, so no plane
    // is copied
    auto plane = [&](int z, float (&co)[19], float (&pf)[19], A& dco, A& dpf) {
        const int s = (z - z0 + 1) & 3;
        const int sn = (s + 1) & 3, sp = (s + 3) & 3, s2 = (s + 2) & 3;
        const bool more = z + 1 < ze;  // plane z+2 is needed by the collision of plane z+1
        if (more) {
            const int z2 = wrap_once(z + 2 >= nz ? z + 2 - nz : z + 2, nz);
            const int zm = wrap_once(z2 - 1, nz), zp = wrap_once(z2 + 1, nz);
            if (own) pull_node<19>(src, N, nx, ny, x, xm, xp, y, ym, yp, z2, zm, zp, pf);
            if (ring) pull_node<19>(src, N, nx, ny, hx, hxm, hxp, hy, hym, hyp, z2, zm, zp, hpre);
        }
        if (own) {
            const A pc = ps[s][ty + 1][tx + 1];
            A fx, fy, fz;
            interaction_sum<19, A>(
                [&](int i) {
                    const int slot = L::ez[i] > 0 ? sn : (L::ez[i] < 0 ? sp : s);
                    return ps[slot][ty + 1 + L::ey[i]][tx + 1 + L::ex[i]];
                },
                fx, fy, fz);
            const A gp = -c.G * pc;
            collide_store<19, A, S, true>(dst, N, (uint32_t)(x + nx * (y + ny * z)), co, dco,
                                          gp * fx, gp * fy, gp * fz, c);
        }
        if (more) {
            if (own) {
                dpf = sum_dev<19, A>(pf);
                ps[s2][ty + 1][tx + 1] = psi_f(c.rho_ref + dpf);
            }
            if (ring) ps[s2][hly][hlx] = psi_f(c.rho_ref + sum_dev<19, A>(hpre));
        }
        __syncthreads();
    };
    for (int z = z0; z < ze; z += 3) {
        plane(z, cur, pre, dcur, dpre);
        if (z + 1 < ze) plane(z + 1, nxt, cur, dnxt, dcur);
        if (z + 2 < ze) plane(z + 2, pre, nxt, dpre, dnxt);
    }
}

// ------------------------------------------------------------------------------------------
// Barrier fix-up (modified Shan-Chen, Sec. 3.1): after the marching kernel has stepped every
// node with the plain force, the frontier nodes -- owned nodes next to a node of another,
// un-merged bubble, listed by the test pass -- are stepped again from the same source with the
// neighbours of that other bubble seen as bulk liquid, psi(rho_l), and overwrite their outputs.
// Same operations in the same order as the marching kernel, so only the substitution differs,
// and the result does not depend on the marching kernel's tile.
// ------------------------------------------------------------------------------------------
template <int Q, typename S, typename A, bool EXT>
__global__ void __launch_bounds__(256) k_barrier_fix(const S* __restrict__ src,
                                                     S* __restrict__ dst, StepArgs a,
                                                     const uint32_t* __restrict__ list, int count)
{
    using L = lat<Q>;
    const Coef<A> c = coef_of(a, A());
    const int nx = a.nx, ny = a.ny, nz = a.nz;
    const int64_t N = a.N;
    const uint16_t* __restrict__ ownr = a.owner;
    auto pull = [&](int x, int y, int z, float* g) {
        pull_node<Q>(src, N, nx, ny, x, wrap_once(x - 1, nx), wrap_once(x + 1, nx), y,
                     wrap_once(y - 1, ny), wrap_once(y + 1, ny), z,
                     Q == 19 ? wrap_once(z - 1, nz) : 0, Q == 19 ? wrap_once(z + 1, nz) : 0, g);
    };
    for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < count; k += gridDim.x * blockDim.x) {
        const uint32_t n = list[k];
        const int x = (int)(n % (uint32_t)nx);
        const uint32_t r = n / (uint32_t)nx;
        const int y = (int)(r % (uint32_t)ny), z = (int)(r / (uint32_t)ny);
        float g[Q];
        pull(x, y, z, g);
        const A drho = sum_dev<Q, A>(g);
        const A pc = psi_f(c.rho_ref + drho);
        const uint16_t o = ownr[n];
        A fx, fy, fz;
        interaction_sum<Q, A>(
            [&](int i) -> A {
                const int xx = wrap_once(x + L::ex[i], nx), yy = wrap_once(y + L::ey[i], ny);
                const int zz = Q == 19 ? wrap_once(z + L::ez[i], nz) : 0;
                const uint16_t on = ownr[xx + (int64_t)nx * (yy + (int64_t)ny * zz)];
                if (o != 0 && on != 0 && on != o) return c.psi_l;  // another bubble's lattice
                float h[Q];
                pull(xx, yy, zz, h);
                return psi_f(c.rho_ref + sum_dev<Q, A>(h));
            },
            fx, fy, fz);
        const A gp = -c.G * pc;
        collide_store<Q, A, S, false, EXT>(dst, N, n, g, drho, gp * fx, gp * fy,
                                           Q == 19 ? gp * fz : (A)0, c);
    }
}

hipError_t launch_barrier_fix(int q, int storage, int compute, const void* src, void* dst,
                              const StepArgs& a, const uint32_t* list, int count, hipStream_t st)
{
    if (count <= 0) return hipSuccess;
    if (!a.owner) return hipErrorInvalidValue;
    const dim3 grid((unsigned)std::min(65535, (count + 255) / 256)), block(256);
    const bool g = a.grav != 0;
    if (storage != SC_STORE_F32) {
        // 16-bit storage: FP32 arithmetic
        if (compute == SC_COMPUTE_F64) return hipErrorInvalidValue;
#define SC_FIX16(QQ, SS)                                                                         \
    do {                                                                                         \
        if (g)                                                                                   \
            hipLaunchKernelGGL((k_barrier_fix<QQ, SS, float, true>), grid, block, 0, st,         \
                               (const SS*)src, (SS*)dst, a, list, count);                        \
        else                                                                                     \
            hipLaunchKernelGGL((k_barrier_fix<QQ, SS, float, false>), grid, block, 0, st,        \
                               (const SS*)src, (SS*)dst, a, list, count);                        \
    } while (0)
        if (storage == SC_STORE_F16) {
            if (q == 9) SC_FIX16(9, _Float16); else SC_FIX16(19, _Float16);
        } else if (storage == SC_STORE_BF16) {
            if (q == 9) SC_FIX16(9, __bf16); else SC_FIX16(19, __bf16);
        } else {
            return hipErrorInvalidValue;
        }
#undef SC_FIX16
        return hipGetLastError();
    }
    const float* s = (const float*)src;
    float* d = (float*)dst;
#define SC_FIX(QQ, AA, EE) \
    hipLaunchKernelGGL((k_barrier_fix<QQ, float, AA, EE>), grid, block, 0, st, s, d, a, list, count)
    if (compute == SC_COMPUTE_F64) {
        if (q == 9) { if (g) SC_FIX(9, double, true); else SC_FIX(9, double, false); }
        else { if (g) SC_FIX(19, double, true); else SC_FIX(19, double, false); }
    } else {
        if (q == 9) { if (g) SC_FIX(9, float, true); else SC_FIX(9, float, false); }
        else { if (g) SC_FIX(19, float, true); else SC_FIX(19, float, false); }
    }
#undef SC_FIX
    return hipGetLastError();
}

// ------------------------------------------------------------------------------------------
// Launch
// ------------------------------------------------------------------------------------------
bool step_shape_supported(int q, const StepShape& s)
{
    if (s.tile_z < 1) return false;
    if (s.variant < 1 || s.variant > 3 || (q == 9 && s.variant == 2)) return false;
    if (q == 9) return s.tile_y == 1 && (s.tile_x == 64 || s.tile_x == 128 || s.tile_x == 256 ||
                                          s.tile_x == 512);
    if (q == 19) {
        const int tx = s.tile_x, ty = s.tile_y;
        const bool known = (tx == 32 && (ty == 4 || ty == 8 || ty == 16)) ||
                           (tx == 64 && (ty == 4 || ty == 8)) ||
                           (tx == 128 && (ty == 4 || ty == 8)) ||
                           (tx == 256 && ty == 4) || (tx == 16 && ty == 16);
        return known && 2 * (tx + 2) + 2 * ty <= tx * ty;
    }
    return false;
}

template <typename S, typename A>
static hipError_t step_typed(int q, const S* src, S* dst, const StepArgs& a, const StepShape& s,
                             hipStream_t st)
{
    StepGrid g;
    if (q == 9) {
        g.gx = (a.nx + s.tile_x - 1) / s.tile_x;
        g.gy = (a.ny + a.planes - 1) / a.planes;
        g.gz = 1;
    } else {
        g.gx = (a.nx + s.tile_x - 1) / s.tile_x;
        g.gy = (a.ny + s.tile_y - 1) / s.tile_y;
        g.gz = (a.nz + a.planes - 1) / a.planes;
    }
    const int nb = g.gx * g.gy * g.gz;
    g.remap = (nb % 8 == 0) ? 1 : 0;
    dim3 grid(nb);
    // the extended kernels (gravity) exist for the marching variants only
    const bool ext = a.grav != 0;
    if (ext && s.variant == 2) return hipErrorInvalidValue;
#define SC_L2(TX)                                                                                \
    if (s.tile_x == TX) {                                                                        \
        if (ext) {                                                                               \
            if (s.variant == 3)                                                                  \
                hipLaunchKernelGGL((k_step2d<S, A, TX, true, true>), grid, dim3(TX), 0, st,      \
                                   src, dst, a, g);                                              \
            else                                                                                 \
                hipLaunchKernelGGL((k_step2d<S, A, TX, false, true>), grid, dim3(TX), 0, st,     \
                                   src, dst, a, g);                                              \
            return hipGetLastError();                                                            \
        }                                                                                        \
        if (s.variant == 3)                                                                      \
            hipLaunchKernelGGL((k_step2d<S, A, TX, true>), grid, dim3(TX), 0, st, src, dst, a,   \
                               g);                                                               \
        else                                                                                     \
            hipLaunchKernelGGL((k_step2d<S, A, TX>), grid, dim3(TX), 0, st, src, dst, a, g);     \
        return hipGetLastError();                                                                \
    }
#define SC_L3(TX, TY)                                                                            \
    if (s.tile_x == TX && s.tile_y == TY) {                                                      \
        if (ext) {                                                                               \
            if (s.variant == 3)                                                                  \
                hipLaunchKernelGGL((k_step3d<S, A, TX, TY, true, true>), grid,                   \
                                   dim3(TX * TY), 0, st, src, dst, a, g);                        \
            else                                                                                 \
                hipLaunchKernelGGL((k_step3d<S, A, TX, TY, false, true>), grid,                  \
                                   dim3(TX * TY), 0, st, src, dst, a, g);                        \
            return hipGetLastError();                                                            \
        }                                                                                        \
        if (s.variant == 2)                                                                      \
            hipLaunchKernelGGL((k_step3d_pipe<S, A, TX, TY>), grid, dim3(TX * TY), 0, st, src,   \
                               dst, a, g);                                                       \
        else if (s.variant == 3)                                                                 \
            hipLaunchKernelGGL((k_step3d<S, A, TX, TY, true>), grid, dim3(TX * TY), 0, st, src,  \
                               dst, a, g);                                                       \
        else                                                                                     \
            hipLaunchKernelGGL((k_step3d<S, A, TX, TY>), grid, dim3(TX * TY), 0, st, src, dst,   \
                               a, g);                                                            \
        return hipGetLastError();                                                                \
    }
    if (q == 9) {
        SC_L2(64) SC_L2(128) SC_L2(256) SC_L2(512)
    } else {
        SC_L3(32, 4) SC_L3(32, 8) SC_L3(32, 16) SC_L3(64, 4) SC_L3(64, 8) SC_L3(128, 4)
        SC_L3(16, 16) SC_L3(128, 8) SC_L3(256, 4)
    }
#undef SC_L2
#undef SC_L3
    return hipErrorInvalidValue;
}

bool step_combo_supported(int storage, int compute)
{
    if (compute == SC_COMPUTE_F32) return storage >= SC_STORE_F32 && storage <= SC_STORE_BF16;
    if (compute == SC_COMPUTE_F64) return storage == SC_STORE_F32;
    return false;
}

hipError_t launch_step(int q, int storage, int compute, const void* src, void* dst,
                       const StepArgs& a, const StepShape& s, hipStream_t st)
{
    if (!step_shape_supported(q, s)) return hipErrorInvalidValue;
    if (compute == SC_COMPUTE_F64) {
        if (storage == SC_STORE_F32)
            return step_typed<float, double>(q, (const float*)src, (float*)dst, a, s, st);
        return hipErrorInvalidValue;
    }
    switch (storage) {
        case SC_STORE_F32:
            return step_typed<float, float>(q, (const float*)src, (float*)dst, a, s, st);
        case SC_STORE_F16:
            return step_typed<_Float16, float>(q, (const _Float16*)src, (_Float16*)dst, a, s, st);
        case SC_STORE_BF16:
            return step_typed<__bf16, float>(q, (const __bf16*)src, (__bf16*)dst, a, s, st);
    }
    return hipErrorInvalidValue;
}

// ------------------------------------------------------------------------------------------
// State kernels: initial fill, nucleus painting, equilibrium from fields, population export.
// ------------------------------------------------------------------------------------------
template <int Q>
__device__ __forceinline__ int64_t upstream_of(int x, int y, int z, int i, const InitArgs& a)
{
    // storage slot of f_i(x): the node x - e_i
    using L = lat<Q>;
    const int sx = wrap_once(x - L::ex[i], a.nx);
    const int sy = wrap_once(y - L::ey[i], a.ny);
    const int sz = wrap_once(z - L::ez[i], a.nz);
    return (int64_t)sx + (int64_t)a.nx * ((int64_t)sy + (int64_t)a.ny * sz);
}

__device__ __forceinline__ void coords_of(int64_t n, const InitArgs& a, int& x, int& y, int& z)
{
    x = (int)(n % a.nx);
    const int64_t r = n / a.nx;
    y = (int)(r % a.ny);
    z = (int)(r / a.ny);
}

template <int Q, typename S>
__device__ __forceinline__ void write_rest(S* f, int64_t N, int x, int y, int z, double rho,
                                           const InitArgs& a)
{
    using L = lat<Q>;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        const double g = L::wd[i] * (rho - a.rho_ref);
        f[(int64_t)i * N + upstream_of<Q>(x, y, z, i, a)] = store_f<S>((float)g);
    }
}

template <int Q, typename S>
__global__ void k_init(S* f, InitArgs a)
{
    for (int64_t n = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; n < a.N;
         n += (int64_t)gridDim.x * blockDim.x) {
        int x, y, z;
        coords_of(n, a, x, y, z);
        const double rho = a.rho + a.amp * (2.0 * unit_noise(a.seed, n) - 1.0);
        write_rest<Q, S>(f, a.N, x, y, z, rho, a);
    }
}

template <int Q, typename S>
__global__ void k_paint(S* f, InitArgs a, double cx, double cy, double cz, double R, int bx0,
                        int by0, int bz0, int ex, int ey, int ez)
{
#pragma clang fp contract(off)
    const int64_t tot = (int64_t)ex * ey * ez;
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < tot;
         k += (int64_t)gridDim.x * blockDim.x) {
        const int ox = (int)(k % ex);
        const int oy = (int)((k / ex) % ey);
        const int oz = (int)(k / ((int64_t)ex * ey));
        int x = (bx0 + ox) % a.nx; if (x < 0) x += a.nx;
        int y = (by0 + oy) % a.ny; if (y < 0) y += a.ny;
        int z = (bz0 + oz) % a.nz; if (z < 0) z += a.nz;
        double dx = (double)x - cx, dy = (double)y - cy, dz = (double)z - cz;
        dx = dx - a.nx * floor(dx / a.nx + 0.5);
        dy = dy - a.ny * floor(dy / a.ny + 0.5);
        dz = (lat<Q>::d == 3) ? dz - a.nz * floor(dz / a.nz + 0.5) : 0.0;
        if (dx * dx + dy * dy + dz * dz <= R * R) {
            const int64_t n = (int64_t)x + (int64_t)a.nx * ((int64_t)y + (int64_t)a.ny * z);
            const double rho = a.rho + a.amp * (2.0 * unit_noise(a.seed, n) - 1.0);
            write_rest<Q, S>(f, a.N, x, y, z, rho, a);
        }
    }
}

template <int Q, typename S>
__global__ void k_set_eq(S* f, InitArgs a, const double* rho_d, const double* u_d)
{
    using L = lat<Q>;
    for (int64_t n = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; n < a.N;
         n += (int64_t)gridDim.x * blockDim.x) {
        int x, y, z;
        coords_of(n, a, x, y, z);
        const double rho = rho_d[n];
        double u[3] = {0.0, 0.0, 0.0};
        if (u_d)
            for (int c = 0; c < L::d; ++c) u[c] = u_d[(int64_t)c * a.N + n];
        const double usq = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            const double eu = L::ex[i] * u[0] + L::ey[i] * u[1] + L::ez[i] * u[2];
            const double feq = L::wd[i] * rho * (1.0 + 3.0 * eu + 4.5 * eu * eu - 1.5 * usq);
            f[(int64_t)i * a.N + upstream_of<Q>(x, y, z, i, a)] =
                store_f<S>((float)(feq - L::wd[i] * a.rho_ref));
        }
    }
}

template <int Q, typename S>
__global__ void k_get_f(const S* f, double* out, InitArgs a)
{
    using L = lat<Q>;
    for (int64_t n = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; n < a.N;
         n += (int64_t)gridDim.x * blockDim.x) {
        int x, y, z;
        coords_of(n, a, x, y, z);
#pragma unroll
        for (int i = 0; i < Q; ++i)
            out[(int64_t)i * a.N + n] =
                (double)load_f(f[(int64_t)i * a.N + upstream_of<Q>(x, y, z, i, a)]) +
                L::wd[i] * a.rho_ref;
    }
}

template <int Q, typename S>
__global__ void k_set_f(S* f, const double* in, InitArgs a)
{
    using L = lat<Q>;
    for (int64_t n = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; n < a.N;
         n += (int64_t)gridDim.x * blockDim.x) {
        int x, y, z;
        coords_of(n, a, x, y, z);
#pragma unroll
        for (int i = 0; i < Q; ++i)
            f[(int64_t)i * a.N + upstream_of<Q>(x, y, z, i, a)] =
                store_f<S>((float)(in[(int64_t)i * a.N + n] - L::wd[i] * a.rho_ref));
    }
}

static dim3 grid_for(int64_t n)
{
    int64_t b = (n + 255) / 256;
    if (b > 65536) b = 65536;
    if (b < 1) b = 1;
    return dim3((unsigned)b);
}

#define SC_DISPATCH(q, storage, CALL)                                                             \
    do {                                                                                          \
        if (q == 9 && storage == SC_STORE_F32) { constexpr int QQ = 9; using SS = float; CALL; }  \
        else if (q == 9 && storage == SC_STORE_F16) { constexpr int QQ = 9; using SS = _Float16; CALL; } \
        else if (q == 9 && storage == SC_STORE_BF16) { constexpr int QQ = 9; using SS = __bf16; CALL; } \
        else if (q == 19 && storage == SC_STORE_F32) { constexpr int QQ = 19; using SS = float; CALL; } \
        else if (q == 19 && storage == SC_STORE_F16) { constexpr int QQ = 19; using SS = _Float16; CALL; } \
        else if (q == 19 && storage == SC_STORE_BF16) { constexpr int QQ = 19; using SS = __bf16; CALL; } \
        else return hipErrorInvalidValue;                                                         \
    } while (0)

hipError_t launch_init(int q, int storage, void* f, const InitArgs& a, hipStream_t st)
{
    SC_DISPATCH(q, storage,
                hipLaunchKernelGGL((k_init<QQ, SS>), grid_for(a.N), dim3(256), 0, st, (SS*)f, a));
    return hipGetLastError();
}

hipError_t launch_paint(int q, int storage, void* f, const InitArgs& a, const double c[3],
                        double R, hipStream_t st)
{
    if (!(R >= 0.0)) return hipSuccess;
    const int r = (int)ceil(R) + 1;
    const int bx0 = (int)floor(c[0]) - r, by0 = (int)floor(c[1]) - r;
    const int ex = 2 * r + 2, ey = 2 * r + 2;
    int bz0 = 0, ez = 1;
    if (q == 19) {
        bz0 = (int)floor(c[2]) - r;
        ez = 2 * r + 2;
    }
    const int64_t tot = (int64_t)ex * ey * ez;
    SC_DISPATCH(q, storage,
                hipLaunchKernelGGL((k_paint<QQ, SS>), grid_for(tot), dim3(256), 0, st, (SS*)f, a,
                                   c[0], c[1], q == 19 ? c[2] : 0.0, R, bx0, by0, bz0, ex, ey,
                                   ez));
    return hipGetLastError();
}

hipError_t launch_set_eq(int q, int storage, void* f, const InitArgs& a, const double* rho_d,
                         const double* u_d, hipStream_t st)
{
    SC_DISPATCH(q, storage,
                hipLaunchKernelGGL((k_set_eq<QQ, SS>), grid_for(a.N), dim3(256), 0, st, (SS*)f,
                                   a, rho_d, u_d));
    return hipGetLastError();
}

hipError_t launch_get_f(int q, int storage, const void* f, double* out_d, const InitArgs& a,
                        hipStream_t st)
{
    SC_DISPATCH(q, storage,
                hipLaunchKernelGGL((k_get_f<QQ, SS>), grid_for(a.N), dim3(256), 0, st,
                                   (const SS*)f, out_d, a));
    return hipGetLastError();
}

hipError_t launch_set_f(int q, int storage, void* f, const double* in_d, const InitArgs& a,
                        hipStream_t st)
{
    SC_DISPATCH(q, storage,
                hipLaunchKernelGGL((k_set_f<QQ, SS>), grid_for(a.N), dim3(256), 0, st, (SS*)f,
                                   in_d, a));
    return hipGetLastError();
}

}  // namespace sc
