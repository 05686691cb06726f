// sc_step2c.hip -- the two-component step (liquid l, gas v) and the mixture's reported fields.
//
// Shan-Doolen mixture with psi = rho (the liquid and the gas component run side by side on one
// lattice, Sec. 3 and 3.1): the force on component a is F_a = -Gx rho_a(x) sum_i w_i rho_b(x+e_i)
// e_i (b the other component); both relax to equilibria at the common velocity
//   u' = sum_a (j_a / tau_a) / sum_a (rho_a / tau_a),  u_a^eq = u' + tau_a F_a / rho_a,
// then stream.  Storage: FP32 populations with FP64 arithmetic (unshifted unless rho_ref is
// set), or FP16 / BF16 populations with FP32 arithmetic; shifted storage holds f_i - w_i rho_ref
// per component (the liquid's rho_ref, the gas component's dissolved density).  Densities travel as deviations from the shift: the
// interaction sums need only differences (sum_i w_i e_i = 0), and the shift is added back where
// the density itself enters.
//
// One fused kernel per step, built like the one-component marching kernels: a block owns a tile
// of one plane (a row segment in 2D, an x-y tile in 3D) and marches along the remaining axis.
// The densities of both components over the tile and its one-node ring, for three planes, live
// in LDS (in the arithmetic type); the tile's own populations of both components stay in
// registers from their load until the collision one plane later.  Each plane of both components
// is read once and written once: 2 x 2 Q x sizeof(storage) bytes per node and step.
#include <algorithm>

#include "sc_device.hpp"
#include "sc_internal.hpp"
#include "sc_stepcore.hpp"

namespace sc {

namespace {

// Momentum j = sum_i g_i e_i of one component from its stored values (the shift w_i rho_ref
// drops out: sum_i w_i e_i = 0).
template <int Q, typename A>
__device__ __forceinline__ void momentum(const float* g, A& jx, A& jy, A& jz)
{
    using L = lat<Q>;
    jx = jy = jz = (A)0;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        if (L::ex[i] > 0) jx += (A)g[i]; else if (L::ex[i] < 0) jx -= (A)g[i];
        if (L::ey[i] > 0) jy += (A)g[i]; else if (L::ey[i] < 0) jy -= (A)g[i];
        if (L::ez[i] > 0) jz += (A)g[i]; else if (L::ez[i] < 0) jz -= (A)g[i];
    }
}

template <typename A>
struct MixCoef {
    A tau_l, tau_v, il, iv, Gx;  // il = 1 / tau_l, iv = 1 / tau_v
    A ref_l, ref_v;              // storage shifts of the liquid and the gas component
};

template <typename A>
__device__ __forceinline__ MixCoef<A> mix_coef(const Step2cArgs& a)
{
    return MixCoef<A>{(A)a.tau_l, (A)a.tau_v, (A)(1.0 / a.tau_l), (A)(1.0 / a.tau_v), (A)a.Gx,
                      (A)a.ref_l, (A)a.ref_v};
}

// Collision of both components of one node and the stores.  drl, drv are the density
// deviations from the storage shifts; (sl*) is the interaction sum over the gas density seen by
// the liquid, (sv*) the one over the liquid density seen by the gas.
template <int Q, typename S, typename A, bool NT>
__device__ __forceinline__ void mix_collide(S* __restrict__ dl, S* __restrict__ dv, int64_t N,
                                            uint32_t lane, const float* gl, const float* gv,
                                            A drl, A drv, A slx, A sly, A slz, A svx, A svy,
                                            A svz, const MixCoef<A>& c)
{
    A jlx, jly, jlz, jvx, jvy, jvz;
    momentum<Q, A>(gl, jlx, jly, jlz);
    momentum<Q, A>(gv, jvx, jvy, jvz);
    const A rl = c.ref_l + drl, rv = c.ref_v + drv;
    const A iden = recip(fmad(rl, c.il, rv * c.iv));
    const A upx = fmad(jlx, c.il, jvx * c.iv) * iden;
    const A upy = fmad(jly, c.il, jvy * c.iv) * iden;
    const A upz = fmad(jlz, c.il, jvz * c.iv) * iden;
    // tau_a F_a / rho_a = -tau_a Gx (sum over the other component): rho_a cancels
    const A kl = -c.tau_l * c.Gx, kv = -c.tau_v * c.Gx;
    relax_store<Q, A, S, NT>(dl, N, lane, gl, drl, rl, fmad(kl, slx, upx), fmad(kl, sly, upy),
                             fmad(kl, slz, upz), c.il);
    relax_store<Q, A, S, NT>(dv, N, lane, gv, drv, rv, fmad(kv, svx, upx), fmad(kv, svy, upy),
                             fmad(kv, svz, upz), c.iv);
}

// ------------------------------------------------------------------------------------------
// D2Q9: a block owns TX nodes of a row and marches `planes` rows in y.
// ------------------------------------------------------------------------------------------
template <typename S, typename A, int TX, bool NT>
__global__ void __launch_bounds__(TX) k_mix2d(const S* __restrict__ sl, const S* __restrict__ sv,
                                              S* __restrict__ dl, S* __restrict__ dv,
                                              Step2cArgs a, StepGrid grid)
{
    using L = lat<9>;
    __shared__ A rls[4][TX + 2], rvs[4][TX + 2];  // density deviations
    const MixCoef<A> c = mix_coef<A>(a);
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
    const bool ring = tx < 2;  // ring nodes x0 - 1 (thread 0) and x0 + wx (thread 1)
    const int hx = tx == 0 ? wrap_once(x0 - 1, nx) : wrap_once(x0 + wx, nx);
    const int hxm = wrap_once(hx - 1, nx), hxp = wrap_once(hx + 1, nx);
    const int hl = tx == 0 ? 0 : wx + 1;

    float cl[9], cv[9], nl[9], nv[9];
    A rcl = (A)0, rcv = (A)0, rnl = (A)0, rnv = (A)0;

    // densities of row y into slot k; the tile's own populations into (gl, gv)
    auto load_row = [&](int y, int k, float* gl, float* gv, A& dl_, A& dv_) {
        const int ym = wrap_once(y - 1, ny), yp = wrap_once(y + 1, ny);
        if (own) {
            pull_node<9>(sl, N, nx, ny, x, xm, xp, y, ym, yp, 0, 0, 0, gl);
            pull_node<9>(sv, N, nx, ny, x, xm, xp, y, ym, yp, 0, 0, 0, gv);
            dl_ = sum_dev<9, A>(gl);
            dv_ = sum_dev<9, A>(gv);
            rls[k][tx + 1] = dl_;
            rvs[k][tx + 1] = dv_;
        }
        if (ring) {
            float h[9];
            pull_node<9>(sl, N, nx, ny, hx, hxm, hxp, y, ym, yp, 0, 0, 0, h);
            rls[k][hl] = sum_dev<9, A>(h);
            pull_node<9>(sv, N, nx, ny, hx, hxm, hxp, y, ym, yp, 0, 0, 0, h);
            rvs[k][hl] = sum_dev<9, A>(h);
        }
    };
    {
        float tl[9], tv[9];
        A el, ev;
        load_row(wrap_once(y0 - 1, ny), 0, tl, tv, el, ev);
    }
    load_row(y0, 1, cl, cv, rcl, rcv);

    for (int y = y0; y < ye; ++y) {
        const int s = (y - y0 + 1) & 3;
        const int sn = (s + 1) & 3, sp = (s + 3) & 3;
        load_row(wrap_once(y + 1, ny), sn, nl, nv, rnl, rnv);
        __syncthreads();
        if (own) {
            A slx, sly, slz, svx, svy, svz;
            auto slot = [&](int i) { return L::ey[i] > 0 ? sn : (L::ey[i] < 0 ? sp : s); };
            interaction_sum<9, A>([&](int i) { return rvs[slot(i)][tx + 1 + L::ex[i]]; }, slx,
                                  sly, slz);
            interaction_sum<9, A>([&](int i) { return rls[slot(i)][tx + 1 + L::ex[i]]; }, svx,
                                  svy, svz);
            mix_collide<9, S, A, NT>(dl, dv, N, (uint32_t)(x + nx * y), cl, cv, rcl, rcv, slx,
                                     sly, (A)0, svx, svy, (A)0, c);
        }
#pragma unroll
        for (int i = 0; i < 9; ++i) {
            cl[i] = nl[i];
            cv[i] = nv[i];
        }
        rcl = rnl;
        rcv = rnv;
    }
}

// ------------------------------------------------------------------------------------------
// D3Q19: a block owns a TX x TY tile of an x-y plane and marches `planes` planes in z.
// ------------------------------------------------------------------------------------------
template <typename S, typename A, int TX, int TY, bool NT>
__global__ void __launch_bounds__(TX* TY) k_mix3d(const S* __restrict__ sl,
                                                  const S* __restrict__ sv, S* __restrict__ dl,
                                                  S* __restrict__ dv, Step2cArgs a,
                                                  StepGrid grid)
{
    using L = lat<19>;
    __shared__ A rls[4][TY + 2][TX + 2], rvs[4][TY + 2][TX + 2];  // density deviations
    const MixCoef<A> c = mix_coef<A>(a);
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

    float cl[19], cv[19], nl[19], nv[19];
    A rcl = (A)0, rcv = (A)0, rnl = (A)0, rnv = (A)0;

    auto load_plane = [&](int z, int k, float* gl, float* gv, A& dl_, A& dv_) {
        const int zm = wrap_once(z - 1, nz), zp = wrap_once(z + 1, nz);
        if (own) {
            pull_node<19>(sl, N, nx, ny, x, xm, xp, y, ym, yp, z, zm, zp, gl);
            pull_node<19>(sv, N, nx, ny, x, xm, xp, y, ym, yp, z, zm, zp, gv);
            dl_ = sum_dev<19, A>(gl);
            dv_ = sum_dev<19, A>(gv);
            rls[k][ty + 1][tx + 1] = dl_;
            rvs[k][ty + 1][tx + 1] = dv_;
        }
        if (ring) {
            float h[19];
            pull_node<19>(sl, N, nx, ny, hx, hxm, hxp, hy, hym, hyp, z, zm, zp, h);
            rls[k][hly][hlx] = sum_dev<19, A>(h);
            pull_node<19>(sv, N, nx, ny, hx, hxm, hxp, hy, hym, hyp, z, zm, zp, h);
            rvs[k][hly][hlx] = sum_dev<19, A>(h);
        }
    };
    {
        float tl[19], tv[19];
        A el, ev;
        load_plane(wrap_once(z0 - 1, nz), 0, tl, tv, el, ev);
    }
    load_plane(z0, 1, cl, cv, rcl, rcv);

    for (int z = z0; z < ze; ++z) {
        const int s = (z - z0 + 1) & 3;
        const int sn = (s + 1) & 3, sp = (s + 3) & 3;
        load_plane(wrap_once(z + 1, nz), sn, nl, nv, rnl, rnv);
        __syncthreads();
        if (own) {
            A slx, sly, slz, svx, svy, svz;
            auto slot = [&](int i) { return L::ez[i] > 0 ? sn : (L::ez[i] < 0 ? sp : s); };
            interaction_sum<19, A>(
                [&](int i) { return rvs[slot(i)][ty + 1 + L::ey[i]][tx + 1 + L::ex[i]]; }, slx,
                sly, slz);
            interaction_sum<19, A>(
                [&](int i) { return rls[slot(i)][ty + 1 + L::ey[i]][tx + 1 + L::ex[i]]; }, svx,
                svy, svz);
            mix_collide<19, S, A, NT>(dl, dv, N, (uint32_t)(x + nx * (y + ny * z)), cl, cv, rcl,
                                      rcv, slx, sly, slz, svx, svy, svz, c);
        }
#pragma unroll
        for (int i = 0; i < 19; ++i) {
            cl[i] = nl[i];
            cv[i] = nv[i];
        }
        rcl = rnl;
        rcv = rnv;
    }
}

// ------------------------------------------------------------------------------------------
// D3Q19, one component per wave: threads [0, T) carry the liquid of the T = TX x TY tile nodes,
// threads [T, 2T) the gas, so each thread holds one component's populations (the register
// budget of the one-component kernel) and every wave reads and writes a single component
// through scalar bases.  Besides the density rings, the momenta of both components go to LDS at
// load time (three plane slots: plane z is read between the barriers of iterations z and z+1,
// plane z+3 is written only after the second of them); the collision reads its partner's
// density and momentum there.
// ------------------------------------------------------------------------------------------
template <typename S, typename A, int TX, int TY, bool NT>
__global__ void __launch_bounds__(2 * TX* TY) k_mix3d_split(const S* __restrict__ sl,
                                                            const S* __restrict__ sv,
                                                            S* __restrict__ dl,
                                                            S* __restrict__ dv, Step2cArgs a,
                                                            StepGrid grid)
{
    using L = lat<19>;
    constexpr int T = TX * TY;
    __shared__ A rs[2][4][TY + 2][TX + 2];  // [component][plane slot][y][x] density deviations
    __shared__ A js[2][3][3][T];            // [component][plane slot][axis][node] momenta
    const int nx = a.nx, ny = a.ny, nz = a.nz;
    const int64_t N = a.N;
    const int lb = logical_block(grid);
    const int bx = lb % grid.gx;
    const int by = (lb / grid.gx) % grid.gy;
    const int bz = lb / (grid.gx * grid.gy);
    // component of this wave (T is a multiple of 64, so no wave straddles the two halves)
    const int comp = __builtin_amdgcn_readfirstlane((int)threadIdx.x >= T ? 1 : 0);
    const int oc = comp ^ 1;
    const int t = (int)threadIdx.x - comp * T;
    const S* __restrict__ src = comp ? sv : sl;
    S* __restrict__ dst = comp ? dv : dl;
    const A il = (A)(1.0 / a.tau_l), iv = (A)(1.0 / a.tau_v);
    const A ia = comp ? iv : il;
    const A ka = (A)(-(comp ? a.tau_v : a.tau_l) * a.Gx);  // tau_a F_a / rho_a = ka sum(rho_b)
    const A ref_l = (A)a.ref_l, ref_v = (A)a.ref_v, ref_a = comp ? ref_v : ref_l;
    const int tx = t % TX, ty = t / TX;
    const int x0 = bx * TX, y0 = by * TY, z0 = bz * a.planes;
    const int wx = min(TX, nx - x0), wy = min(TY, ny - y0);
    const int ze = min(z0 + a.planes, nz);
    const bool own = tx < wx && ty < wy;
    const int x = x0 + (own ? tx : 0), y = y0 + (own ? ty : 0);
    const int xm = wrap_once(x - 1, nx), xp = wrap_once(x + 1, nx);
    const int ym = wrap_once(y - 1, ny), yp = wrap_once(y + 1, ny);

    // ring node of this thread for its component (the host checks 2 (TX + 2) + 2 TY <= T)
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

    // plane z: density into ring slot k, momentum into slot k3 (k3 < 0: not needed)
    auto load_plane = [&](int z, int k, int k3, float* g) {
        const int zm = wrap_once(z - 1, nz), zp = wrap_once(z + 1, nz);
        if (own) {
            pull_node<19>(src, N, nx, ny, x, xm, xp, y, ym, yp, z, zm, zp, g);
            rs[comp][k][ty + 1][tx + 1] = sum_dev<19, A>(g);
            if (k3 >= 0) {
                A jx, jy, jz;
                momentum<19, A>(g, jx, jy, jz);
                js[comp][k3][0][t] = jx;
                js[comp][k3][1][t] = jy;
                js[comp][k3][2][t] = jz;
            }
        }
        if (ring) {
            float h[19];
            pull_node<19>(src, N, nx, ny, hx, hxm, hxp, hy, hym, hyp, z, zm, zp, h);
            rs[comp][k][hly][hlx] = sum_dev<19, A>(h);
        }
    };
    load_plane(wrap_once(z0 - 1, nz), 0, -1, nxt);
    load_plane(z0, 1, 0, cur);

    int s3 = 0;  // momentum slot of plane z
    for (int z = z0; z < ze; ++z) {
        const int s = (z - z0 + 1) & 3;
        const int sn = (s + 1) & 3, sp = (s + 3) & 3;
        const int n3 = s3 == 2 ? 0 : s3 + 1;
        load_plane(wrap_once(z + 1, nz), sn, n3, nxt);
        __syncthreads();
        if (own) {
            // both components in a fixed order (liquid first), so the two threads of a node
            // form the same common velocity
            const A da = rs[comp][s][ty + 1][tx + 1], db = rs[oc][s][ty + 1][tx + 1];
            const A rl = ref_l + (comp ? db : da), rv = ref_v + (comp ? da : db);
            A jl[3], jv[3];
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                jl[c] = js[0][s3][c][t];
                jv[c] = js[1][s3][c][t];
            }
            const A iden = recip(fmad(rl, il, rv * iv));
            const A upx = fmad(jl[0], il, jv[0] * iv) * iden;
            const A upy = fmad(jl[1], il, jv[1] * iv) * iden;
            const A upz = fmad(jl[2], il, jv[2] * iv) * iden;
            auto slot = [&](int i) { return L::ez[i] > 0 ? sn : (L::ez[i] < 0 ? sp : s); };
            A sx, sy, sz;
            interaction_sum<19, A>(
                [&](int i) { return rs[oc][slot(i)][ty + 1 + L::ey[i]][tx + 1 + L::ex[i]]; }, sx,
                sy, sz);
            relax_store<19, A, S, NT>(dst, N, (uint32_t)(x + nx * (y + ny * z)), cur, da,
                                      ref_a + da, fmad(ka, sx, upx), fmad(ka, sy, upy),
                                      fmad(ka, sz, upz), ia);
        }
#pragma unroll
        for (int i = 0; i < 19; ++i) cur[i] = nxt[i];
        s3 = n3;
    }
}

// ------------------------------------------------------------------------------------------
// Reported fields: both densities (FP64, shift added back, one pass), then rho_l, rho_v and the
// barycentric
// velocity u = (j_l + j_v + (F_l + F_v) / 2) / (rho_l + rho_v).  Grid-stride, test cadence only.
// ------------------------------------------------------------------------------------------
template <int Q, typename S>
__device__ __forceinline__ void pull_at(const S* src, int64_t N, int nx, int ny, int nz,
                                        int64_t n, float* g)
{
    const int x = (int)(n % nx);
    const int64_t r = n / nx;
    const int y = (int)(r % ny), z = (int)(r / ny);
    pull_node<Q>(src, N, nx, ny, x, wrap_once(x - 1, nx), wrap_once(x + 1, nx), y,
                 wrap_once(y - 1, ny), wrap_once(y + 1, ny), z,
                 Q == 19 ? wrap_once(z - 1, nz) : 0, Q == 19 ? wrap_once(z + 1, nz) : 0, g);
}

template <int Q, typename S>
__global__ void __launch_bounds__(256) k_dens2c(const S* __restrict__ fl,
                                                const S* __restrict__ fv,
                                                double* __restrict__ dens, Step2cArgs a)
{
    for (int64_t n = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; n < a.N;
         n += (int64_t)gridDim.x * blockDim.x) {
        float g[Q];
        pull_at<Q>(fl, a.N, a.nx, a.ny, a.nz, n, g);
        dens[n] = a.ref_l + sum_dev<Q, double>(g);
        pull_at<Q>(fv, a.N, a.nx, a.ny, a.nz, n, g);
        dens[a.N + n] = a.ref_v + sum_dev<Q, double>(g);
    }
}

// Node n + e_i, periodic.
template <int Q>
__device__ __forceinline__ int64_t node_plus(int x, int y, int z, int i, const Step2cArgs& a)
{
    using L = lat<Q>;
    return wrap_once(x + L::ex[i], a.nx) +
           (int64_t)a.nx * (wrap_once(y + L::ey[i], a.ny) +
                            (int64_t)a.ny * (Q == 19 ? wrap_once(z + L::ez[i], a.nz) : 0));
}

template <int Q, typename S>
__global__ void __launch_bounds__(256) k_fields2c(const S* __restrict__ fl,
                                                  const S* __restrict__ fv,
                                                  const double* __restrict__ dens, float* rl_out,
                                                  float* rv_out, float* u_out, Step2cArgs a)
{
    for (int64_t n = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; n < a.N;
         n += (int64_t)gridDim.x * blockDim.x) {
        const double rl = dens[n], rv = dens[a.N + n];
        if (rl_out) rl_out[n] = (float)rl;
        if (rv_out) rv_out[n] = (float)rv;
        if (!u_out) continue;
        const int x = (int)(n % a.nx);
        const int64_t r = n / a.nx;
        const int y = (int)(r % a.ny), z = (int)(r / a.ny);
        float gl[Q], gv[Q];
        pull_at<Q>(fl, a.N, a.nx, a.ny, a.nz, n, gl);
        pull_at<Q>(fv, a.N, a.nx, a.ny, a.nz, n, gv);
        double sx, sy, sz, tx, ty, tz, j[2][3];
        interaction_sum<Q, double>([&](int i) { return dens[a.N + node_plus<Q>(x, y, z, i, a)]; },
                                   sx, sy, sz);
        interaction_sum<Q, double>([&](int i) { return dens[node_plus<Q>(x, y, z, i, a)]; },
                                   tx, ty, tz);
        momentum<Q, double>(gl, j[0][0], j[0][1], j[0][2]);
        momentum<Q, double>(gv, j[1][0], j[1][1], j[1][2]);
        const double Sf[3] = {rl * sx + rv * tx, rl * sy + rv * ty, rl * sz + rv * tz};
        for (int c = 0; c < lat<Q>::d; ++c)
            u_out[(int64_t)c * a.N + n] =
                (float)((j[0][c] + j[1][c] - 0.5 * a.Gx * Sf[c]) / (rl + rv));
    }
}

dim3 grid_nodes(int64_t N)
{
    int64_t b = (N + 255) / 256;
    return dim3((unsigned)std::max<int64_t>(1, std::min<int64_t>(b, 1 << 16)));
}

}  // namespace

bool step2c_shape_supported(int q, const StepShape& s)
{
    if (s.tile_z < 1) return false;
    if (q == SC_D2Q9)
        return (s.variant == 1 || s.variant == 3) && s.tile_y == 1 &&
               (s.tile_x == 64 || s.tile_x == 128 || s.tile_x == 256 || s.tile_x == 512);
    if (s.variant < 1 || s.variant > 5 || s.variant == 2) return false;
    if (q == SC_D3Q19) {
        const int tx = s.tile_x, ty = s.tile_y;
        return (tx == 32 && (ty == 4 || ty == 8)) || (tx == 64 && (ty == 4 || ty == 8)) ||
               (tx == 128 && ty == 4);
    }
    return false;
}

namespace {

template <typename S, typename A>
hipError_t step2c_typed(int q, const S* src_l, const S* src_v, S* dst_l, S* dst_v,
                        const Step2cArgs& a, const StepShape& s, const StepGrid& g,
                        hipStream_t st)
{
    const dim3 grid(g.gx * g.gy * g.gz);
    const bool nt = s.variant == 3 || s.variant == 5;
    const bool split = s.variant >= 4;
#define SC_M2(TX)                                                                                \
    if (s.tile_x == TX) {                                                                        \
        if (nt)                                                                                  \
            hipLaunchKernelGGL((k_mix2d<S, A, TX, true>), grid, dim3(TX), 0, st, src_l, src_v,   \
                               dst_l, dst_v, a, g);                                              \
        else                                                                                     \
            hipLaunchKernelGGL((k_mix2d<S, A, TX, false>), grid, dim3(TX), 0, st, src_l, src_v,  \
                               dst_l, dst_v, a, g);                                              \
        return hipGetLastError();                                                                \
    }
#define SC_M3(TX, TY)                                                                            \
    if (s.tile_x == TX && s.tile_y == TY) {                                                      \
        if (split) {                                                                             \
            if (nt)                                                                              \
                hipLaunchKernelGGL((k_mix3d_split<S, A, TX, TY, true>), grid, dim3(2 * TX * TY), \
                                   0, st, src_l, src_v, dst_l, dst_v, a, g);                     \
            else                                                                                 \
                hipLaunchKernelGGL((k_mix3d_split<S, A, TX, TY, false>), grid,                   \
                                   dim3(2 * TX * TY), 0, st, src_l, src_v, dst_l, dst_v, a, g);  \
            return hipGetLastError();                                                            \
        }                                                                                        \
        if (nt)                                                                                  \
            hipLaunchKernelGGL((k_mix3d<S, A, TX, TY, true>), grid, dim3(TX * TY), 0, st, src_l, \
                               src_v, dst_l, dst_v, a, g);                                       \
        else                                                                                     \
            hipLaunchKernelGGL((k_mix3d<S, A, TX, TY, false>), grid, dim3(TX * TY), 0, st,       \
                               src_l, src_v, dst_l, dst_v, a, g);                                \
        return hipGetLastError();                                                                \
    }
    if (q == SC_D2Q9) {
        SC_M2(64) SC_M2(128) SC_M2(256) SC_M2(512)
    } else {
        SC_M3(32, 4) SC_M3(32, 8) SC_M3(64, 4) SC_M3(64, 8) SC_M3(128, 4)
    }
#undef SC_M2
#undef SC_M3
    return hipErrorInvalidValue;
}

template <typename S>
hipError_t fields2c_typed(int q, const S* f_l, const S* f_v, double* dens, float* rho_l,
                          float* rho_v, float* u, const Step2cArgs& a, hipStream_t st)
{
    const dim3 grid = grid_nodes(a.N);
    if (q == SC_D2Q9) {
        hipLaunchKernelGGL((k_dens2c<9, S>), grid, dim3(256), 0, st, f_l, f_v, dens, a);
        hipLaunchKernelGGL((k_fields2c<9, S>), grid, dim3(256), 0, st, f_l, f_v, dens, rho_l,
                           rho_v, u, a);
    } else if (q == SC_D3Q19) {
        hipLaunchKernelGGL((k_dens2c<19, S>), grid, dim3(256), 0, st, f_l, f_v, dens, a);
        hipLaunchKernelGGL((k_fields2c<19, S>), grid, dim3(256), 0, st, f_l, f_v, dens, rho_l,
                           rho_v, u, a);
    } else {
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace

hipError_t launch_step2c(int q, int storage, const void* src_l, const void* src_v, void* dst_l,
                         void* dst_v, const Step2cArgs& a0, const StepShape& s, hipStream_t st)
{
    if (!step2c_shape_supported(q, s)) return hipErrorInvalidValue;
    Step2cArgs a = a0;
    a.planes = s.tile_z;
    StepGrid g;
    g.gx = (a.nx + s.tile_x - 1) / s.tile_x;
    if (q == SC_D2Q9) {
        g.gy = (a.ny + a.planes - 1) / a.planes;
        g.gz = 1;
    } else {
        g.gy = (a.ny + s.tile_y - 1) / s.tile_y;
        g.gz = (a.nz + a.planes - 1) / a.planes;
    }
    g.remap = ((g.gx * g.gy * g.gz) % 8 == 0) ? 1 : 0;
    switch (storage) {
        case SC_STORE_F32:
            return step2c_typed<float, double>(q, (const float*)src_l, (const float*)src_v,
                                               (float*)dst_l, (float*)dst_v, a, s, g, st);
        case SC_STORE_F16:
            return step2c_typed<_Float16, float>(q, (const _Float16*)src_l,
                                                 (const _Float16*)src_v, (_Float16*)dst_l,
                                                 (_Float16*)dst_v, a, s, g, st);
        case SC_STORE_BF16:
            return step2c_typed<__bf16, float>(q, (const __bf16*)src_l, (const __bf16*)src_v,
                                               (__bf16*)dst_l, (__bf16*)dst_v, a, s, g, st);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_fields2c(int q, int storage, const void* f_l, const void* f_v, double* dens,
                           float* rho_l, float* rho_v, float* u, const Step2cArgs& a,
                           hipStream_t st)
{
    switch (storage) {
        case SC_STORE_F32:
            return fields2c_typed<float>(q, (const float*)f_l, (const float*)f_v, dens, rho_l,
                                         rho_v, u, a, st);
        case SC_STORE_F16:
            return fields2c_typed<_Float16>(q, (const _Float16*)f_l, (const _Float16*)f_v, dens,
                                            rho_l, rho_v, u, a, st);
        case SC_STORE_BF16:
            return fields2c_typed<__bf16>(q, (const __bf16*)f_l, (const __bf16*)f_v, dens, rho_l,
                                          rho_v, u, a, st);
    }
    return hipErrorInvalidValue;
}

}  // namespace sc
