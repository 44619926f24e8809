// lbm_kernels.hip -- gfx950 kernels of the fused lattice-Boltzmann LES canopy
// step and its auxiliary passes (init, state import/export, moments,
// deterministic FP64 reductions, plane statistics).
//
// Method (Shao et al., arXiv 2206.15454): D3Q19 BGK with Guo forcing
// (Sec. 2.1, Eqs. lbe, bgk, local_eq, bodyforce, density, momentum, tensor),
// Smagorinsky eddy viscosity (Sec. 2.2), forest drag as a body force
// (Sec. 2.3, Eq. forestForce), per-step order of Algorithm 1 (Sec. 3):
// stream, velocity, forest force, corrected velocity, collide with the force.
//
// Storage scheme (this implementation, not the paper's double population):
// one population buffer updated in place with the AA access pattern.
//   local step  (parity 1): cell x reads slot q of x (incoming f_q) and writes
//                           f*_q to slot opp(q) of x;
//   neighbour step (parity 0): cell x reads slot opp(q) of x - c_q (which holds
//                           f*_q of the upstream cell) and writes f*_q to slot
//                           q of x + c_q.
// In both, a cell reads and writes the same 19 slots, so no two cells touch a
// common slot and the update is race free.  Walls are folded into the slot
// map: halfway bounce-back keeps a population in its own cell with the
// opposite direction; free slip moves it tangentially within the wall row
// with the y component reversed.
#include "lbm_device.h"
#include "mlp_closure.h"

namespace lbmx {

namespace {

template <class C> __device__ __forceinline__ C wave_sum(C v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}
__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
    return v;
}

// Deterministic block sum of K values (256 threads = 4 waves): wave
// butterflies, then a fixed-order sum of the 4 wave results in FP64.
// Thread c < K adds the block total of value c into acc[c].  The barrier on
// entry orders this call's writes of sh after the previous call's reads
// (the persistent kernel calls it once per tile and again at its end).
template <int K, class C>
__device__ __forceinline__ void block_accumulate(const C (&v)[K], double *acc, double *sh) {
    const int tid = threadIdx.x + threadIdx.y * blockDim.x;
    const int lane = tid & 63, wave = tid >> 6;
    __syncthreads();
#pragma unroll
    for (int c = 0; c < K; ++c) {
        C s = wave_sum(v[c]);
        if (lane == 0) sh[wave * K + c] = (double)s;
    }
    __syncthreads();
    if (tid < K) {
        double t = sh[tid] + sh[K + tid];
        t += sh[2 * K + tid];
        t += sh[3 * K + tid];
        acc[tid] += t;
    }
}

// One tile (BX x 1 x BZ cells of row j) of one fused time step.
// wave-local ordering of LDS accesses (each wave stages into its own region)
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <int ST, bool LEARNED, int VAR>
__device__ __forceinline__ void step_tile(const StepArgs &a, const int tile, const MlpFrag &frag,
                                          const MlpConst *mc, short *zst, double *sh,
                                          double (&imp)[3],
                                          typename Codec<ST>::C *pst, unsigned &fallbacks) {
    // a * b + c is fused only inside one expression, as written: the
    // rounding then does not depend on how the compiler lays out a kernel's
    // blocks (the plain and the persistent learned-closure kernels share this
    // code and give bit-identical populations when every cell falls back)
#pragma clang fp contract(on)
    using CD = Codec<ST>;
    using T = typename CD::T;
    using C = typename CD::C;
    // population array: buffer resources, or 64-bit addresses for arrays
    // too large for them.  The learned-closure kernel uses the two array
    // resources for every type: 19 per-plane resources would take the scalar
    // registers that the network needs.
    using Pop = std::conditional_t<(VAR & VAR_WIDE) != 0, PopGlobal<ST>,
                                   std::conditional_t<LEARNED, PopBuf<PopArray<ST>>, PopBufOf<ST>>>;
    Pop pop;
    pop.init(static_cast<T *>(a.f), a.qs);
    // kernel scalars in the arithmetic type (FP32 copies avoid per-thread conversions)
    constexpr bool F32 = std::is_same_v<C, float>;
    auto sc = [](double d, float fl) -> C {
        if constexpr (F32) return fl; else return (C)d;
    };

    // tile numbering, x tile fastest: row-major (then the z tile, then the row
    // j) or, with FLAG_MEMORDER and in the learned-closure kernel, memory
    // order (then the row j, then the z tile), in which the tiles that run at
    // the same time touch neighbouring rows of each plane
    const int nx = a.nx, ny = a.ny, nz = a.nz;
    const int rest = (int)div_by((uint32_t)tile, a.m_nbx, a.s_nbx);
    const int bx = tile - rest * a.nbx;
    int j, bz;  // the whole block lies in row j
    if (LEARNED || (a.flags & FLAG_MEMORDER) != 0) {
        bz = (int)div_by((uint32_t)rest, a.m_ny, a.s_ny);
        j = rest - bz * a.nrows;
    } else {
        j = (int)div_by((uint32_t)rest, a.m_nbz, a.s_nbz);
        bz = rest - j * a.nbz;
    }
    j += a.j0;  // the launch's rows
    const int i = bx * (int)blockDim.x + (int)threadIdx.x;
    // the z row: uniform per wave (tiles are 64, 128 or 256 cells wide); the
    // plain step holds it, and so its z offsets, in scalar registers (+1.3 %
    // for FP32 at 512x128x256); the learned-closure kernel, whose scalar
    // registers are full, keeps them in vector registers (held in scalar
    // ones, they tripled its spills to vector lanes)
    const int kv = bz * (int)blockDim.y + (int)threadIdx.y;
    const int k = LEARNED ? kv : __builtin_amdgcn_readfirstlane(kv);
    const bool active = (i < nx) && (k < nz);
    const int ic = i < nx ? i : nx - 1;  // clamped: inactive lanes load valid memory
    // pad lanes (on a padded row's cells nx <= i < px) load and store their
    // own pad cells, x offsets 0, so that every cache line of the row is
    // written whole (rows whose last line was written in part ran 6 % slower
    // at 350 cells); they never touch a cell of the grid, and no cell reads
    // their values
    const int px = a.px;
    const bool pad = (i >= nx) && (i < px) && (k < nz);
    const int kc = k < nz ? k : nz - 1;

    // neighbour coordinates with periodic wrap (y wraps only if periodic;
    // otherwise out-of-range rows go through the wall branches)
    // The neighbour's index is the own index plus one offset per axis: x
    // and z wrap per thread (a select), y is uniform per block, so the 18
    // neighbours cost additions only.
    // self: the cell's dense index (moments, forest index, rounding hash);
    // pself: its population index, rows laid out with the pitch px >= nx
    // (rows padded to whole cache lines)
    const int plane = a.zp;  // z-layer pitch (>= px ny)
    const int self = (kc * ny + j) * nx + ic;
    const int pself = kc * plane + j * px + (pad ? i : ic);
    const int xo[3] = {pad ? 0 : ic == 0 ? nx - 1 : -1, 0, pad ? 0 : ic == nx - 1 ? 1 - nx : 1};
    const int yo[3] = {(j == 0 ? ny - 1 : -1) * px, 0, (j == ny - 1 ? 1 - ny : 1) * px};
    const int zo[3] = {kc == 0 ? (nz - 1) * plane : -plane, 0,
                       kc == nz - 1 ? (1 - nz) * plane : plane};
    auto cell = [&](int dx, int dy, int dz) -> int {
        return pself + xo[dx + 1] + yo[dy + 1] + zo[dz + 1];
    };

    // ---- a1/a2: stream in (AA slot map with walls), decode ----------------
    // a forced-equilibrium boundary supplies feq(1, u_wall) - w for every
    // population entering through it (both parities)
    auto feq_wall = [&](int q) -> C {
        const C uwx = sc(a.u_wall[0], a.u_wallf[0]), uwy = sc(a.u_wall[1], a.u_wallf[1]),
                uwz = sc(a.u_wall[2], a.u_wallf[2]);
        const C cu = (C)CX[q] * uwx + (C)CY[q] * uwy + (C)CZ[q] * uwz;
        const C uu = uwx * uwx + uwy * uwy + uwz * uwz;
        return (C)weight(q) * (C(3) * cu + C(4.5) * cu * cu - C(1.5) * uu);
    };
    // Every direction is loaded first (a direction entering through a
    // forced-equilibrium boundary reads a valid slot of its own cell, as for
    // bounce-back) and replaced afterwards, so no decode waits inside a
    // per-direction branch.
    // heterogeneous forest: the cell's table index is loaded before the
    // populations, so that the dependent table load overlaps with them
    // (vmcnt retires loads in order: issued after them, each would wait for
    // all 19)
    [[maybe_unused]] uint32_t fidx = 0;
    if constexpr ((VAR & VAR_FOREST) != 0) fidx = a.fidx[self];

    C v[NQ];
    // rows whose neighbour step crosses a non-periodic y boundary (uniform per
    // block); the other rows stream without per-direction wall tests
    const bool wall_row = (j == 0 && a.bc_lo != BC_PERIODIC) || (j == ny - 1 && a.bc_hi != BC_PERIODIC);
    auto load = [&](auto stream) {
        constexpr bool S = decltype(stream)::value;
        if (a.parity) {
            static_for<NQ>([&](auto qc) {
                constexpr int q = decltype(qc)::value;
                v[q] = pop.template ld<policy_local<S>()>(q, pself);
            });
        } else if (!wall_row) {
            static_for<NQ>([&](auto qc) {
                constexpr int q = decltype(qc)::value;
                v[q] = pop.template ld<policy_neigh<S>(q)>(opp(q), cell(-CX[q], -CY[q], -CZ[q]));
            });
        } else {
            static_for<NQ>([&](auto qc) {
                constexpr int q = decltype(qc)::value;
                constexpr int cx = CX[q], cy = CY[q], cz = CZ[q];
                constexpr int pol = policy_neigh<S>(q);
                const int js = j - cy;
                if (cy != 0 && (js < 0 || js >= ny) &&
                    (js < 0 ? a.bc_lo : a.bc_hi) != BC_PERIODIC) {
                    if ((js < 0 ? a.bc_lo : a.bc_hi) != BC_FREESLIP)
                        v[q] = pop.template ld<pol>(q, pself);  // left this cell towards the wall
                    else  // free slip: left the wall row upstream, moving towards the wall
                        v[q] = pop.template ld<pol>(opp(mir(q)), cell(-cx, 0, -cz));
                } else {
                    v[q] = pop.template ld<pol>(opp(q), cell(-cx, -cy, -cz));
                }
            });
        }
    };
    // the plain step kernel has the policy as a compile-time variant; the
    // learned-closure kernel branches on the flag (uniform per launch)
    constexpr bool kStream = (VAR & VAR_STREAM) != 0;
    [[maybe_unused]] const bool streaming = LEARNED ? (a.flags & FLAG_STREAMING) != 0 : kStream;
    if constexpr (!LEARNED)
        load(std::bool_constant<kStream>{});
    else if (streaming)
        load(std::true_type{});
    else
        load(std::false_type{});
    if ((j == 0 && a.bc_lo == BC_EQUILIBRIUM) || (j == ny - 1 && a.bc_hi == BC_EQUILIBRIUM)) {
        static_for<NQ>([&](auto qc) {  // uniform per block (one row per block)
            constexpr int q = decltype(qc)::value;
            const int js = j - CY[q];
            if (CY[q] != 0 && (js < 0 || js >= ny) &&
                (js < 0 ? a.bc_lo : a.bc_hi) == BC_EQUILIBRIUM)
                v[q] = feq_wall(q);
        });
    }

    // the cell's LAD (heterogeneous forest): issued right behind the
    // population loads, it needs only the index, which arrived first
    [[maybe_unused]] C lad_cell = 0;
    if constexpr ((VAR & VAR_FOREST) != 0) {
        if constexpr (F32)
            lad_cell = a.ftabf[fidx];
        else
            lad_cell = (C)a.ftab[fidx];
        __builtin_amdgcn_sched_barrier(0);  // keep the load here
    }

    // ---- a3: moments from the shifted values (no cancellation) ------------
    // drho = sum f~, j = sum f~ c, P = sum f~ c c  (f = f~ + w; sum w c c = I/3).
    // Opposite directions q, q+1 enter through their sum (the even moments)
    // and their difference (the odd moments).  The sums start from -0, which
    // adds nothing in IEEE arithmetic, so the first term costs no operation.
    C drho = v[0];
    C jx = C(-0.0), jy = C(-0.0), jz = C(-0.0);
    C pxx = C(-0.0), pyy = C(-0.0), pzz = C(-0.0), pxy = C(-0.0), pxz = C(-0.0), pyz = C(-0.0);
    static_for<(NQ - 1) / 2>([&](auto pc) {
        constexpr int q = 2 * decltype(pc)::value + 1;  // q and q + 1 = opp(q)
        constexpr int cx = CX[q], cy = CY[q], cz = CZ[q];
        const C sum = v[q] + v[q + 1], dif = v[q] - v[q + 1];
        drho += sum;
        if (cx) jx += cx > 0 ? dif : -dif;
        if (cy) jy += cy > 0 ? dif : -dif;
        if (cz) jz += cz > 0 ? dif : -dif;
        if (cx) pxx += sum;
        if (cy) pyy += sum;
        if (cz) pzz += sum;
        if (cx && cy) pxy += (cx * cy > 0) ? sum : -sum;
        if (cx && cz) pxz += (cx * cz > 0) ? sum : -sum;
        if (cy && cz) pyz += (cy * cz > 0) ? sum : -sum;
    });
    const C rho = C(1) + drho;
    const C irho = arith_rcp(rho);

    // ---- a4: velocity with the driving force, canopy drag, corrected u ----
    // VAR_FX: the driving force and the drag act along x only, so F_y = F_z =
    // 0 is known here and the terms they enter are left out (the general
    // form gives the same values: those terms are exact zeros)
    constexpr bool FX = (VAR & VAR_FX) != 0;
    const C gx = sc(a.g[0], a.gf[0]);
    const C gy = FX ? C(0) : sc(a.g[1], a.gf[1]), gz = FX ? C(0) : sc(a.g[2], a.gf[2]);
    C ux = (jx + C(0.5) * rho * gx) * irho;
    C uy = FX ? jy * irho : (jy + C(0.5) * rho * gy) * irho;
    C uz = FX ? jz * irho : (jz + C(0.5) * rho * gz) * irho;
    C ax = gx, ay = gy, az = gz;  // total acceleration
    auto drag = [&](C lad) {
        const C speed = arith_sqrt(ux * ux + uy * uy + uz * uz);
        const C kd = -sc(a.cd, a.cdf) * lad * speed;  // drag acceleration per unit velocity
        const C adx = kd * ux;
        ax += adx;
        if (!FX && (a.flags & FLAG_VECTOR_DRAG)) {
            const C ady = kd * uy, adz = kd * uz;
            ay += ady;
            az += adz;
            uy += C(0.5) * ady;
            uz += C(0.5) * adz;
        }
        ux += C(0.5) * adx;
    };
    // LAD of the cell for a heterogeneous forest, else of the row (uniform
    // per block: the block is one row)
    C lad;
    if constexpr ((VAR & VAR_FOREST) != 0)
        lad = lad_cell;
    else
        lad = (C)a.lad[j];
    if (lad > C(0)) drag(lad);
    const C Fx = rho * ax, Fy = FX ? C(0) : rho * ay, Fz = FX ? C(0) : rho * az;

    // ---- a5: Smagorinsky: Pi_neq = P - drho/3 I - rho u u -----------------
    const C third = C(1) / C(3);
    const C nxx = pxx - drho * third - rho * ux * ux;
    const C nyy = pyy - drho * third - rho * uy * uy;
    const C nzz = pzz - drho * third - rho * uz * uz;
    const C nxy = pxy - rho * ux * uy;
    const C nxz = pxz - rho * ux * uz;
    const C nyz = pyz - rho * uy * uz;
    const C tau0 = sc(a.tau0, a.tau0f);
    // tau = (tau0 + sqrt(tau0^2 + X))/2, X = 18 sqrt2 C Q^(1/2)/rho, written
    // as tau0 + 3 nu_t with nu_t = X / (6 (sqrt(tau0^2 + X) + tau0))
    auto smagorinsky = [&]() -> C {
        const C Qh = arith_sqrt(nxx * nxx + nyy * nyy + nzz * nzz +
                                C(2) * (nxy * nxy + nxz * nxz + nyz * nyz));
        const C X = sc(a.ksmag, a.ksmagf) * Qh * irho;
        return X * arith_rcp(C(6) * (arith_sqrt(tau0 * tau0 + X) + tau0));
    };
    const long long ncell = (long long)nx * ny * nz;
    C nut;
    if constexpr ((VAR & VAR_NUT_IN) != 0) {
        // the learned closure's nu_t of its last evaluation, reused
        nut = static_cast<const C *>(a.mom)[4 * ncell + self];
    } else if constexpr (!LEARNED) {
        nut = smagorinsky();
    } else {
        // learned closure where the features are inside the trained range,
        // Smagorinsky elsewhere (evaluated only in a wavefront that has such
        // a cell: the test is uniform per wavefront)
        const int tid = threadIdx.x + threadIdx.y * blockDim.x;
        const int lane = tid & 63;
        float x[9];
        mlp_features((float)nxx, (float)nyy, (float)nzz, (float)nxy, (float)nxz, (float)nyz,
                     (float)rho, ((float)j + 0.5f) * mc->inv_h, (float)lad, x);
        bool in_range = true;
        short z[16];
#pragma unroll
        for (int c = 0; c < 9; ++c) {
            in_range = in_range && active && (x[c] >= mc->lo[c]) && (x[c] <= mc->hi[c]);
            z[c] = bf16_bits(x[c] * mc->zs[c] + mc->zo[c]);
        }
        z[9] = z[10] = bf16_bits(1.0f);
#pragma unroll
        for (int c = 11; c < 16; ++c) z[c] = 0;
        // A wavefront whose 64 cells all fall back skips the network (the
        // test is uniform per wavefront; the results are the same).
        bool use = false;
        float learned = 0.0f;
        if (__builtin_amdgcn_ballot_w64(in_range) != 0) {
            // park the populations in LDS while the network runs (frees registers)
            static_for<NQ>([&](auto qc) {
                constexpr int q = decltype(qc)::value;
                pst[q * 256 + tid] = v[q];
            });
            wave_lds_sync();  // the previous tile's reads of this wave's staging area are done
            mlp_stage_inputs(zst, lane, z);
            wave_lds_sync();
            const float o = mlp_forward_wave(frag, zst, lane, mc->b3);
            static_for<NQ>([&](auto qc) {
                constexpr int q = decltype(qc)::value;
                v[q] = pst[q * 256 + tid];
            });
            // a cell whose network activations left the FP16 range (|x| >
            // 65504) gets a non-finite output: it falls back like an
            // out-of-range cell
            learned = mc->scale * mlp_softplus(o);
            use = in_range && __builtin_isfinite(learned);
        }
        nut = (C)learned;
        if (__builtin_amdgcn_ballot_w64(!use) != 0) {
            const C ns = smagorinsky();
            if (!use) nut = ns;
        }
        fallbacks += (!use && active) ? 1u : 0u;
    }
    const C tau = tau0 + C(3) * nut;
    const C itau = arith_rcp(tau);

    // ---- a6: equilibrium + Guo forcing + BGK (shifted) ----------------------
    // Directions q (odd) and q+1 are opposite: c.u and c.F change sign.  The
    // shifted equilibrium times 1/tau plus the Guo term of the pair splits
    // into a part even and a part odd in c:
    //   even = w (K + (c.u) (a1 (c.u) + a2 (c.F))),  odd = w (b1 (c.u) + b2 (c.F)),
    //   K = (drho - 1.5 rho u.u) / tau - 3 pref u.F,  a1 = 4.5 rho / tau,
    //   a2 = 9 pref,  b1 = 3 rho / tau,  b2 = 3 pref,  pref = 1 - 1/(2 tau),
    // then f~_q <- (1 - 1/tau) f~_q + even + odd and f~_{q+1} <- ... + even - odd.
    // The weight is folded into the per-cell scalars of its class (1/18 for
    // the axis directions, 1/36 for the edge directions).
    const C usq15 = C(1.5) * (ux * ux + uy * uy + uz * uz);
    const C uF = FX ? ux * Fx : ux * Fx + uy * Fy + uz * Fz;
    const C pref = C(1) - C(0.5) * itau;
    const C om = C(1) - itau;
    const C K = itau * (drho - rho * usq15) - C(3) * pref * uF;
    const C ri = rho * itau;
    constexpr C w1 = (C)weight(1), w2 = (C)weight(7);
    const C Kw[2] = {w1 * K, w2 * K};
    const C a1w[2] = {(w1 * C(4.5)) * ri, (w2 * C(4.5)) * ri};
    const C a2w[2] = {(w1 * C(9)) * pref, (w2 * C(9)) * pref};
    const C b1w[2] = {(w1 * C(3)) * ri, (w2 * C(3)) * ri};
    const C b2w[2] = {(w1 * C(3)) * pref, (w2 * C(3)) * pref};
    v[0] = v[0] * om + (C)weight(0) * K;
    static_for<(NQ - 1) / 2>([&](auto pc) {
        constexpr int q = 2 * decltype(pc)::value + 1;  // q and q + 1 = opp(q)
        constexpr int cx = CX[q], cy = CY[q], cz = CZ[q];
        constexpr int cls = weight(q) == weight(1) ? 0 : 1;
        C cu = C(-0.0), cF = C(-0.0);
        if (cx) { cu += cx > 0 ? ux : -ux; cF += cx > 0 ? Fx : -Fx; }
        if (cy) { cu += cy > 0 ? uy : -uy; if (!FX) cF += cy > 0 ? Fy : -Fy; }
        if (cz) { cu += cz > 0 ? uz : -uz; if (!FX) cF += cz > 0 ? Fz : -Fz; }
        C even, odd;
        if constexpr (FX && cx == 0) {  // c.F = 0
            even = Kw[cls] + cu * (a1w[cls] * cu);
            odd = b1w[cls] * cu;
        } else {
            even = Kw[cls] + cu * (a1w[cls] * cu + a2w[cls] * cF);
            odd = b1w[cls] * cu + b2w[cls] * cF;
        }
        v[q] = v[q] * om + (even + odd);
        v[q + 1] = v[q + 1] * om + (even - odd);
    });

    // ---- a7: store in place --------------------------------------------------
    // random bits for stochastic rounding (unused by the other storage types):
    // one hash of (step seed, cell), then one step of Marsaglia's xorshift32
    // generator (shifts 13, 17, 5; "Xorshift RNGs", J. Stat. Softw. 8, 2003)
    // per pair of directions, whose low and high 16 bits serve the two
    // directions
    uint32_t rstate = (ST == ST_BF16SR) ? mix32(a.seed ^ ((uint32_t)self * 0x9E3779B1u)) | 1u : 0u;
    uint32_t rpair = 0;
    auto rnd = [&](int q) -> uint32_t {
        if (ST != ST_BF16SR) return 0u;
        if ((q & 1) == 0) {  // q = 0 and every second direction start a new word
            rstate ^= rstate << 13;
            rstate ^= rstate >> 17;
            rstate ^= rstate << 5;
            rpair = rstate;
        }
        return (q & 1) ? rpair : (rpair >> 16);
    };
    auto store = [&](auto stream) {
        constexpr bool S = decltype(stream)::value;
        if (a.parity) {
            static_for<NQ>([&](auto qc) {
                constexpr int q = decltype(qc)::value;
                pop.template st<policy_local<S>()>(opp(q), pself, v[q], rnd(q));
            });
        } else if (!wall_row) {
            static_for<NQ>([&](auto qc) {
                constexpr int q = decltype(qc)::value;
                pop.template st<policy_neigh<S>(q)>(q, cell(CX[q], CY[q], CZ[q]), v[q], rnd(q));
            });
        } else {
            static_for<NQ>([&](auto qc) {
                constexpr int q = decltype(qc)::value;
                constexpr int cx = CX[q], cy = CY[q], cz = CZ[q];
                constexpr int pol = policy_neigh<S>(q);
                const int jt = j + cy;
                if (cy != 0 && (jt < 0 || jt >= ny) &&
                    (jt < 0 ? a.bc_lo : a.bc_hi) != BC_PERIODIC) {
                    // bounce-back, and the forced-equilibrium boundary, keep the
                    // leaving population in the own cell's opposite slot (a
                    // forced-equilibrium boundary never reads it back)
                    if ((jt < 0 ? a.bc_lo : a.bc_hi) != BC_FREESLIP)
                        pop.template st<pol>(opp(q), pself, v[q], rnd(q));
                    else
                        pop.template st<pol>(mir(q), cell(cx, 0, cz), v[q], rnd(q));
                } else {
                    pop.template st<pol>(q, cell(cx, cy, cz), v[q], rnd(q));
                }
            });
        }
    };
    if (active || pad) {
        if constexpr (!LEARNED)
            store(std::bool_constant<kStream>{});
        else if (streaming)
            store(std::true_type{});
        else
            store(std::false_type{});
    }

    // ---- a8: moments of this collision -------------------------------------
    // (FLAG_NUT_OUT: only nu_t, kept for the steps that reuse it)
    if ((a.flags & (FLAG_MOMENTS | FLAG_NUT_OUT)) && active) {
        C *m = static_cast<C *>(a.mom);
        if (a.flags & FLAG_MOMENTS) {
            m[self] = rho;
            m[ncell + self] = ux;
            m[2 * ncell + self] = uy;
            m[3 * ncell + self] = uz;
        }
        m[4 * ncell + self] = nut;
    }

    // ---- a9: FP64 diagnostics of this collision, one record per wavefront --
    // (mass, momentum, max |u|, non-finite cells of the moments written
    // above); lbm_moments reduces the records instead of reading the moment
    // planes again.  A non-finite cell adds nothing to the sums.
    if (a.flags & FLAG_MOMENTS) {
        const bool fin = active && __builtin_isfinite(rho) && __builtin_isfinite(ux) &&
                         __builtin_isfinite(uy) && __builtin_isfinite(uz) &&
                         __builtin_isfinite(nut);
        const double r = fin ? (double)rho : 0.0;
        const double dux = fin ? (double)ux : 0.0, duy = fin ? (double)uy : 0.0,
                     duz = fin ? (double)uz : 0.0;
        const double m0 = wave_sum(r), m1 = wave_sum(r * dux), m2 = wave_sum(r * duy),
                     m3 = wave_sum(r * duz);
        const double umax = wave_max(sqrt(dux * dux + duy * duy + duz * duz));
        const unsigned long long bad = __builtin_amdgcn_ballot_w64(active && !fin);
        const int tid = threadIdx.x + threadIdx.y * blockDim.x;
        if ((tid & 63) == 0) {
            double *rec = a.dg + 6 * (4 * (long long)tile + (tid >> 6));
            rec[0] = m0;
            rec[1] = m1;
            rec[2] = m2;
            rec[3] = m3;
            rec[4] = umax;
            rec[5] = (double)__builtin_popcountll(bad);
        }
    }

    // ---- body-force impulse and plane statistics (FP64 accumulators) ------
    if (a.flags & FLAG_IMPULSE) {
        const C z = 0;
        const C fv[3] = {active ? Fx : z, active ? Fy : z, active ? Fz : z};
        if constexpr (LEARNED) {
            // persistent blocks: per-thread FP64 sums over the block's tiles,
            // reduced once at the end of the kernel
            imp[0] += (double)fv[0];
            imp[1] += (double)fv[1];
            imp[2] += (double)fv[2];
        } else {
            // one FP64 accumulator triple per wavefront (no block barrier);
            // with FLAG_IMPULSE_X the y and z forces are exactly 0
            const int tid = threadIdx.x + threadIdx.y * blockDim.x;
            const bool yz = !(a.flags & FLAG_IMPULSE_X);
            const C s0 = wave_sum(fv[0]);
            const C s1 = yz ? wave_sum(fv[1]) : C(0), s2 = yz ? wave_sum(fv[2]) : C(0);
            if ((tid & 63) == 0) {
                double *acc = a.imp + 3 * (4 * (long long)tile + (tid >> 6));
                acc[0] += (double)s0;
                if (yz) {
                    acc[1] += (double)s1;
                    acc[2] += (double)s2;
                }
            }
        }
    }
    if (a.flags & FLAG_STATS) {
        // selects, not products with 0 or 1: a pad lane's values may be
        // non-finite
        auto m = [&](C v) { return active ? v : C(0); };
        const C sv[10] = {m(ux),      m(uy),      m(uz),      m(ux * ux), m(uy * uy),
                          m(uz * uz), m(ux * uy), m(ux * uz), m(uy * uz), m(nut)};
        const long long slot = ((long long)j * (a.nbx * a.nbz) + bz * a.nbx + bx) * 10;
        block_accumulate<10>(sv, a.stats + slot, sh);
    }
}

template <int ST, int VAR>
__global__ __launch_bounds__(256) void lbm_step_kernel(const StepArgs a) {
    __shared__ double sh[4 * 10];
    int tile = blockIdx.x;
    if (a.flags & FLAG_XCD_REMAP)
        tile = a.xcd_run > 0 ? xcd_remap_runs(tile, a.ntiles, a.xcd_run) : xcd_remap(tile, a.ntiles);
    double unused[3] = {0.0, 0.0, 0.0};
    unsigned nofb = 0;
    step_tile<ST, false, VAR>(a, tile, MlpFrag{}, nullptr, nullptr, sh, unused, nullptr, nofb);
}

// Learned closure: persistent blocks keep the network's weight fragments in
// registers and walk the tiles (linear index it = block + k * grid; with the
// grid a multiple of 8, every tile of a block stays on the block's XCD).
// The walk is in the memory order of the tiles: each XCD's contiguous share
// spans every row j, so the rows whose cells all fall back to Smagorinsky
// (and skip the network) are spread evenly over the XCDs and the blocks.
template <int ST, int VAR>
__global__ __launch_bounds__(256)
__attribute__((amdgpu_waves_per_eu(ST == ST_F64 ? 1 : 3, ST == ST_F64 ? 2 : 3)))
void lbm_step_mlp_kernel(const StepArgs a) {
    __shared__ double sh[4 * 10];
    __shared__ __attribute__((aligned(16))) short zst[4][64 * 16];
    __shared__ typename Codec<ST>::C pst[NQ * 256];  // populations parked during the network
    const int tid = threadIdx.x + threadIdx.y * blockDim.x;
    MlpParams *P = static_cast<MlpParams *>(const_cast<void *>(a.mlp));
    // fallback counters alternate between evaluations: clear the other one
    if (blockIdx.x == 0 && tid == 0) P->fallback[a.fb_slot ^ 1] = 0;
    __shared__ half8 w2s[4 * 2 * 64];
    mlp_stage_w2(P, w2s, tid, 256);
    // the closure scalars in LDS: read per tile with LDS loads instead of
    // occupying scalar registers for the whole walk
    __shared__ MlpConst mcs;
    static_assert(sizeof(MlpConst) % 4 == 0 && sizeof(MlpConst) / 4 <= 256, "one float per thread");
    if (tid < (int)(sizeof(MlpConst) / 4))
        reinterpret_cast<float *>(&mcs)[tid] = reinterpret_cast<const float *>(&a.mc)[tid];
    __syncthreads();
    const MlpFrag frag = mlp_load_frag(P, tid & 63, w2s);
    double imp[3] = {0.0, 0.0, 0.0};
    unsigned fallbacks = 0;
    for (int it = blockIdx.x; it < a.ntiles; it += gridDim.x) {
        const int tile = (a.flags & FLAG_XCD_REMAP) ? xcd_remap(it, a.ntiles) : it;
        step_tile<ST, true, VAR>(a, tile, frag, &mcs, zst[tid >> 6], sh, imp, pst, fallbacks);
    }
    // cells that fell back: one atomic per wave
    unsigned fsum = fallbacks;
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) fsum += __shfl_xor(fsum, off, 64);
    if ((tid & 63) == 0 && fsum) atomicAdd(&P->fallback[a.fb_slot], (unsigned long long)fsum);
    if (a.flags & FLAG_IMPULSE)
        block_accumulate<3>(imp, a.imp + 3 * (long long)blockIdx.x, sh);  // grid <= ntiles
}

// f = feq(rho, u) as post-collision populations, stored shifted in the
// layout a neighbour step reads (slot opp(q) of the own cell).
template <int ST>
__global__ __launch_bounds__(256) void init_kernel(void *fp, long long qs, int nx, int px,
                                                   int ny, int zp, void *mom, const double *rho,
                                                   const double *u, int n) {
    using CD = Codec<ST>;
    using T = typename CD::T;
    using C = typename CD::C;
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= n) return;
    T *f = static_cast<T *>(fp);
    const int row = x / nx;  // population index: rows of pitch px, z-layers of pitch zp
    const long long xp = (long long)(row / ny) * zp + (long long)(row % ny) * px + x % nx;
    const double r = rho[x], ux = u[x], uy = u[n + x], uz = u[2 * (long long)n + x];
    const double usq15 = 1.5 * (ux * ux + uy * uy + uz * uz);
    static_for<NQ>([&](auto qc) {
        constexpr int q = decltype(qc)::value;
        const double cu = CX[q] * ux + CY[q] * uy + CZ[q] * uz;
        const double w = weight(q);
        const double fs = w * ((r - 1.0) + r * (3.0 * cu + 4.5 * cu * cu - usq15));
        CD::st(f + opp(q) * qs + xp, (C)fs);
    });
    C *m = static_cast<C *>(mom);
    m[x] = (C)r;
    m[n + x] = (C)ux;
    m[2 * (long long)n + x] = (C)uy;
    m[3 * (long long)n + x] = (C)uz;
    m[4 * (long long)n + x] = (C)0;
}

// Slot of the in-place buffer that holds the post-collision population
// f*_q(x) before a step of the given AA parity: after a local step (parity 0
// next) slot opp(q) of x; after a neighbour step (parity 1 next) where the
// neighbour step wrote it (slot q of x + c_q, or the wall's slot).  A
// bijection of the 19 N slots (every cell reads and writes the same 19).
__device__ __forceinline__ long long slot_of(int q, int i, int j, int k, int nx, int px, int zp,
                                             int ny, int nz, int parity, int bc_lo, int bc_hi,
                                             long long qs) {
    // rows of pitch px, z-layers of pitch zp
    const long long own = (long long)k * zp + (long long)j * px + i;
    if (parity == 0) return opp(q) * qs + own;
    const int cx = CX[q], cy = CY[q], cz = CZ[q];
    const int it = (i + cx + nx) % nx, kt = (k + cz + nz) % nz;
    const int jt = j + cy;
    if (cy != 0 && (jt < 0 || jt >= ny) && (jt < 0 ? bc_lo : bc_hi) != BC_PERIODIC) {
        if ((jt < 0 ? bc_lo : bc_hi) != BC_FREESLIP)  // bounce-back or forced equilibrium
            return opp(q) * qs + own;
        return mir(q) * qs + (long long)kt * zp + (long long)j * px + it;
    }
    return q * qs + (long long)kt * zp + (long long)((jt + ny) % ny) * px + it;
}

template <int ST>
__global__ __launch_bounds__(256) void set_f_kernel(void *fp, long long qs, const double *fin,
                                                    int nx, int px, int zp, int ny, int nz,
                                                    int parity, int bc_lo, int bc_hi) {
    using CD = Codec<ST>;
    using T = typename CD::T;
    using C = typename CD::C;
    const long long n = (long long)nx * ny * nz;
    const long long x = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= n) return;
    T *f = static_cast<T *>(fp);
    const int i = (int)(x % nx);
    const int j = (int)((x / nx) % ny);
    const int k = (int)(x / ((long long)nx * ny));
    static_for<NQ>([&](auto qc) {
        constexpr int q = decltype(qc)::value;
        const long long at = slot_of(q, i, j, k, nx, px, zp, ny, nz, parity, bc_lo, bc_hi, qs);
        CD::st(f + at, (C)(fin[(long long)q * n + x] - weight(q)));
    });
}

// post-collision populations f*_q(x) from the in-place buffer: after a local
// step (parity 0 next) they sit in slot opp(q) of x; after a neighbour step
// (parity 1 next) where the neighbour step wrote them.
template <int ST>
__global__ __launch_bounds__(256) void get_f_kernel(const void *fp, long long qs, double *fout,
                                                    int nx, int px, int zp, int ny, int nz,
                                                    int parity, int bc_lo, int bc_hi) {
    using CD = Codec<ST>;
    using T = typename CD::T;
    const long long n = (long long)nx * ny * nz;
    const long long x = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= n) return;
    const T *f = static_cast<const T *>(fp);
    const int i = (int)(x % nx);
    const int j = (int)((x / nx) % ny);
    const int k = (int)(x / ((long long)nx * ny));
    static_for<NQ>([&](auto qc) {
        constexpr int q = decltype(qc)::value;
        const long long at = slot_of(q, i, j, k, nx, px, zp, ny, nz, parity, bc_lo, bc_hi, qs);
        fout[q * n + x] = (double)CD::ld(f + at) + weight(q);
    });
}

template <int ST>
__global__ __launch_bounds__(256) void moments_out_kernel(const void *mom, double *rho,
                                                          double *u, double *nut, int n) {
    using C = typename Codec<ST>::C;
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= n) return;
    const C *m = static_cast<const C *>(mom);
    const long long N = n;
    if (rho) rho[x] = (double)m[x];
    if (u) {
        u[x] = (double)m[N + x];
        u[N + x] = (double)m[2 * N + x];
        u[2 * N + x] = (double)m[3 * N + x];
    }
    if (nut) nut[x] = (double)m[4 * N + x];
}

// pass 1: block b reduces cells [b*chunk, (b+1)*chunk) in FP64:
// mass, rho u (3), max |u|, non-finite count
template <int ST>
__global__ __launch_bounds__(256) void diag_partial_kernel(const void *mom, int n, int chunk,
                                                           double *partial) {
    using C = typename Codec<ST>::C;
    const C *m = static_cast<const C *>(mom);
    const long long N = n;
    const int beg = blockIdx.x * chunk;
    const int end = min(n, beg + chunk);
    double s[6] = {0, 0, 0, 0, 0, 0};
    for (int x = beg + threadIdx.x; x < end; x += blockDim.x) {
        const double r = m[x], ux = m[N + x], uy = m[2 * N + x], uz = m[3 * N + x];
        const double nt = m[4 * N + x];
        if (!(isfinite(r) && isfinite(ux) && isfinite(uy) && isfinite(uz) && isfinite(nt))) {
            s[5] += 1.0;
            continue;
        }
        s[0] += r;
        s[1] += r * ux;
        s[2] += r * uy;
        s[3] += r * uz;
        s[4] = fmax(s[4], sqrt(ux * ux + uy * uy + uz * uz));
    }
    __shared__ double sh[6][256];
    for (int c = 0; c < 6; ++c) sh[c][threadIdx.x] = s[c];
    __syncthreads();
    for (int w = 128; w >= 1; w >>= 1) {
        if ((int)threadIdx.x < w) {
            for (int c = 0; c < 6; ++c) {
                if (c == 4)
                    sh[c][threadIdx.x] = fmax(sh[c][threadIdx.x], sh[c][threadIdx.x + w]);
                else
                    sh[c][threadIdx.x] += sh[c][threadIdx.x + w];
            }
        }
        __syncthreads();
    }
    if (threadIdx.x < 6) partial[blockIdx.x * 6 + threadIdx.x] = sh[threadIdx.x][0];
}

// Deterministic tree sum over the 256 threads of a block: K values per
// thread in sh[K][256]; component cmax (if >= 0) takes the maximum.
template <int K>
__device__ __forceinline__ void block_tree(double (*sh)[256], int cmax) {
    __syncthreads();
    for (int w = 128; w >= 1; w >>= 1) {
        if ((int)threadIdx.x < w) {
            for (int c = 0; c < K; ++c) {
                if (c == cmax)
                    sh[c][threadIdx.x] = fmax(sh[c][threadIdx.x], sh[c][threadIdx.x + w]);
                else
                    sh[c][threadIdx.x] += sh[c][threadIdx.x + w];
            }
        }
        __syncthreads();
    }
}

// Per-wavefront records, pass 1: block b reduces records [b*chunk,
// (b+1)*chunk) of dg ([n][6]: mass, momentum (3), max |u|, non-finite; may
// be null) and imp ([n][3]: impulse) in FP64 into partial[b][9] = mass,
// momentum (3), impulse (3), max |u|, non-finite.
__global__ __launch_bounds__(256) void diag_records_kernel(const double *dg, const double *imp,
                                                           int n, int chunk, double *partial) {
    __shared__ double sh[9][256];
    const int beg = blockIdx.x * chunk;
    const int end = min(n, beg + chunk);
    double s[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    for (int x = beg + (int)threadIdx.x; x < end; x += blockDim.x) {
        if (dg) {
            const double *d = dg + 6 * (long long)x;
            s[0] += d[0];
            s[1] += d[1];
            s[2] += d[2];
            s[3] += d[3];
            s[7] = fmax(s[7], d[4]);
            s[8] += d[5];
        }
        const double *m = imp + 3 * (long long)x;
        s[4] += m[0];
        s[5] += m[1];
        s[6] += m[2];
    }
    for (int c = 0; c < 9; ++c) sh[c][threadIdx.x] = s[c];
    block_tree<9>(sh, 7);
    if (threadIdx.x < 9) partial[blockIdx.x * 9 + threadIdx.x] = sh[threadIdx.x][0];
}

// pass 2 (one block): fixed-order sums of the nb records of pass 1 and, when
// the mass, momentum, max |u| and non-finite count come from the moment
// planes instead (pm != null: diag_partial_kernel's nm records of 6), of
// those.  out: mass, mom[3], impulse[3], max|u|, nonfinite
__global__ __launch_bounds__(256) void diag_final_kernel(const double *ps, int nb,
                                                         const double *pm, int nm,
                                                         double *out) {
    __shared__ double sh[9][256];
    double s[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    for (int b = threadIdx.x; b < nb; b += blockDim.x) {
        for (int c = 0; c < 9; ++c) {
            if (c == 7)
                s[c] = fmax(s[c], ps[b * 9 + c]);
            else
                s[c] += ps[b * 9 + c];
        }
    }
    if (pm) {
        s[0] = s[1] = s[2] = s[3] = s[7] = s[8] = 0.0;
        for (int b = threadIdx.x; b < nm; b += blockDim.x) {
            s[0] += pm[b * 6 + 0];
            s[1] += pm[b * 6 + 1];
            s[2] += pm[b * 6 + 2];
            s[3] += pm[b * 6 + 3];
            s[7] = fmax(s[7], pm[b * 6 + 4]);
            s[8] += pm[b * 6 + 5];
        }
    }
    for (int c = 0; c < 9; ++c) sh[c][threadIdx.x] = s[c];
    block_tree<9>(sh, 7);
    if (threadIdx.x < 9) out[threadIdx.x] = sh[threadIdx.x][0];
}

// one block per row j: fixed-order sum over the tiles of the row
__global__ __launch_bounds__(256) void stats_read_kernel(const double *stats, int tpp,
                                                         double *prof) {
    const int j = blockIdx.x;
    __shared__ double sh[10][256];
    double s[10] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
    const double *row = stats + (long long)j * tpp * 10;
    for (int t = threadIdx.x; t < tpp; t += blockDim.x)
        for (int c = 0; c < 10; ++c) s[c] += row[t * 10 + c];
    for (int c = 0; c < 10; ++c) sh[c][threadIdx.x] = s[c];
    __syncthreads();
    for (int w = 128; w >= 1; w >>= 1) {
        if ((int)threadIdx.x < w)
            for (int c = 0; c < 10; ++c) sh[c][threadIdx.x] += sh[c][threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x < 10) prof[j * 10 + threadIdx.x] = sh[threadIdx.x][0];
}

__global__ __launch_bounds__(256) void fill_kernel(double *p, double v, size_t n) {
    const size_t x = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (x < n) p[x] = v;
}

}  // namespace

#define LBMX_DISPATCH(storage, CALL)                 \
    switch (storage) {                               \
    case ST_F64: { constexpr int S = ST_F64; CALL; } break;     \
    case ST_F32: { constexpr int S = ST_F32; CALL; } break;     \
    case ST_F16S: { constexpr int S = ST_F16S; CALL; } break;   \
    case ST_BF16S: { constexpr int S = ST_BF16S; CALL; } break; \
    case ST_BF16SR: { constexpr int S = ST_BF16SR; CALL; } break; \
    default: return hipErrorInvalidValue;            \
    }

// auxiliary kernels: the stochastically rounded type maps to BF16S
#define LBMX_DISPATCH_AUX(storage, CALL)                           \
    switch (aux_storage(storage)) {                                \
    case ST_F64: { constexpr int S = ST_F64; CALL; } break;       \
    case ST_F32: { constexpr int S = ST_F32; CALL; } break;       \
    case ST_F16S: { constexpr int S = ST_F16S; CALL; } break;     \
    case ST_BF16S: { constexpr int S = ST_BF16S; CALL; } break;   \
    default: return hipErrorInvalidValue;                          \
    }

static unsigned blocks_for(long long n) { return (unsigned)((n + 255) / 256); }

// compile-time variant from the launch flags (VAR_FX only without 64-bit
// addresses: a launch with both takes the general kernel)
#define LBMX_VARIANT(flags, CALL)                                                  \
    switch (((flags) & FLAG_FOREST ? VAR_FOREST : 0) |                             \
            ((flags) & FLAG_NUT_IN ? VAR_NUT_IN : 0) |                             \
            ((flags) & FLAG_WIDE ? VAR_WIDE : 0) |                                 \
            ((flags) & FLAG_STREAMING ? VAR_STREAM : 0) |                          \
            (((flags) & FLAG_FX) && !((flags) & FLAG_WIDE) ? VAR_FX : 0)) {        \
    case 0: { constexpr int V = 0; CALL; } break;                                  \
    case 1: { constexpr int V = 1; CALL; } break;                                  \
    case 2: { constexpr int V = 2; CALL; } break;                                  \
    case 3: { constexpr int V = 3; CALL; } break;                                  \
    case 4: { constexpr int V = 4; CALL; } break;                                  \
    case 5: { constexpr int V = 5; CALL; } break;                                  \
    case 6: { constexpr int V = 6; CALL; } break;                                  \
    case 7: { constexpr int V = 7; CALL; } break;                                  \
    case 8: { constexpr int V = 8; CALL; } break;                                  \
    case 9: { constexpr int V = 9; CALL; } break;                                  \
    case 10: { constexpr int V = 10; CALL; } break;                                \
    case 11: { constexpr int V = 11; CALL; } break;                                \
    case 12: { constexpr int V = 12; CALL; } break;                                \
    case 13: { constexpr int V = 13; CALL; } break;                                \
    case 14: { constexpr int V = 14; CALL; } break;                                \
    case 15: { constexpr int V = 15; CALL; } break;                                \
    case VAR_FX | 0: { constexpr int V = VAR_FX | 0; CALL; } break;                \
    case VAR_FX | 1: { constexpr int V = VAR_FX | 1; CALL; } break;                \
    case VAR_FX | 2: { constexpr int V = VAR_FX | 2; CALL; } break;                \
    case VAR_FX | 3: { constexpr int V = VAR_FX | 3; CALL; } break;                \
    case VAR_FX | 8: { constexpr int V = VAR_FX | 8; CALL; } break;                \
    case VAR_FX | 9: { constexpr int V = VAR_FX | 9; CALL; } break;                \
    case VAR_FX | 10: { constexpr int V = VAR_FX | 10; CALL; } break;              \
    default: { constexpr int V = VAR_FX | 11; CALL; } break;                       \
    }

// the learned-closure kernel's variants (it computes nu_t: never VAR_NUT_IN)
#define LBMX_VARIANT_MLP(flags, CALL)                                              \
    switch (((flags) & FLAG_FOREST ? VAR_FOREST : 0) |                             \
            ((flags) & FLAG_WIDE ? VAR_WIDE : 0) |                                 \
            (((flags) & FLAG_FX) && !((flags) & FLAG_WIDE) ? VAR_FX : 0)) {        \
    case 0: { constexpr int V = 0; CALL; } break;                                  \
    case VAR_FOREST: { constexpr int V = VAR_FOREST; CALL; } break;                \
    case VAR_WIDE: { constexpr int V = VAR_WIDE; CALL; } break;                    \
    case VAR_FOREST | VAR_WIDE: { constexpr int V = VAR_FOREST | VAR_WIDE; CALL; } break; \
    case VAR_FX: { constexpr int V = VAR_FX; CALL; } break;                        \
    default: { constexpr int V = VAR_FX | VAR_FOREST; CALL; } break;               \
    }

hipError_t launch_step(int storage, const StepArgs &a, int bx, int bz, hipStream_t s) {
    if (bx * bz != 256 || bx % 64 != 0 || a.ntiles < 1) return hipErrorInvalidValue;
    dim3 block(bx, bz), grid(a.ntiles);
    LBMX_DISPATCH(storage, LBMX_VARIANT(a.flags, hipLaunchKernelGGL((lbm_step_kernel<S, V>), grid,
                                                                    block, 0, s, a)));
    return hipGetLastError();
}

hipError_t mlp_launch_grid(int storage, int flags, int ntiles, int *grid) {
    int dev = 0, ncu = 0, per_cu = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return e;
    LBMX_DISPATCH(storage, LBMX_VARIANT_MLP(flags, e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
                               &per_cu, reinterpret_cast<const void *>(lbm_step_mlp_kernel<S, V>),
                               256, 0)));
    if (e != hipSuccess) return e;
    int g = (per_cu > 0 ? per_cu : 1) * ncu;
    g = g >= 8 ? g / 8 * 8 : g;
    if (g > ntiles) g = ntiles;
    *grid = g > 0 ? g : 1;
    return hipSuccess;
}

hipError_t launch_step_mlp(int storage, const StepArgs &a, int bx, int bz, int grid,
                           hipStream_t s) {
    if (bx * bz != 256 || bx % 64 != 0 || a.ntiles < 1 || a.mlp == nullptr || grid < 1 ||
        grid > a.ntiles)
        return hipErrorInvalidValue;
    if (a.flags & FLAG_NUT_IN) return hipErrorInvalidValue;  // the network computes nu_t
    LBMX_DISPATCH(storage, LBMX_VARIANT_MLP(a.flags, hipLaunchKernelGGL((lbm_step_mlp_kernel<S, V>),
                                                                        dim3(grid), dim3(bx, bz),
                                                                        0, s, a)));
    return hipGetLastError();
}

hipError_t launch_init(int storage, void *f, long long qs, int nx, int px, int ny, int zp,
                       void *mom, const double *rho, const double *u, int n, hipStream_t s) {
    LBMX_DISPATCH_AUX(storage, hipLaunchKernelGGL(init_kernel<S>, dim3(blocks_for(n)), dim3(256), 0,
                                              s, f, qs, nx, px, ny, zp, mom, rho, u, n));
    return hipGetLastError();
}

hipError_t launch_set_f(int storage, void *f, long long qs, const double *fin, int nx, int px,
                        int zp, int ny, int nz, int parity, int bc_lo, int bc_hi, hipStream_t s) {
    const long long n = (long long)nx * ny * nz;
    LBMX_DISPATCH_AUX(storage, hipLaunchKernelGGL(set_f_kernel<S>, dim3(blocks_for(n)), dim3(256), 0,
                                              s, f, qs, fin, nx, px, zp, ny, nz, parity, bc_lo,
                                              bc_hi));
    return hipGetLastError();
}

hipError_t launch_get_f(int storage, const void *f, long long qs, double *fout, int nx, int px,
                        int zp, int ny, int nz, int parity, int bc_lo, int bc_hi, hipStream_t s) {
    const long long n = (long long)nx * ny * nz;
    LBMX_DISPATCH_AUX(storage, hipLaunchKernelGGL(get_f_kernel<S>, dim3(blocks_for(n)), dim3(256), 0,
                                              s, f, qs, fout, nx, px, zp, ny, nz, parity, bc_lo,
                                              bc_hi));
    return hipGetLastError();
}

hipError_t launch_moments_out(int storage, const void *mom, double *rho, double *u,
                              double *nut, int n, hipStream_t s) {
    LBMX_DISPATCH_AUX(storage, hipLaunchKernelGGL(moments_out_kernel<S>, dim3(blocks_for(n)),
                                              dim3(256), 0, s, mom, rho, u, nut, n));
    return hipGetLastError();
}

hipError_t launch_diag(int storage, const void *mom, int n, const double *dg, const double *imp,
                       int nrec, double *red, double *out, hipStream_t s) {
    double *pm = nullptr;
    int nm = 0;
    if (!dg) {
        // the moment planes (after lbm_init): one pass over N cells
        const int chunk = (n + kDiagPlaneBlocks - 1) / kDiagPlaneBlocks;
        nm = (n + chunk - 1) / chunk;
        pm = red;
        LBMX_DISPATCH_AUX(storage, hipLaunchKernelGGL(diag_partial_kernel<S>, dim3(nm), dim3(256),
                                                  0, s, mom, n, chunk, pm));
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    double *ps = red + kDiagPlaneBlocks * 6;
    int nb = (nrec + 255) / 256;
    if (nb > kDiagRecordBlocks) nb = kDiagRecordBlocks;
    if (nb < 1) nb = 1;
    const int chunk = (nrec + nb - 1) / nb;
    nb = chunk > 0 ? (nrec + chunk - 1) / chunk : 1;
    hipLaunchKernelGGL(diag_records_kernel, dim3(nb), dim3(256), 0, s, dg, imp, nrec,
                       chunk > 0 ? chunk : 1, ps);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(diag_final_kernel, dim3(1), dim3(256), 0, s, ps, nb, pm, nm, out);
    return hipGetLastError();
}

hipError_t launch_stats_read(const double *stats, int ny, int tpp, double *prof,
                             hipStream_t s) {
    hipLaunchKernelGGL(stats_read_kernel, dim3(ny), dim3(256), 0, s, stats, tpp, prof);
    return hipGetLastError();
}

hipError_t launch_fill(double *p, double v, size_t n, hipStream_t s) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(fill_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, v, n);
    return hipGetLastError();
}

}  // namespace lbmx
