// The sweep at omega = 1 (tau_lb = 1) as a scalar stencil, for gfx950.
//
// With omega = 1 the collision forgets f_i: after any sweep the post-collision
// state is f*_i = phi_i Phi + chi_i S (Sec. 4 separable equilibrium and
// source), so the next sweep's moment is
//     Phi'(x) = sum_i phi_i Phi(x - v_i) + G(x),   G(x) = sum_i chi_i S(x - v_i)
// exactly.  The state shrinks from Q populations to one field, and one sweep
// moves 3 values per cell (read Phi, read G, write Phi') instead of 2Q + 1.
//
// Tiling: a 256-thread block owns TX x TY x TZ output cells and stages the
// tile plus its halo (the largest velocity component on each side, periodic
// wrap) in LDS.  Each thread computes CY cells along y; for every (dx, dz)
// offset pair it walks the needed LDS rows once and adds each value to every
// one of its CY outputs that uses it, so a staged value is read from LDS once
// per thread instead of once per output.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>

#include "device_common.hpp"
#include "kernels.hpp"
#include "stencil.hpp"
#include "lattices.hpp"

namespace lkp {
namespace stencil_detail {

using namespace dev;

// 1D and 2D: the block stages its whole tile plus halo (k_stencil).
template <int DIM> struct Tile;
template <> struct Tile<1> { static constexpr int TX = 256, TY = 1, TZ = 1, CY = 1; };
template <> struct Tile<2> { static constexpr int TX = 64, TY = 16, TZ = 1, CY = 4; };

template <int SM> struct SModeTraits;
template <> struct SModeTraits<SMODE_F64> {
  using TIN = double; using TOUT = double; using TSRC = double; using TC = double;
  static constexpr bool RESID = false;
};
template <> struct SModeTraits<SMODE_F32> {
  using TIN = float; using TOUT = float; using TSRC = float; using TC = float;
  static constexpr bool RESID = false;
};
template <> struct SModeTraits<SMODE_RESID> {
  using TIN = double; using TOUT = float; using TSRC = double; using TC = double;
  static constexpr bool RESID = true;
};

#pragma clang fp contract(off)

template <int LID, int SM, int FLAGS>
__global__ void __launch_bounds__(256) k_stencil(StencilParams p) {
  using L = Lattice<LID>;
  using MT = SModeTraits<SM>;
  using TIN = typename MT::TIN;
  using TOUT = typename MT::TOUT;
  using TSRC = typename MT::TSRC;
  using TC = typename MT::TC;
  using T = Tile<L::DIM>;
  constexpr int VMX = L::VMX, VMY = L::VMY, VMZ = L::VMZ;
  constexpr int LX = T::TX + 2 * VMX, LY = T::TY + 2 * VMY, LZ = T::TZ + 2 * VMZ;
  constexpr int NL = LX * LY * LZ;
  constexpr int RY = T::TY / T::CY;  // thread rows in y
  __shared__ TIN tile[NL];

  const unsigned nx = p.nx, ny = p.ny, nz = p.nz;
  const int x0 = (int)(blockIdx.x * T::TX), y0 = (int)(blockIdx.y * T::TY),
            z0 = (int)(blockIdx.z * T::TZ);
  const bool simple = p.simple_wrap != 0;
  const TIN *__restrict__ xin = reinterpret_cast<const TIN *>(p.xin);

  // stage the tile and its periodic halo
  for (int e = threadIdx.x; e < NL; e += 256) {
    const int lx = e % LX, ly = (e / LX) % LY, lz = e / (LX * LY);
    const unsigned gx = wrap_coord(0u, -(x0 + lx - VMX), nx, simple && nx > (unsigned)(T::TX + VMX));
    const unsigned gy = wrap_coord(0u, -(y0 + ly - VMY), ny, simple && ny > (unsigned)(T::TY + VMY));
    const unsigned gz = wrap_coord(0u, -(z0 + lz - VMZ), nz, simple && nz > (unsigned)(T::TZ + VMZ));
    tile[e] = xin[((size_t)gz * ny + gy) * nx + gx];
  }
  __syncthreads();

  const int tx = threadIdx.x % T::TX;
  const int ty = (threadIdx.x / T::TX) % RY;
  const int tz = threadIdx.x / (T::TX * RY);
  const int ly0 = ty * T::CY;  // first output row of this thread (tile coordinates)
  TC acc[T::CY];
#pragma unroll
  for (int k = 0; k < T::CY; ++k) acc[k] = (TC)0;

  // acc[k] += phi(v) * Phi(x_k - v): x_k - v sits at tile (tx + VMX - vx,
  // ly0 + k + VMY - vy, tz + VMZ - vz); walk row r = k + VMY - vy once.
  static_for<-VMX, VMX + 1>([&](auto DX) __attribute__((always_inline)) {
    static_for<-VMZ, VMZ + 1>([&](auto DZ) __attribute__((always_inline)) {
      constexpr int vx = (int)DX, vz = (int)DZ;
      static_for<0, T::CY + 2 * VMY>([&](auto R) __attribute__((always_inline)) {
        constexpr int r = (int)R;
        constexpr bool used = [] {
          for (int k = 0; k < T::CY; ++k) {
            const int vy = k + VMY - r;
            if (vy >= -VMY && vy <= VMY && L::vel(vx, vy, vz) >= 0) return true;
          }
          return false;
        }();
        if constexpr (used) {
          const TC v = (TC)tile[((tz + VMZ - vz) * LY + (ly0 + r)) * LX + (tx + VMX - vx)];
          static_for<0, T::CY>([&](auto K) __attribute__((always_inline)) {
            constexpr int k = (int)K;
            constexpr int vy = k + VMY - r;
            if constexpr (vy >= -VMY && vy <= VMY) {
              constexpr int i = L::vel(vx, vy, vz);
              if constexpr (i >= 0) {
                constexpr int o = L::orbit(i);
                TC c;
                if constexpr (sizeof(TC) == 8) c = (TC)p.coef.d[o];
                else c = (TC)p.coef.f[o];
                acc[k] = acc[k] + c * v;
              }
            }
          });
        }
      });
      // Compiler-only fence (emits nothing): the accumulators pass through it
      // and it clobbers memory, so this column's arithmetic cannot sink below
      // it and the next column's LDS reads cannot rise above it.  Without it
      // the scheduler issues every LDS read of the stencil first and spills
      // the staged values to scratch.
#pragma unroll
      for (int k = 0; k < T::CY; ++k) asm volatile("" : "+v"(acc[k]) : : "memory");
    });
  });

  double v[NUM_NORMS] = {0, 0, 0, 0, 0, 0};
  const TSRC *__restrict__ src = reinterpret_cast<const TSRC *>(p.src);
  TOUT *__restrict__ xout = reinterpret_cast<TOUT *>(p.xout);
  const int gx = x0 + tx, gz = z0 + tz;
#pragma unroll
  for (int k = 0; k < T::CY; ++k) {
    const int gy = y0 + ly0 + k;
    if (gx < (int)nx && gy < (int)ny && gz < (int)nz) {
      const size_t c = ((size_t)gz * ny + gy) * nx + gx;
      TC out = acc[k];
      if (src) out = out + (TC)src[c];
      const double centre = (double)tile[((tz + VMZ) * LY + (ly0 + k + VMY)) * LX + (tx + VMX)];
      if constexpr (MT::RESID) {
        const double r = (double)out - centre;  // R = A X + G - X
        xout[c] = (TOUT)r;
        if constexpr ((FLAGS & FLAG_REDUCE) != 0) {
          const bool ok = __builtin_isfinite(r) && __builtin_isfinite((double)out);
          v[NORM_SUM_R2] += ok ? r * r : 0.0;
          v[NORM_SUM_PHI2] += ok ? (double)out * (double)out : 0.0;
          v[NORM_SUM_PHI] += ok ? (double)out : 0.0;
          v[NORM_MAX_DPHI] = ok ? fmax(v[NORM_MAX_DPHI], fabs(r)) : v[NORM_MAX_DPHI];
          v[NORM_SUM_DPHI2] += ok ? r * r : 0.0;
          v[NORM_BAD] += ok ? 0.0 : 1.0;
        }
      } else {
        xout[c] = (TOUT)out;
        if constexpr ((FLAGS & FLAG_REDUCE) != 0) {
          const double o = (double)(TOUT)out;
          const double d = o - centre;
          const bool ok = __builtin_isfinite(o) && __builtin_isfinite(d);
          v[NORM_MAX_DPHI] = ok ? fmax(v[NORM_MAX_DPHI], fabs(d)) : v[NORM_MAX_DPHI];
          v[NORM_SUM_DPHI2] += ok ? d * d : 0.0;
          v[NORM_SUM_PHI2] += ok ? o * o : 0.0;
          v[NORM_SUM_PHI] += ok ? o : 0.0;
          v[NORM_BAD] += ok ? 0.0 : 1.0;
        }
      }
    }
  }
  if constexpr ((FLAGS & FLAG_REDUCE) != 0) {
    const unsigned blk = (blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x;
    block_norms(v, p.partials + (size_t)blk * NUM_NORMS);
  }
}

// 3D: a block owns a 64 x (4 CY) column of cells and marches through BZ
// output planes ((CY, BZ) one of the tile variants the runtime times).  Each input plane, with its x-y halo, is staged in LDS once
// and every staged value is pushed into the accumulators of all output planes
// that use it (z = z_in + vz for |vz| <= VMZ), which live in a register ring
// of 2 VMZ + 1 planes x CY rows.  Output plane m is complete once input plane
// m + VMZ has been consumed.  The next input plane is fetched into registers
// while the current one is consumed, and the products are fused
// multiply-adds.  For D3Q111 with CY = 2 an output cell costs 26 LDS reads
// (72.5 when a whole 32 x 8 x 4 tile plus halo is staged and read per
// z-offset) and staging reads 1.9 input values per output (5.2).
template <int SM> struct FmaT;
template <> struct FmaT<SMODE_F64> {
  static __device__ __forceinline__ double f(double a, double b, double c) { return __builtin_fma(a, b, c); }
};
template <> struct FmaT<SMODE_RESID> : FmaT<SMODE_F64> {};
template <> struct FmaT<SMODE_F32> {
  static __device__ __forceinline__ float f(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
};

__device__ __forceinline__ int pmod(int a, int n) {
  const int r = a % n;
  return r < 0 ? r + n : r;
}

// Which staged rows a thread reads for each x-offset, and the orbit weight
// (or -1) of every (x-offset, row, output row, z-offset) combination.
template <int LID, int CY>
struct Plan3 {
  using L = Lattice<LID>;
  static constexpr int NX = 2 * L::VMX + 1, NR = CY + 2 * L::VMY, NZ = 2 * L::VMZ + 1;
  struct Table {
    bool used[NX][NR];
    signed char orb[NX][NR][CY][NZ];
  };
  static constexpr Table make() {
    Table t{};
    for (int ix = 0; ix < NX; ++ix)
      for (int r = 0; r < NR; ++r) {
        t.used[ix][r] = false;
        for (int k = 0; k < CY; ++k)
          for (int iz = 0; iz < NZ; ++iz) {
            const int i = L::vel(ix - L::VMX, k + L::VMY - r, iz - L::VMZ);
            t.orb[ix][r][k][iz] = (signed char)(i >= 0 ? L::orbit(i) : -1);
            if (i >= 0) t.used[ix][r] = true;
          }
      }
    return t;
  }
  static constexpr Table t = make();
};

// Separable form for sets made of whole shells (every sign change of a
// velocity is in the set, with the same weight): the sum over a shell is a sum
// over its distinct component permutations (a, b, c) >= 0 of
//   S_c^z S_b^y S_a^x Phi,   S_d f(x) = f(x + d) + f(x - d) (d > 0), S_0 f = f.
// orb[a][b][c] is the weight (orbit) index of the permutation, or -1.
template <int LID>
struct SepPlan3 {
  using L = Lattice<LID>;
  static constexpr int AX = L::VMX, AY = L::VMY, AZ = L::VMZ;
  struct Table {
    signed char orb[AX + 1][AY + 1][AZ + 1];
    bool pair[AX + 1][AY + 1];
    bool closed;  // every sign change of every velocity is in the set, same orbit
  };
  static constexpr Table make() {
    Table t{};
    t.closed = true;
    for (int a = 0; a <= AX; ++a)
      for (int b = 0; b <= AY; ++b) {
        t.pair[a][b] = false;
        for (int c = 0; c <= AZ; ++c) {
          const int i = L::vel(a, b, c);
          t.orb[a][b][c] = (signed char)(i >= 0 ? L::orbit(i) : -1);
          if (i >= 0) t.pair[a][b] = true;
          for (int sg = 1; sg < 8; ++sg) {
            const int j = L::vel((sg & 1) ? -a : a, (sg & 2) ? -b : b, (sg & 4) ? -c : c);
            if ((i >= 0) != (j >= 0) || (i >= 0 && L::orbit(i) != L::orbit(j))) t.closed = false;
          }
        }
      }
    return t;
  }
  static constexpr Table t = make();
};

template <int LID, int SM, int FLAGS, int CY, int BZ, bool SEP>
__global__ void __launch_bounds__(256) k_stencil3(StencilParams p) {
  using Plan = Plan3<LID, CY>;
  using SP = SepPlan3<LID>;
  using L = Lattice<LID>;
  using MT = SModeTraits<SM>;
  using TIN = typename MT::TIN;
  using TOUT = typename MT::TOUT;
  using TSRC = typename MT::TSRC;
  using TC = typename MT::TC;
  constexpr int TX = 64, RY = 4, TY = RY * CY;
  constexpr int VMX = L::VMX, VMY = L::VMY, VMZ = L::VMZ;
  constexpr int NZR = 2 * VMZ + 1;
  constexpr int LX = TX + 2 * VMX, LY = TY + 2 * VMY, NL = LX * LY;
  constexpr int NST = (NL + 255) / 256;  // staging loads per thread and plane
  constexpr int NSTEPS = BZ + 2 * VMZ;   // input planes per block
  constexpr bool CENTRE = MT::RESID || (FLAGS & FLAG_REDUCE) != 0;
  static_assert(!SEP || SP::t.closed, "the separable form needs a set of whole shells");
  __shared__ TIN tile[2][NL];
  // separable form: S_a^x Phi of the current input plane, a = 1..VMX, on all
  // LY rows of the tile (no x halo)
  __shared__ TC xs[SEP ? VMX : 1][SEP ? TX * LY : 1];

  const int nx = (int)p.nx, ny = (int)p.ny, nz = (int)p.nz;
  // one linear grid; p.remap > 0 deals runs of p.remap consecutive blocks
  // (neighbours along x, then y) to one XCD, so the halos they share meet
  // in that XCD's L2
  const unsigned nb = gridDim.x;
  const unsigned lin = p.remap ? xcd_runs(blockIdx.x, nb, p.remap) : blockIdx.x;
  const unsigned bxi = lin % p.gbx, byi = (lin / p.gbx) % p.gby, bzi = lin / (p.gbx * p.gby);
  const int x0 = (int)bxi * TX, y0 = (int)byi * TY, z0 = (int)bzi * BZ;
  const unsigned pcells = (unsigned)nx * (unsigned)ny;
  const TIN *__restrict__ xin = reinterpret_cast<const TIN *>(p.xin);

  // in-plane offsets of this thread's staging elements (periodic wrap)
  unsigned soff[NST];
#pragma unroll
  for (int j = 0; j < NST; ++j) {
    const int e = (int)threadIdx.x + 256 * j;
    const int lx = e % LX, ly = e / LX;
    soff[j] = (e < NL) ? (unsigned)(pmod(y0 + ly - VMY, ny) * nx + pmod(x0 + lx - VMX, nx)) : 0u;
  }
  TIN pre[NST];
  auto fetch = [&](int step) {
    const unsigned base = (unsigned)pmod(z0 - VMZ + step, nz) * pcells;
#pragma unroll
    for (int j = 0; j < NST; ++j)
      if (j + 1 < NST || (int)threadIdx.x + 256 * j < NL) pre[j] = xin[base + soff[j]];
  };

  const int tx = threadIdx.x % TX;
  const int ly0 = (int)(threadIdx.x / TX) * CY;
  TC acc[NZR][CY];
  TC cen[CENTRE ? NZR : 1][CY];
#pragma unroll
  for (int j = 0; j < NZR; ++j)
#pragma unroll
    for (int k = 0; k < CY; ++k) acc[j][k] = (TC)0;

  double v[NUM_NORMS] = {0, 0, 0, 0, 0, 0};
  const TSRC *__restrict__ src = reinterpret_cast<const TSRC *>(p.src);
  TOUT *__restrict__ xout = reinterpret_cast<TOUT *>(p.xout);
  const int gx = x0 + tx;

  fetch(0);
  for (int s0 = 0; s0 < NSTEPS; s0 += NZR) {
    static_for<0, NZR>([&](auto PH) __attribute__((always_inline)) {
      constexpr int ph = (int)PH;
      const int step = s0 + ph;  // s0 is a multiple of NZR: ring slots are static
      if (step < NSTEPS) {       // block-uniform
        TIN *t = tile[step & 1];
#pragma unroll
        for (int j = 0; j < NST; ++j)
          if (j + 1 < NST || (int)threadIdx.x + 256 * j < NL) t[threadIdx.x + 256 * j] = pre[j];
        // source values of this step's output plane, loaded before the next
        // plane's prefetch (waiting for them must not wait for the prefetch)
        const int m = step - 2 * VMZ;
        const int gz = z0 + m;
        TC sv[CY];
#pragma unroll
        for (int k = 0; k < CY; ++k) {
          sv[k] = (TC)0;
          const int gy = y0 + ly0 + k;
          if (src && m >= 0 && gz < nz && gx < nx && gy < ny)
            sv[k] = (TC)src[((size_t)gz * ny + gy) * nx + gx];
        }
        __syncthreads();
        if (step + 1 < NSTEPS) fetch(step + 1);
        if constexpr (CENTRE) {
          constexpr int cs = ((ph - VMZ) % NZR + NZR) % NZR;  // output m = step - VMZ
#pragma unroll
          for (int k = 0; k < CY; ++k) cen[cs][k] = (TC)t[(ly0 + k + VMY) * LX + tx + VMX];
        }
        if constexpr (SEP) {
          // x sums of this plane for every tile row (rows dealt over the 4
          // row groups), then the block meets before the y sums read them
          const int rg = (int)(threadIdx.x / TX);
#pragma unroll
          for (int r0 = 0; r0 < LY; r0 += RY) {
            const int r = r0 + rg;
            if (r0 + RY <= LY || r < LY) {
              const TIN *row = t + r * LX + tx + VMX;
              static_for<1, VMX + 1>([&](auto A) __attribute__((always_inline)) {
                constexpr int a = (int)A;
                xs[a - 1][r * TX + tx] = (TC)row[a] + (TC)row[-a];
              });
            }
          }
          __syncthreads();
          constexpr int NR = CY + 2 * VMY;
          static_for<0, VMX + 1>([&](auto A) __attribute__((always_inline)) {
            constexpr int a = (int)A;
            TC col[NR];
#pragma unroll
            for (int r = 0; r < NR; ++r)
              col[r] = a == 0 ? (TC)t[(ly0 + r) * LX + tx + VMX] : xs[a == 0 ? 0 : a - 1][(ly0 + r) * TX + tx];
            static_for<0, VMY + 1>([&](auto B) __attribute__((always_inline)) {
              constexpr int b = (int)B;
              if constexpr (SP::t.pair[a][b]) {
#pragma unroll
                for (int k = 0; k < CY; ++k) {
                  const TC y = b == 0 ? col[k + VMY] : col[k + VMY + b] + col[k + VMY - b];
                  static_for<0, VMZ + 1>([&](auto Cz) __attribute__((always_inline)) {
                    constexpr int c = (int)Cz;
                    constexpr int o = SP::t.orb[a][b][c];
                    if constexpr (o >= 0) {
                      TC w;
                      if constexpr (sizeof(TC) == 8) w = (TC)p.coef.d[o];
                      else w = (TC)p.coef.f[o];
                      // input plane step feeds outputs m = step - VMZ + vz, vz = +-c
                      constexpr int sp = ((ph - VMZ + c) % NZR + NZR) % NZR;
                      acc[sp][k] = FmaT<SM>::f(w, y, acc[sp][k]);
                      if constexpr (c > 0) {
                        constexpr int sm = ((ph - VMZ - c) % NZR + NZR) % NZR;
                        acc[sm][k] = FmaT<SM>::f(w, y, acc[sm][k]);
                      }
                    }
                  });
                }
              }
            });
#pragma unroll
            for (int j = 0; j < NZR; ++j)
#pragma unroll
              for (int k = 0; k < CY; ++k) asm volatile("" : "+v"(acc[j][k]) : : "memory");
          });
        } else {
        // Columns of staged values (one x-offset each) are read one column
        // ahead: the LDS reads of column ix + 1 are in flight while the
        // multiply-adds of column ix run, so the LDS and the FP pipes overlap.
        constexpr int NR = CY + 2 * VMY;
        TC col[2][NR];
        auto read_col = [&](auto IXc) __attribute__((always_inline)) {
          constexpr int ix = (int)IXc;
#pragma unroll
          for (int r = 0; r < NR; ++r)
            if (Plan::t.used[ix][r]) col[ix & 1][r] = (TC)t[(ly0 + r) * LX + tx + 2 * VMX - ix];  // vx = ix - VMX
        };
        read_col(std::integral_constant<int, 0>{});
        static_for<0, 2 * VMX + 1>([&](auto IX) __attribute__((always_inline)) {
          constexpr int ix = (int)IX;
          if constexpr (ix + 1 < 2 * VMX + 1) read_col(std::integral_constant<int, ix + 1>{});
#pragma unroll
          for (int r = 0; r < NR; ++r) {
            if (Plan::t.used[ix][r]) {
              const TC val = col[ix & 1][r];
#pragma unroll
              for (int k = 0; k < CY; ++k)
#pragma unroll
                for (int iz = 0; iz < NZR; ++iz) {
                  const int o = Plan::t.orb[ix][r][k][iz];
                  if (o >= 0) {
                    const int slot = (ph + iz - 2 * VMZ + 2 * NZR) % NZR;  // m = step + vz - VMZ
                    TC c;
                    if constexpr (sizeof(TC) == 8) c = (TC)p.coef.d[o];
                    else c = (TC)p.coef.f[o];
                    acc[slot][k] = FmaT<SM>::f(c, val, acc[slot][k]);
                  }
                }
            }
          }
          // compiler-only fence: at most two columns of staged values live,
          // and the reads of the column after next stay below this point
#pragma unroll
          for (int j = 0; j < NZR; ++j)
#pragma unroll
            for (int k = 0; k < CY; ++k) asm volatile("" : "+v"(acc[j][k]) : : "memory");
        });
        }
        // output plane m = step - 2 VMZ is complete
        constexpr int fs = (ph + 1) % NZR;
        if (m >= 0 && gz < nz) {
#pragma unroll
          for (int k = 0; k < CY; ++k) {
            const int gy = y0 + ly0 + k;
            if (gx < nx && gy < ny) {
              const size_t c = ((size_t)gz * ny + gy) * nx + gx;
              TC out = acc[fs][k];
              if (src) out = out + sv[k];
              if constexpr (MT::RESID) {
                const double r = (double)out - (double)cen[fs][k];  // R = A X + G - X
                xout[c] = (TOUT)r;
                if constexpr ((FLAGS & FLAG_REDUCE) != 0) {
                  const bool ok = __builtin_isfinite(r) && __builtin_isfinite((double)out);
                  v[NORM_SUM_R2] += ok ? r * r : 0.0;
                  v[NORM_SUM_PHI2] += ok ? (double)out * (double)out : 0.0;
                  v[NORM_SUM_PHI] += ok ? (double)out : 0.0;
                  v[NORM_MAX_DPHI] = ok ? fmax(v[NORM_MAX_DPHI], fabs(r)) : v[NORM_MAX_DPHI];
                  v[NORM_SUM_DPHI2] += ok ? r * r : 0.0;
                  v[NORM_BAD] += ok ? 0.0 : 1.0;
                }
              } else {
                xout[c] = (TOUT)out;
                if constexpr ((FLAGS & FLAG_REDUCE) != 0) {
                  const double o = (double)(TOUT)out;
                  const double d = o - (double)cen[fs][k];
                  const bool ok = __builtin_isfinite(o) && __builtin_isfinite(d);
                  v[NORM_MAX_DPHI] = ok ? fmax(v[NORM_MAX_DPHI], fabs(d)) : v[NORM_MAX_DPHI];
                  v[NORM_SUM_DPHI2] += ok ? d * d : 0.0;
                  v[NORM_SUM_PHI2] += ok ? o * o : 0.0;
                  v[NORM_SUM_PHI] += ok ? o : 0.0;
                  v[NORM_BAD] += ok ? 0.0 : 1.0;
                }
              }
            }
          }
        }
#pragma unroll
        for (int k = 0; k < CY; ++k) acc[fs][k] = (TC)0;
      }
    });
  }
  if constexpr ((FLAGS & FLAG_REDUCE) != 0) block_norms(v, p.partials + (size_t)lin * NUM_NORMS);
}

// Two adjacent values, read or written as one 2-element access (16 bytes in
// FP64: one ds_read_b128 from LDS).
template <class T>
struct alignas(2 * sizeof(T)) Pair2 {
  T a, b;
};

// The plane sums of one staged input plane for a thread's two adjacent x
// cells on CY rows: T[c][k][q] = sum_{a,b} w[a,b,c] S_b^y S_a^x Phi at output
// row k, cell q (rows in y order, then a in order).  `row0` points at the
// staged value x0 + 2 ip - VMX - XS of the thread's first row (row r of the
// staged plane at row0 + r PITCH); XS = 1 when the rows were staged from one
// cell further left (an even x origin), so that the 2-element reads stay
// aligned.  Rows are read one ahead: the reads of row r + 1 are in flight
// while row r's multiply-adds run.
template <int LID, int SM, int CY, int PITCH, int XS, class TIN, class TC>
__device__ __forceinline__ void plane_sums(const TIN *row0, const StencilParams &p,
                                           TC (&T)[Lattice<LID>::VMZ + 1][CY][2]) {
  using SP = SepPlan3<LID>;
  using L = Lattice<LID>;
  constexpr int VMX = L::VMX, VMY = L::VMY, VMZ = L::VMZ;
  constexpr int SEG = 2 + 2 * VMX;      // values around a cell pair
  constexpr int NP = (SEG + XS + 1) / 2;  // 2-element reads per row
  constexpr int NR = CY + 2 * VMY;      // staged rows a thread reads
#pragma unroll
  for (int c = 0; c <= VMZ; ++c)
#pragma unroll
    for (int k = 0; k < CY; ++k) T[c][k][0] = T[c][k][1] = (TC)0;
  TIN seg[2][2 * NP];
  auto read_row = [&](auto Rc) __attribute__((always_inline)) {
    constexpr int r = (int)Rc;
#pragma unroll
    for (int e = 0; e < NP; ++e) {
      const Pair2<TIN> q = *reinterpret_cast<const Pair2<TIN> *>(row0 + r * PITCH + 2 * e);
      seg[r & 1][2 * e] = q.a;
      seg[r & 1][2 * e + 1] = q.b;
    }
  };
  read_row(std::integral_constant<int, 0>{});
  static_for<0, NR>([&](auto R) __attribute__((always_inline)) {
    constexpr int r = (int)R;
    if constexpr (r + 1 < NR) read_row(std::integral_constant<int, r + 1>{});
    // x sums of the two cells: X[a][q] = S_a^x Phi at cell q
    TC X[VMX + 1][2];
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      X[0][q] = (TC)seg[r & 1][XS + VMX + q];
#pragma unroll
      for (int a = 1; a <= VMX; ++a)
        X[a][q] = (TC)seg[r & 1][XS + VMX + q + a] + (TC)seg[r & 1][XS + VMX + q - a];
    }
    static_for<0, CY>([&](auto K) __attribute__((always_inline)) {
      constexpr int k = (int)K;
      constexpr int dy = r - VMY - k;  // y offset of this row for output row k
      constexpr int b = dy < 0 ? -dy : dy;
      if constexpr (b <= VMY) {
        static_for<0, VMZ + 1>([&](auto Cz) __attribute__((always_inline)) {
          constexpr int c = (int)Cz;
          static_for<0, VMX + 1>([&](auto A) __attribute__((always_inline)) {
            constexpr int a = (int)A;
            constexpr int o = SP::t.orb[a][b][c];
            if constexpr (o >= 0) {
              TC w;
              if constexpr (sizeof(TC) == 8) w = (TC)p.coef.d[o];
              else w = (TC)p.coef.f[o];
              T[c][k][0] = FmaT<SM>::f(w, X[a][0], T[c][k][0]);
              T[c][k][1] = FmaT<SM>::f(w, X[a][1], T[c][k][1]);
            }
          });
        });
      }
    });
    // compiler-only fence: at most two staged rows live
#pragma unroll
    for (int c = 0; c <= VMZ; ++c)
#pragma unroll
      for (int k = 0; k < CY; ++k) asm volatile("" : "+v"(T[c][k][0]), "+v"(T[c][k][1]) : : "memory");
  });
}

// Store a thread's finished output cells (two adjacent x cells on CY rows of
// one plane): Phi' = acc + src, or R = acc + src - centre in SMODE_RESID, and
// on check sweeps add their norms to v.  Cell offsets are 32-bit (grids stay
// below 2^29 cells): `plane` is the plane's first cell (block-uniform) and
// `cell0` the thread's first cell within the plane, gy0 nx + gx.
template <int SM, int FLAGS, int CY, class TC, class TOUT>
__device__ __forceinline__ void emit_rows(const TC (&acc)[CY][2], const TC (&sv)[CY][2],
                                          const TC (&cv)[CY][2], bool has_src, TOUT *xout,
                                          unsigned plane, unsigned cell0, int gy0, int gx, int nx,
                                          int ny, double (&v)[NUM_NORMS]) {
  using MT = SModeTraits<SM>;
#pragma unroll
  for (int k = 0; k < CY; ++k) {
    const int gy = gy0 + k;
    if (gy < ny) {
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        if (gx + q < nx) {
          const unsigned c = cell0 + (plane + (unsigned)(k * nx)) + (unsigned)q;
          TC out = acc[k][q];
          if (has_src) out = out + sv[k][q];
          const TC centre = cv[k][q];
          if constexpr (MT::RESID) {
            const double r = (double)out - (double)centre;  // R = A X + G - X
            xout[c] = (TOUT)r;
            if constexpr ((FLAGS & FLAG_REDUCE) != 0) {
              const bool ok = __builtin_isfinite(r) && __builtin_isfinite((double)out);
              v[NORM_SUM_R2] += ok ? r * r : 0.0;
              v[NORM_SUM_PHI2] += ok ? (double)out * (double)out : 0.0;
              v[NORM_SUM_PHI] += ok ? (double)out : 0.0;
              v[NORM_MAX_DPHI] = ok ? fmax(v[NORM_MAX_DPHI], fabs(r)) : v[NORM_MAX_DPHI];
              v[NORM_SUM_DPHI2] += ok ? r * r : 0.0;
              v[NORM_BAD] += ok ? 0.0 : 1.0;
            }
          } else {
            xout[c] = (TOUT)out;
            if constexpr ((FLAGS & FLAG_REDUCE) != 0) {
              const double o = (double)(TOUT)out;
              const double d = o - (double)centre;
              const bool ok = __builtin_isfinite(o) && __builtin_isfinite(d);
              v[NORM_MAX_DPHI] = ok ? fmax(v[NORM_MAX_DPHI], fabs(d)) : v[NORM_MAX_DPHI];
              v[NORM_SUM_DPHI2] += ok ? d * d : 0.0;
              v[NORM_SUM_PHI2] += ok ? o * o : 0.0;
              v[NORM_SUM_PHI] += ok ? o : 0.0;
              v[NORM_BAD] += ok ? 0.0 : 1.0;
            }
          }
        }
      }
    }
  }
}

// Plane-sum form of the 3D stencil for sets of whole shells.  With
// S_d f(x) = f(x + d) + f(x - d) (S_0 f = f) the stencil is
//   Phi'(z) = sum_c S_c^z T_c,   T_c = sum_{a,b} w[a,b,c] S_b^y S_a^x Phi,
// and T_c of one input plane serves the outputs at z +- c.  A block owns
// 64 x (8 CY) x BZ output cells; a thread owns two adjacent x cells on CY
// rows.  Per staged input plane it reads, for each of its CY + 2 VMY rows,
// the 2 + 2 VMX values around its pair with 2-element LDS reads, forms the
// x sums in registers, and accumulates T_c for its cells (rows in y order,
// then a in order), so a plane costs one barrier and about half the LDS bytes
// of the separable form.  The output ring then takes T_0 into plane z and
// T_c into planes z +- c, input planes in z order.  The summation order of
// every output cell is the same for every CY and BZ, so the variants of this
// family give the same bits; it rounds differently from the other families.
template <int LID, int SM, int FLAGS, int CY, int BZ>
__global__ void __launch_bounds__(256) k_stencil3p(StencilParams p) {
  // planes fetched ahead into registers (two, with the unroll that needs,
  // pushed the FP64 variants past 256 VGPRs)
  constexpr int PD = 1;
  using SP = SepPlan3<LID>;
  using L = Lattice<LID>;
  using MT = SModeTraits<SM>;
  using TIN = typename MT::TIN;
  using TOUT = typename MT::TOUT;
  using TSRC = typename MT::TSRC;
  using TC = typename MT::TC;
  constexpr int VMX = L::VMX, VMY = L::VMY, VMZ = L::VMZ;
  constexpr int TX = 64, NG = 8, TY = NG * CY;  // 32 cell pairs x 8 row groups
  constexpr int NZR = 2 * VMZ + 1;
  constexpr int LX = TX + 2 * VMX, LY = TY + 2 * VMY, NL = LX * LY;
  constexpr int NST = (NL + 255) / 256;
  constexpr int NSTEPS = BZ + 2 * VMZ;
  constexpr bool CENTRE = MT::RESID || (FLAGS & FLAG_REDUCE) != 0;
  static_assert(SP::t.closed, "the plane-sum form needs a set of whole shells");
  static_assert(LX % 2 == 0 && NL % 2 == 0, "2-element LDS reads need even rows");
  __shared__ __align__(16) TIN tile[2][NL];

  const int nx = (int)p.nx, ny = (int)p.ny, nz = (int)p.nz;
  const unsigned nb = gridDim.x;
  const unsigned lin = p.remap ? xcd_runs(blockIdx.x, nb, p.remap) : blockIdx.x;
  const unsigned bxi = lin % p.gbx, byi = (lin / p.gbx) % p.gby, bzi = lin / (p.gbx * p.gby);
  const int x0 = (int)bxi * TX, y0 = (int)byi * TY, z0 = (int)bzi * BZ;
  const unsigned pcells = (unsigned)nx * (unsigned)ny;
  const TIN *__restrict__ xin = reinterpret_cast<const TIN *>(p.xin);

  unsigned soff[NST];
#pragma unroll
  for (int j = 0; j < NST; ++j) {
    const int e = (int)threadIdx.x + 256 * j;
    const int lx = e % LX, ly = e / LX;
    soff[j] = (e < NL) ? (unsigned)(pmod(y0 + ly - VMY, ny) * nx + pmod(x0 + lx - VMX, nx)) : 0u;
  }
  // PD register sets of prefetched planes: plane `step` sits in set step % PD
  TIN pre[PD][NST];
  auto fetch = [&](auto PIc, int step) __attribute__((always_inline)) {
    constexpr int pi = (int)PIc;
    const unsigned base = (unsigned)pmod(z0 - VMZ + step, nz) * pcells;
#pragma unroll
    for (int j = 0; j < NST; ++j)
      if (j + 1 < NST || (int)threadIdx.x + 256 * j < NL) pre[pi][j] = xin[base + soff[j]];
  };

  const int ip = (int)(threadIdx.x % 32);  // cell pair
  const int g = (int)(threadIdx.x / 32);   // row group
  const int gx = x0 + 2 * ip;
  const unsigned cell0 = (unsigned)((y0 + g * CY) * nx + gx);  // first cell of the thread's rows
  TC acc[NZR][CY][2];
#pragma unroll
  for (int j = 0; j < NZR; ++j)
#pragma unroll
    for (int k = 0; k < CY; ++k) acc[j][k][0] = acc[j][k][1] = (TC)0;

  double v[NUM_NORMS] = {0, 0, 0, 0, 0, 0};
  const TSRC *__restrict__ src = reinterpret_cast<const TSRC *>(p.src);
  TOUT *__restrict__ xout = reinterpret_cast<TOUT *>(p.xout);

  static_for<0, PD>([&](auto PI) __attribute__((always_inline)) {
    if ((int)PI < NSTEPS) fetch(PI, (int)PI);
  });
  // steps unrolled by NZR * PD: ring slots and prefetch sets are static
  for (int s0 = 0; s0 < NSTEPS; s0 += NZR * PD) {
    static_for<0, NZR * PD>([&](auto PHX) __attribute__((always_inline)) {
      constexpr int ph = (int)PHX % NZR;
      constexpr int pi = (int)PHX % PD;
      const int step = s0 + (int)PHX;
      if (step < NSTEPS) {  // block-uniform
        TIN *t = tile[step & 1];
#pragma unroll
        for (int j = 0; j < NST; ++j)
          if (j + 1 < NST || (int)threadIdx.x + 256 * j < NL) t[threadIdx.x + 256 * j] = pre[pi][j];
        // the source (and centre) values of this step's output plane are
        // loaded before the next plane's prefetch, so that waiting for them
        // at the output does not also wait for the prefetch
        const int m = step - 2 * VMZ;
        const int gz = z0 + m;
        const bool emit = m >= 0 && gz < nz;
        const unsigned plane = (unsigned)gz * pcells;
        TC sv[CY][2], cv[CY][2];
#pragma unroll
        for (int k = 0; k < CY; ++k)
#pragma unroll
          for (int q = 0; q < 2; ++q) {
            sv[k][q] = cv[k][q] = (TC)0;
            const int gy = y0 + g * CY + k;
            if (emit && gy < ny && gx + q < nx) {
              const unsigned c = cell0 + (plane + (unsigned)(k * nx)) + (unsigned)q;
              // an FP64 source is read once per sweep: the nontemporal hint
              // leaves the caches to Phi, whose output the next sweep reads back
              // (2 % on the FP64 sweep; on 4-byte FP32 loads it cost 15 %)
              if (src) {
                if constexpr (sizeof(TSRC) == 8) sv[k][q] = (TC)__builtin_nontemporal_load(src + c);
                else sv[k][q] = (TC)src[c];
              }
              if constexpr (CENTRE) cv[k][q] = (TC)xin[c];
            }
          }
        // the next plane's loads go out before the barrier: they only write
        // registers, and the barrier's wait adds to their time to arrive
        if (step + PD < NSTEPS) fetch(std::integral_constant<int, pi>{}, step + PD);
        __syncthreads();

        TC T[VMZ + 1][CY][2];
        plane_sums<LID, SM, CY, LX, 0>(t + g * CY * LX + 2 * ip, p, T);
        // input plane `step` feeds outputs m = step - VMZ + c and step - VMZ - c
        static_for<0, VMZ + 1>([&](auto Cz) __attribute__((always_inline)) {
          constexpr int c = (int)Cz;
          constexpr int sp = ((ph - VMZ + c) % NZR + NZR) % NZR;
#pragma unroll
          for (int k = 0; k < CY; ++k) {
            acc[sp][k][0] = acc[sp][k][0] + T[c][k][0];
            acc[sp][k][1] = acc[sp][k][1] + T[c][k][1];
          }
          if constexpr (c > 0) {
            constexpr int sm = ((ph - VMZ - c) % NZR + NZR) % NZR;
#pragma unroll
            for (int k = 0; k < CY; ++k) {
              acc[sm][k][0] = acc[sm][k][0] + T[c][k][0];
              acc[sm][k][1] = acc[sm][k][1] + T[c][k][1];
            }
          }
        });
        // output plane m = step - 2 VMZ is complete
        constexpr int fs = (ph + 1) % NZR;
        if (emit)
          emit_rows<SM, FLAGS, CY>(acc[fs], sv, cv, src != nullptr, xout, plane, cell0, y0 + g * CY,
                                   gx, nx, ny, v);
#pragma unroll
        for (int k = 0; k < CY; ++k) acc[fs][k][0] = acc[fs][k][1] = (TC)0;
      }
    });
  }
  if constexpr ((FLAGS & FLAG_REDUCE) != 0) block_norms(v, p.partials + (size_t)lin * NUM_NORMS);
}

// s_waitcnt that waits until at most N vector-memory operations of this wave
// are in flight (lgkm and exp counters left alone); wait_vm_n takes N at run
// time (wave-uniform, at most NMAX).
template <int N>
__device__ __forceinline__ void wait_vm() {
  static_assert(N >= 0 && N < 64, "vmcnt range");
  __builtin_amdgcn_s_waitcnt((N & 15) | ((N >> 4) << 14) | (7 << 4) | (15 << 8));
}
template <int NMAX>
__device__ __forceinline__ void wait_vm_n(int n) {
  bool done = false;
  static_for<0, NMAX + 1>([&](auto I) __attribute__((always_inline)) {
    if (!done && n == (int)I) {
      wait_vm<(int)I>();
      done = true;
    }
  });
  if (!done) wait_vm<0>();
}

// Requests of one block for a field of T: NU 16-byte units per lane-slot
// table, every lane issuing the same NR = ceil(NU / 256) direct
// global-to-LDS loads (lanes past the last unit repeat it into the buffer's
// tail), so that every wave has the same number of loads in flight.
template <class T, int NU>
struct LdsRows {
  static constexpr int E = 16 / (int)sizeof(T);  // elements per unit
  static constexpr int NR = (NU + 255) / 256;    // loads per lane
  static constexpr int SLOT = NR * 256 * E;      // elements per buffer
  unsigned off[NR];                              // element offset within a plane
  __device__ __forceinline__ void request(const T *plane, T *buf, int wv) const {
    using LdsPtr = __attribute__((address_space(3))) void *;
    using GlobalPtr = const __attribute__((address_space(1))) void *;
    T *dst = buf + 64 * wv * E;
#pragma unroll
    for (int j = 0; j < NR; ++j)
      __builtin_amdgcn_global_load_lds((GlobalPtr)(plane + off[j]), (LdsPtr)(dst + 256 * j * E), 16, 0,
                                       0);
  }
};

// Plane-sum form with every load a direct global-to-LDS load: NB input planes
// are in LDS or in flight at once (plane step + NB - 1 is requested while
// plane step is summed, so a request has NB - 1 steps' work to arrive instead
// of one), and the source (and centre) rows of each output plane travel the
// same way, NB - 1 steps ahead of their use.  No register waits on a global
// load, so the only waits are the ones below: before step t, for plane t and
// everything requested before it, counting the requests issued after it (a
// wave's vector-memory operations complete in issue order).  Input rows are
// staged from the x origin x0 - VXA (VMX rounded up to whole 16-byte units)
// so that every unit is aligned and none straddles the periodic seam; the
// variant needs nx to be a multiple of a unit's elements.  A step stores the
// previous step's outputs before it requests anything, so the stores never
// enter the count.  The arithmetic is k_stencil3p's (same helpers, same
// order): the variants of both give the same bits.
template <int LID, int SM, int FLAGS, int CY, int BZ, int NB>
__global__ void __launch_bounds__(256) k_stencil3pa(StencilParams p) {
  using SP = SepPlan3<LID>;
  using L = Lattice<LID>;
  using MT = SModeTraits<SM>;
  using TIN = typename MT::TIN;
  using TOUT = typename MT::TOUT;
  using TSRC = typename MT::TSRC;
  using TC = typename MT::TC;
  constexpr int VMX = L::VMX, VMY = L::VMY, VMZ = L::VMZ;
  constexpr int TX = 64, NG = 8, TY = NG * CY;  // 32 cell pairs x 8 row groups
  constexpr int NZR = 2 * VMZ + 1;
  constexpr int E = 16 / (int)sizeof(TIN);     // input elements per unit
  constexpr int ES = 16 / (int)sizeof(TSRC);   // source elements per unit
  constexpr int VXA = (VMX + E - 1) / E * E;    // x halo in whole units
  // a staged row holds TX + 2 VXA cells and one unit more, so that the two
  // row groups of a wave (2 CY rows apart) read different LDS banks
  constexpr int RU = (TX + 2 * VXA) / E + 1;    // units per staged input row
  constexpr int PITCH = RU * E;                 // staged input row (elements)
  constexpr int LY = TY + 2 * VMY;
  constexpr int XS = VXA - VMX;                 // staged cells left of the halo
  constexpr int NSTEPS = BZ + 2 * VMZ;
  constexpr bool CENTRE = MT::RESID || (FLAGS & FLAG_REDUCE) != 0;
  using InRows = LdsRows<TIN, RU * LY>;
  using SrcRows = LdsRows<TSRC, TX * TY / ES>;
  using CenRows = LdsRows<TIN, TX * TY / E>;
  constexpr int NIN = InRows::NR;                                 // loads per input plane
  constexpr int NOUT = SrcRows::NR + (CENTRE ? CenRows::NR : 0);  // loads per output plane
  constexpr int KMAX = (NB - 2) * (NIN + NOUT);
  static_assert(SP::t.closed, "the plane-sum form needs a set of whole shells");
  static_assert(NB >= 3 && KMAX < 64, "three or more buffers; vmcnt range");
  static_assert(2 * VMZ >= NB - 1, "no output plane is requested before the loop");
  __shared__ __align__(16) TIN tile[NB][InRows::SLOT];
  __shared__ __align__(16) TSRC sbuf[NB][SrcRows::SLOT];
  __shared__ __align__(16) TIN cbuf[CENTRE ? NB : 1][CENTRE ? CenRows::SLOT : 4];

  const int nx = (int)p.nx, ny = (int)p.ny, nz = (int)p.nz;
  const unsigned nb = gridDim.x;
  const unsigned lin = p.remap ? xcd_runs(blockIdx.x, nb, p.remap) : blockIdx.x;
  const unsigned bxi = lin % p.gbx, byi = (lin / p.gbx) % p.gby, bzi = lin / (p.gbx * p.gby);
  const int x0 = (int)bxi * TX, y0 = (int)byi * TY, z0 = (int)bzi * BZ;
  const unsigned pcells = (unsigned)nx * (unsigned)ny;
  const TIN *__restrict__ xin = reinterpret_cast<const TIN *>(p.xin);
  // without a source field the source loads read Phi (ignored), so that the
  // count of loads per step stays the same
  const TSRC *__restrict__ src = reinterpret_cast<const TSRC *>(p.src ? p.src : p.xin);
  const bool has_src = p.src != nullptr;
  TOUT *__restrict__ xout = reinterpret_cast<TOUT *>(p.xout);
  const int wv = __builtin_amdgcn_readfirstlane((int)threadIdx.x >> 6);

  // input unit u: staged row u / RU, x = x0 - VXA + E (u % RU), rows and
  // columns wrapped (the last unit of a row is padding, never read)
  InRows in;
#pragma unroll
  for (int j = 0; j < NIN; ++j) {
    const int u = min((int)threadIdx.x + 256 * j, RU * LY - 1);
    in.off[j] = (unsigned)(pmod(y0 + u / RU - VMY, ny) * nx + pmod(x0 - VXA + E * (u % RU), nx));
  }
  // output unit u: row u / (TX / ES) of the tile, x = x0 + ES (u % (TX / ES));
  // rows and columns past the grid wrap (their values are never used)
  SrcRows so;
#pragma unroll
  for (int j = 0; j < SrcRows::NR; ++j) {
    const int u = min((int)threadIdx.x + 256 * j, TX * TY / ES - 1);
    so.off[j] = (unsigned)(pmod(y0 + u / (TX / ES), ny) * nx + pmod(x0 + ES * (u % (TX / ES)), nx));
  }
  CenRows co;
  if constexpr (CENTRE) {
#pragma unroll
    for (int j = 0; j < CenRows::NR; ++j) {
      const int u = min((int)threadIdx.x + 256 * j, TX * TY / E - 1);
      co.off[j] = (unsigned)(pmod(y0 + u / (TX / E), ny) * nx + pmod(x0 + E * (u % (TX / E)), nx));
    }
  }
  // input plane j (z = z0 - VMZ + j) goes to tile[j % NB]; the source and
  // centre rows of step t's output plane (z = z0 + t - 2 VMZ) to sbuf[t % NB]
  auto request_in = [&](int j) __attribute__((always_inline)) {
    in.request(xin + (size_t)pmod(z0 - VMZ + j, nz) * pcells, tile[j % NB], wv);
  };
  auto request_out = [&](int t) __attribute__((always_inline)) {
    const size_t base = (size_t)pmod(z0 + t - 2 * VMZ, nz) * pcells;
    so.request(src + base, sbuf[t % NB], wv);
    if constexpr (CENTRE) co.request(xin + base, cbuf[t % NB], wv);
  };
  // output rows of step t are requested with input plane t + 1, in the step
  // t + 2 - NB, before it: both have landed once plane t + 1 has
  auto out_requested = [](int t) { return t >= 2 * VMZ && t <= NSTEPS - 1; };

  const int ip = (int)(threadIdx.x % 32);  // cell pair
  const int g = (int)(threadIdx.x / 32);   // row group
  const int gx = x0 + 2 * ip;
  const unsigned cell0 = (unsigned)((y0 + g * CY) * nx + gx);  // first cell of the thread's rows
  TC acc[NZR][CY][2];
#pragma unroll
  for (int j = 0; j < NZR; ++j)
#pragma unroll
    for (int k = 0; k < CY; ++k) acc[j][k][0] = acc[j][k][1] = (TC)0;
  double v[NUM_NORMS] = {0, 0, 0, 0, 0, 0};

  // outputs of step t (ring slot `slot`), their source and centre from LDS
  auto emit = [&](auto SLOTc, int t) __attribute__((always_inline)) {
    constexpr int slot = (int)SLOTc;
    const int m = t - 2 * VMZ;
    if (m >= 0 && z0 + m < nz) {
      TC sv[CY][2], cv[CY][2];
#pragma unroll
      for (int k = 0; k < CY; ++k) {
        const int e = (g * CY + k) * TX + 2 * ip;
        const Pair2<TSRC> q = *reinterpret_cast<const Pair2<TSRC> *>(sbuf[t % NB] + e);
        sv[k][0] = (TC)q.a;
        sv[k][1] = (TC)q.b;
        cv[k][0] = cv[k][1] = (TC)0;
        if constexpr (CENTRE) {
          const Pair2<TIN> c = *reinterpret_cast<const Pair2<TIN> *>(cbuf[t % NB] + e);
          cv[k][0] = (TC)c.a;
          cv[k][1] = (TC)c.b;
        }
      }
      emit_rows<SM, FLAGS, CY>(acc[slot], sv, cv, has_src, xout, (unsigned)(z0 + m) * pcells, cell0,
                               y0 + g * CY, gx, nx, ny, v);
    }
#pragma unroll
    for (int k = 0; k < CY; ++k) acc[slot][k][0] = acc[slot][k][1] = (TC)0;
  };

  // the last input plane, opaque to the compiler: every request stays behind
  // a branch, where it does not make the compiler wait for all loads in
  // flight before the next LDS reads (the explicit waits order them)
  int last_plane = NSTEPS - 1;
  asm volatile("" : "+s"(last_plane));
  static_for<0, NB - 1>([&](auto K) __attribute__((always_inline)) {
    if ((int)K <= last_plane) request_in((int)K);
  });
  for (int s0 = 0; s0 < NSTEPS; s0 += NZR) {
    static_for<0, NZR>([&](auto PHX) __attribute__((always_inline)) {
      constexpr int ph = (int)PHX;
      const int step = s0 + ph;
      if (step < NSTEPS) {  // block-uniform
        // plane `step` (and the output rows of step - 1) have landed once
        // only the loads issued after it are left: steps step + 1 - NB + j,
        // j = 1 .. NB - 2, issued output rows of step - 1 + j and plane
        // step + j
        int later = 0;
#pragma unroll
        for (int j = 1; j <= NB - 2; ++j)
          later += (out_requested(step - 1 + j) ? NOUT : 0) + (step + j <= NSTEPS - 1 ? NIN : 0);
        wait_vm_n<KMAX>(later);
        asm volatile("" ::: "memory");
        __builtin_amdgcn_s_barrier();
        asm volatile("" ::: "memory");
        // outputs finished by the previous step (ring slot ph; none at step 0)
        emit(std::integral_constant<int, ph>{}, step - 1);
        // the buffers written next were last read in the previous step,
        // which every wave has finished (barrier above)
        if (out_requested(step + NB - 2)) request_out(step + NB - 2);
        if (step + NB - 1 <= last_plane) request_in(step + NB - 1);

        TC T[VMZ + 1][CY][2];
        plane_sums<LID, SM, CY, PITCH, XS & 1>(tile[step % NB] + g * CY * PITCH + 2 * ip + (XS & ~1),
                                               p, T);
        // input plane `step` feeds outputs m = step - VMZ + c and step - VMZ - c
        static_for<0, VMZ + 1>([&](auto Cz) __attribute__((always_inline)) {
          constexpr int c = (int)Cz;
          constexpr int sp = ((ph - VMZ + c) % NZR + NZR) % NZR;
#pragma unroll
          for (int k = 0; k < CY; ++k) {
            acc[sp][k][0] = acc[sp][k][0] + T[c][k][0];
            acc[sp][k][1] = acc[sp][k][1] + T[c][k][1];
          }
          if constexpr (c > 0) {
            constexpr int sm = ((ph - VMZ - c) % NZR + NZR) % NZR;
#pragma unroll
            for (int k = 0; k < CY; ++k) {
              acc[sm][k][0] = acc[sm][k][0] + T[c][k][0];
              acc[sm][k][1] = acc[sm][k][1] + T[c][k][1];
            }
          }
        });
      }
    });
  }
  // the last step's outputs: their rows were requested with no plane after
  wait_vm<0>();
  asm volatile("" ::: "memory");
  __builtin_amdgcn_s_barrier();
  asm volatile("" ::: "memory");
  emit(std::integral_constant<int, ((NSTEPS - 1) % NZR + 1) % NZR>{}, NSTEPS - 1);
  if constexpr ((FLAGS & FLAG_REDUCE) != 0) block_norms(v, p.partials + (size_t)lin * NUM_NORMS);
}

template <int LID, int SM, int TILE>
hipError_t launch_tile3(int flags, StencilParams p, hipStream_t s) {
  constexpr int CY = kStencilCY[TILE], BZ = kStencilBZ[TILE];
  constexpr int FORM = kStencilForm[TILE];
  if constexpr (FORM != STENCIL_BY_VELOCITY && !SepPlan3<LID>::t.closed) {
    return hipErrorInvalidValue;  // not a set of whole shells
  } else {
    constexpr StencilShape sh = stencil_tile_shape(3, TILE);
    p.gbx = (p.nx + sh.tx - 1) / sh.tx;
    p.gby = (p.ny + sh.ty - 1) / sh.ty;
    const unsigned gbz = (p.nz + sh.tz - 1) / sh.tz;
    const dim3 grid(p.gbx * p.gby * gbz);
    constexpr int NB = kStencilNB[TILE];
    if constexpr (FORM == STENCIL_PLANE_SUM && NB > 0) {
      // whole 16-byte units per row: nx a multiple of their element count
      constexpr unsigned E = 16 / sizeof(typename SModeTraits<SM>::TIN);
      if (p.nx % E != 0) return hipErrorInvalidValue;
      if (flags & FLAG_REDUCE)
        hipLaunchKernelGGL((k_stencil3pa<LID, SM, FLAG_REDUCE, CY, BZ, NB>), grid, dim3(256), 0, s, p);
      else
        hipLaunchKernelGGL((k_stencil3pa<LID, SM, 0, CY, BZ, NB>), grid, dim3(256), 0, s, p);
    } else if constexpr (FORM == STENCIL_PLANE_SUM) {
      if (flags & FLAG_REDUCE)
        hipLaunchKernelGGL((k_stencil3p<LID, SM, FLAG_REDUCE, CY, BZ>), grid, dim3(256), 0, s, p);
      else
        hipLaunchKernelGGL((k_stencil3p<LID, SM, 0, CY, BZ>), grid, dim3(256), 0, s, p);
    } else {
      constexpr bool SEP = FORM == STENCIL_SEPARABLE;
      if (flags & FLAG_REDUCE)
        hipLaunchKernelGGL((k_stencil3<LID, SM, FLAG_REDUCE, CY, BZ, SEP>), grid, dim3(256), 0, s, p);
      else
        hipLaunchKernelGGL((k_stencil3<LID, SM, 0, CY, BZ, SEP>), grid, dim3(256), 0, s, p);
    }
    return hipGetLastError();
  }
}

template <int LID, int SM>
hipError_t launch_smode(int flags, const StencilParams &p, hipStream_t s) {
  constexpr int DIM = Lattice<LID>::DIM;
  if constexpr (DIM == 3) {
    static_assert(kStencilTiles3 == 20, "one case per tile variant");
    switch (p.tile) {
      case 0: return launch_tile3<LID, SM, 0>(flags, p, s);
      case 1: return launch_tile3<LID, SM, 1>(flags, p, s);
      case 2: return launch_tile3<LID, SM, 2>(flags, p, s);
      case 3: return launch_tile3<LID, SM, 3>(flags, p, s);
      case 4: return launch_tile3<LID, SM, 4>(flags, p, s);
      case 5: return launch_tile3<LID, SM, 5>(flags, p, s);
      case 6: return launch_tile3<LID, SM, 6>(flags, p, s);
      case 7: return launch_tile3<LID, SM, 7>(flags, p, s);
      case 8: return launch_tile3<LID, SM, 8>(flags, p, s);
      case 9: return launch_tile3<LID, SM, 9>(flags, p, s);
      case 10: return launch_tile3<LID, SM, 10>(flags, p, s);
      case 11: return launch_tile3<LID, SM, 11>(flags, p, s);
      case 12: return launch_tile3<LID, SM, 12>(flags, p, s);
      case 13: return launch_tile3<LID, SM, 13>(flags, p, s);
      case 14: return launch_tile3<LID, SM, 14>(flags, p, s);
      case 15: return launch_tile3<LID, SM, 15>(flags, p, s);
      case 16: return launch_tile3<LID, SM, 16>(flags, p, s);
      case 17: return launch_tile3<LID, SM, 17>(flags, p, s);
      case 18: return launch_tile3<LID, SM, 18>(flags, p, s);
      case 19: return launch_tile3<LID, SM, 19>(flags, p, s);
    }
    return hipErrorInvalidValue;
  } else {
    using T = Tile<DIM>;
    constexpr StencilShape sh = stencil_tile_shape(DIM, 0);
    static_assert(T::TX == sh.tx && T::TY == sh.ty && T::TZ == sh.tz, "stencil tile");
    if (p.tile != 0) return hipErrorInvalidValue;
    dim3 grid((p.nx + sh.tx - 1) / sh.tx, (p.ny + sh.ty - 1) / sh.ty, (p.nz + sh.tz - 1) / sh.tz);
    if (flags & FLAG_REDUCE)
      hipLaunchKernelGGL((k_stencil<LID, SM, FLAG_REDUCE>), grid, dim3(256), 0, s, p);
    else
      hipLaunchKernelGGL((k_stencil<LID, SM, 0>), grid, dim3(256), 0, s, p);
    return hipGetLastError();
  }
}

}  // namespace stencil_detail

// One precision mode of the stencil form, compiled in a translation unit of
// its own.
template <int LID, int SM>
hipError_t launch_stencil_mode_tu(int flags, const StencilParams &p, hipStream_t s) {
  return stencil_detail::launch_smode<LID, SM>(flags, p, s);
}

template <int LID>
hipError_t launch_stencil_tu(int smode, int flags, const StencilParams &p, hipStream_t s) {
  switch (smode) {
    case SMODE_F64: return launch_stencil_mode_tu<LID, SMODE_F64>(flags, p, s);
    case SMODE_F32: return launch_stencil_mode_tu<LID, SMODE_F32>(flags, p, s);
    case SMODE_RESID: return launch_stencil_mode_tu<LID, SMODE_RESID>(flags, p, s);
  }
  return hipErrorInvalidValue;
}

}  // namespace lkp
