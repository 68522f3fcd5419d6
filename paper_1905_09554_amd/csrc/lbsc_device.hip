// Device code of the D3Q19 pseudo-potential lattice Boltzmann step for gfx950.
//
// Method (arXiv:1905.09554, Sec. 2): populations f_a stream and collide
// (Eq. LBE); moments by Eq. momentum; pseudo-potential psi = rho0 (1 -
// exp(-rho/rho0)); Shan-Chen force of Eq. SC_force; Guo-like forcing with the
// barycentric velocity of Eq. barycentric (plus the Guo source term), or the
// SRT velocity shift of Eq. vel_shift; SRT (BGK) or MRT collision; equation of
// state Eq. EOS_SC.
//
// Storage: node i = (z * ny + y) * nx + x; the nodes are cut into blocks of
// consecutive nodes whose 19 populations are stored one after the other
// (lat_index, lbsc_internal.h), so a work-group streams a few long runs of
// memory rather than 19 arrays.  A lattice holds post-collision values at
// their own node ("pull" layout): the post-streaming population of x is
// f_a(x) = lat[a][x - c_a], so the step reads with +-1 offsets and writes
// aligned.  In float32 storage the values are shifted, g_a = f_a - w_a rho_ref,
// and every formula below is written for g (rho_ref = 0 gives plain f).
//
// The hot kernel fuses streaming, moments, psi, the force gather, forcing
// and collision.  A work-group owns a tile of bx columns by by rows (whole
// rows where they fit) and marches a chunk of z planes.  For each plane it
// pulls the populations of its tile plus a one-node halo ring, reduces them
// to psi and keeps psi in a ring of four LDS planes; the interior
// populations stay in registers for the collision one plane later.  Each
// node therefore reads its 19 populations from HBM once and writes 19; the
// halo ring is re-read, mostly from L2 when the neighbouring tile (placed on
// the same XCD) has just loaded it.
#include "lbsc_internal.h"

#include <hip/hip_runtime.h>

#include <utility>

namespace lbsc {
namespace {

// Compile-time loop: calls f(std::integral_constant<int, I>) for I = 0..N-1,
// so every index below is a constant and per-node arrays live in registers.
template <class F, int... I>
__host__ __device__ inline void static_for_impl(F&& f, std::integer_sequence<int, I...>) {
  (f(std::integral_constant<int, I>{}), ...);
}
template <int N, class F>
__host__ __device__ inline void static_for(F&& f) {
  static_for_impl(f, std::make_integer_sequence<int, N>{});
}

// ------------------------------------------------------------------ lattice
// D3Q19: rest, six axis links, twelve face diagonals; opposite pairs adjacent.
constexpr int CX[Q] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
constexpr int CY[Q] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1};
constexpr int CZ[Q] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1};

template <class R>
__host__ __device__ constexpr R weight(int a) {
  return a == 0 ? R(1) / R(3) : (a < 7 ? R(1) / R(18) : R(1) / R(36));
}

// d'Humieres et al. (2002) D3Q19 moment basis, row i evaluated at velocity a.
// Rows: rho, e, eps, jx, qx, jy, qy, jz, qz, 3pxx, 3pixx, pww, piww, pxy,
// pyz, pxz, mx, my, mz.
__host__ __device__ constexpr int mrt_entry(int i, int a) {
  const int x = CX[a], y = CY[a], z = CZ[a];
  const int c2 = x * x + y * y + z * z;
  switch (i) {
    case 0: return 1;
    case 1: return 19 * c2 - 30;
    case 2: return (21 * c2 * c2 - 53 * c2 + 24) / 2;
    case 3: return x;
    case 4: return (5 * c2 - 9) * x;
    case 5: return y;
    case 6: return (5 * c2 - 9) * y;
    case 7: return z;
    case 8: return (5 * c2 - 9) * z;
    case 9: return 3 * x * x - c2;
    case 10: return (3 * c2 - 5) * (3 * x * x - c2);
    case 11: return y * y - z * z;
    case 12: return (3 * c2 - 5) * (y * y - z * z);
    case 13: return x * y;
    case 14: return y * z;
    case 15: return x * z;
    case 16: return (y * y - z * z) * x;
    case 17: return (z * z - x * x) * y;
    default: return (x * x - y * y) * z;
  }
}

// Squared row norms sum_a M_ia^2 (rows are orthogonal, so M^-1 = M^T D^-1).
__host__ __device__ constexpr int mrt_norm(int i) {
  int s = 0;
  for (int a = 0; a < Q; ++a) s += mrt_entry(i, a) * mrt_entry(i, a);
  return s;
}

// Rate class of a row: 0 conserved, 1 bulk, 2 shear, 3 ghost.
__host__ __device__ constexpr int mrt_class(int i) {
  return (i == 0 || i == 3 || i == 5 || i == 7) ? 0
         : (i == 1) ? 1
         : (i == 9 || i == 11 || i == 13 || i == 14 || i == 15) ? 2
                                                                  : 3;
}

template <class R>
struct Phys {
  R G, psi_rho0, inv_psi_rho0, tau, omega, s_bulk, s_ghost, rho_ref;
};

template <class R>
__host__ __device__ inline Phys<R> make_phys(const StepArgs& a) {
  Phys<R> p;
  p.G = R(a.G);
  p.psi_rho0 = R(a.psi_rho0);
  p.inv_psi_rho0 = R(1.0 / a.psi_rho0);
  p.tau = R(a.tau);
  p.omega = R(a.omega);
  p.s_bulk = R(a.s_bulk);
  p.s_ghost = R(a.s_ghost);
  p.rho_ref = R(a.rho_ref);
  return p;
}

__device__ inline double psi_of(double rho, double rho0, double inv_rho0) {
  return -rho0 * expm1(-rho * inv_rho0);
}
__device__ inline float psi_of(float rho, float rho0, float inv_rho0) {
  return -rho0 * expm1f(-rho * inv_rho0);
}

// ---------------------------------------------------------------- collision
// Error-free sum of two floats (Knuth's TwoSum): a + b = s + e exactly.
__device__ inline void two_sum(float a, float b, float& s, float& e) {
  s = a + b;
  const float bp = s - a;
  e = (a - (s - bp)) + (b - bp);
}

// In-place collision of one node.  f holds the post-streaming populations
// (shifted by w rho_ref), F the Shan-Chen force at the node.
//
// Float32 storage gets three numerical safeguards that are exact identities
// in real arithmetic (so the method is unchanged):
//  * the shifted density sum is compensated (TwoSum), and rho - rho_ref is
//    taken from that sum, never from rho - rho_ref;
//  * momenta are summed over differences of opposite populations, which are
//    nearly equal and subtract with little or no rounding;
//  * the collision is applied as an increment D (f* = f + D) whose mass sum
//    is forced to 0 and momentum sum to F through the rest and axis
//    populations.  Without this, the rounding of the equilibrium repeats
//    with the same sign at slowly moving interface nodes and feeds the
//    Plateau-Rayleigh mode as a systematic mass and momentum source.
template <class R, int COLL, int FORC>
__device__ inline void collide(R (&f)[Q], R Fx, R Fy, R Fz, const Phys<R>& k) {
  constexpr bool kF32 = sizeof(R) == 4;
  R s;
  if constexpr (kF32) {
    float acc = f[0], comp = 0.f;
    static_for<Q - 1>([&](auto ac) {
      constexpr int a = decltype(ac)::value + 1;
      float t, e;
      two_sum(acc, f[a], t, e);
      acc = t;
      comp += e;
    });
    s = acc + comp;
  } else {
    s = R(0);
    static_for<Q>([&](auto ac) { s += f[decltype(ac)::value]; });
  }
  // Opposite pairs are (1,2), (3,4), ..., (17,18).
  R jx = R(0), jy = R(0), jz = R(0);
  static_for<(Q - 1) / 2>([&](auto pc) {
    constexpr int a = 2 * decltype(pc)::value + 1;
    const R d = f[a] - f[a + 1];
    if constexpr (CX[a] != 0) jx += R(CX[a]) * d;
    if constexpr (CY[a] != 0) jy += R(CY[a]) * d;
    if constexpr (CZ[a] != 0) jz += R(CZ[a]) * d;
  });
  const R drho = s;
  const R rho = k.rho_ref + s;
  const R inv_rho = R(1) / rho;
  // Equilibrium velocity: barycentric (Guo) or shifted by tau F / rho (SRT).
  const R fs = (FORC == kGuo) ? R(0.5) : k.tau;
  const R ux = (jx + fs * Fx) * inv_rho;
  const R uy = (jy + fs * Fy) * inv_rho;
  const R uz = (jz + fs * Fz) * inv_rho;
  const R uu15 = R(1.5) * (ux * ux + uy * uy + uz * uz);
  const R uF = ux * Fx + uy * Fy + uz * Fz;

  R D[Q];
  if constexpr (COLL == kBGK) {
    const R om = k.omega;
    const R src_fac = R(1) - R(0.5) * om;
    static_for<Q>([&](auto ac) {
      constexpr int a = decltype(ac)::value;
      const R w = weight<R>(a);
      R cu = R(0), cF = R(0);
      if constexpr (CX[a] != 0) { cu += R(CX[a]) * ux; cF += R(CX[a]) * Fx; }
      if constexpr (CY[a] != 0) { cu += R(CY[a]) * uy; cF += R(CY[a]) * Fy; }
      if constexpr (CZ[a] != 0) { cu += R(CZ[a]) * uz; cF += R(CZ[a]) * Fz; }
      const R geq = w * drho + w * rho * (R(3) * cu + R(4.5) * cu * cu - uu15);
      R d = om * (geq - f[a]);
      if constexpr (FORC == kGuo) d += src_fac * (w * (R(3) * (cF - uF) + R(9) * cu * cF));
      D[a] = d;
    });
  } else {
    // MRT: f* = f - M^T D^-1 [Lambda (M f - m_eq) - (I - Lambda/2) M S],
    // using M^-1 = M^T D^-1 (orthogonal rows, D their squared norms).  The
    // equilibrium moments m_eq = M f^eq(rho, u^b) and the source moments M S
    // of the quadratic D3Q19 equilibrium and the Guo term have closed forms,
    // so only M f is transformed numerically.  With shifted storage
    // (g = f - w rho_ref) the rows e and eps see M (w rho_ref) = (-11, 3)
    // rho_ref, which is folded into their equilibria through drho.
    const R ux2 = ux * ux, uy2 = uy * uy, uz2 = uz * uz;
    const R usq = ux2 + uy2 + uz2;
    const R pxx = R(2) * ux2 - uy2 - uz2;       // 3 p_xx / rho
    const R pww = uy2 - uz2;                     // p_ww / rho
    const R sxx = R(2) * ux * Fx - uy * Fy - uz * Fz;
    const R sww = uy * Fy - uz * Fz;
    R meq[Q], msrc[Q];
    static_for<Q>([&](auto ic) { meq[decltype(ic)::value] = R(0); msrc[decltype(ic)::value] = R(0); });
    meq[1] = R(-11) * drho + R(19) * rho * usq;  msrc[1] = R(38) * uF;
    meq[2] = R(3) * drho - R(5.5) * rho * usq;   msrc[2] = R(-11) * uF;
    meq[4] = R(-2.0 / 3.0) * rho * ux;           msrc[4] = R(-2.0 / 3.0) * Fx;
    meq[6] = R(-2.0 / 3.0) * rho * uy;           msrc[6] = R(-2.0 / 3.0) * Fy;
    meq[8] = R(-2.0 / 3.0) * rho * uz;           msrc[8] = R(-2.0 / 3.0) * Fz;
    meq[9] = rho * pxx;                          msrc[9] = R(2) * sxx;
    meq[10] = R(-0.5) * rho * pxx;               msrc[10] = -sxx;
    meq[11] = rho * pww;                         msrc[11] = R(2) * sww;
    meq[12] = R(-0.5) * rho * pww;               msrc[12] = -sww;
    meq[13] = rho * ux * uy;                     msrc[13] = ux * Fy + uy * Fx;
    meq[14] = rho * uy * uz;                     msrc[14] = uy * Fz + uz * Fy;
    meq[15] = rho * ux * uz;                     msrc[15] = ux * Fz + uz * Fx;
    R kk[Q];
    static_for<Q>([&](auto ic) {
      constexpr int i = decltype(ic)::value;
      kk[i] = R(0);
      if constexpr (mrt_class(i) != 0) {
        R m = R(0);
        static_for<Q>([&](auto ac) {
          constexpr int a = decltype(ac)::value;
          if constexpr (mrt_entry(i, a) != 0) m += R(mrt_entry(i, a)) * f[a];
        });
        const R lam = mrt_class(i) == 1 ? k.s_bulk : (mrt_class(i) == 2 ? k.omega : k.s_ghost);
        kk[i] = (lam * (m - meq[i]) - (R(1) - R(0.5) * lam) * msrc[i]) *
                (R(1) / R(mrt_norm(i)));
      }
    });
    // Conserved rows: the density row carries nothing; the momentum rows
    // contribute exactly M^-1 (0, F) whatever their rate (their
    // non-equilibrium moment is -F/2 and their source moment F).
    static_for<Q>([&](auto ac) {
      constexpr int a = decltype(ac)::value;
      R acc = R(0);
      static_for<Q>([&](auto ic) {
        constexpr int i = decltype(ic)::value;
        if constexpr (mrt_class(i) != 0 && mrt_entry(i, a) != 0) acc += R(mrt_entry(i, a)) * kk[i];
      });
      R fc = R(0);
      if constexpr (CX[a] != 0) fc += R(CX[a]) * Fx;
      if constexpr (CY[a] != 0) fc += R(CY[a]) * Fy;
      if constexpr (CZ[a] != 0) fc += R(CZ[a]) * Fz;
      D[a] = R(0.1) * fc - acc;
    });
  }
  if constexpr (kF32) {
    // Mass change 0 and momentum change F, enforced on the rounded increment.
    R d0 = R(0), dx = -Fx, dy = -Fy, dz = -Fz;
    static_for<Q>([&](auto ac) {
      constexpr int a = decltype(ac)::value;
      d0 += D[a];
      if constexpr (CX[a] != 0) dx += R(CX[a]) * D[a];
      if constexpr (CY[a] != 0) dy += R(CY[a]) * D[a];
      if constexpr (CZ[a] != 0) dz += R(CZ[a]) * D[a];
    });
    D[0] -= d0;
    D[1] -= R(0.5) * dx;
    D[2] += R(0.5) * dx;
    D[3] -= R(0.5) * dy;
    D[4] += R(0.5) * dy;
    D[5] -= R(0.5) * dz;
    D[6] += R(0.5) * dz;
  }
  static_for<Q>([&](auto ac) {
    constexpr int a = decltype(ac)::value;
    f[a] += D[a];
  });
}

// --------------------------------------------------------------- addressing
struct Nbr {
  unsigned xo[3];  // x - 1, x, x + 1 (periodic)
  unsigned yo[3];  // row offsets of y - 1, y, y + 1
  unsigned zo[3];  // plane offsets of z - 1, z, z + 1
};

__device__ inline Nbr neighbours(int x, int y, int z, int nx, int ny, int nz, int plane) {
  Nbr b;
  b.xo[0] = x == 0 ? nx - 1 : x - 1;
  b.xo[1] = x;
  b.xo[2] = x == nx - 1 ? 0 : x + 1;
  b.yo[0] = (y == 0 ? ny - 1 : y - 1) * nx;
  b.yo[1] = y * nx;
  b.yo[2] = (y == ny - 1 ? 0 : y + 1) * nx;
  b.zo[0] = (unsigned)(z == 0 ? nz - 1 : z - 1) * (unsigned)plane;
  b.zo[1] = (unsigned)z * (unsigned)plane;
  b.zo[2] = (unsigned)(z == nz - 1 ? 0 : z + 1) * (unsigned)plane;
  return b;
}

// Post-streaming populations of a node: f_a(x) = lat[a][x - c_a].
template <class T, class R>
__device__ inline void pull(const T* __restrict__ lat, long long ps, const Nbr& b, R (&f)[Q]) {
#pragma unroll
  for (int a = 0; a < Q; ++a) {
    const unsigned idx = b.zo[1 - CZ[a]] + b.yo[1 - CY[a]] + b.xo[1 - CX[a]];
    f[a] = R(lat[lat_index<T>(a, idx, ps)]);
  }
}

template <class T, class R>
__device__ inline R pull_sum(const T* __restrict__ lat, long long ps, const Nbr& b) {
  R s = R(0);
#pragma unroll
  for (int a = 0; a < Q; ++a) {
    const unsigned idx = b.zo[1 - CZ[a]] + b.yo[1 - CY[a]] + b.xo[1 - CX[a]];
    s += R(lat[lat_index<T>(a, idx, ps)]);
  }
  return s;
}

__device__ inline int remap_xcd(int b, int nb) {
  // Work-groups are dispatched round-robin over the 8 XCDs: group b runs on
  // XCD k = b mod 8 as that XCD's j = b div 8-th group.  Give each XCD a
  // contiguous range of logical tiles, so that tiles sharing halo rows share
  // an L2.  With nb = 8 q + r, XCD k holds q + [k < r] groups and its range
  // starts at k q + min(k, r); the ranges tile [0, nb) exactly.
  const int k = b & 7, j = b >> 3, q = nb >> 3, r = nb & 7;
  return k * q + min(k, r) + j;
}

// psi at a node and its 18 neighbours: c; the axis neighbours x+ x- y+ y-
// z+ z-; the diagonal pairs (+,+) (-,-) (+,-) (-,+) in the xy, xz and yz
// planes.
template <class R>
struct Psi19 {
  R c, xp, xm, yp, ym, zp, zm;
  R xy_pp, xy_mm, xy_pm, xy_mp, xz_pp, xz_mm, xz_pm, xz_mp, yz_pp, yz_mm, yz_pm, yz_mp;
};

// Shan-Chen force F = -G psi(x) sum_a w_a psi(x + c_a) c_a (Eq. SC_force),
// axis links weight 1/18, diagonals 1/36, summed as differences of opposite
// neighbours.  Both step forms call this, so they agree bitwise.
template <class R>
__device__ inline void sc_force(const Psi19<R>& q, R G, R& Fx, R& Fy, R& Fz) {
  const R ax = q.xp - q.xm;
  const R ay = q.yp - q.ym;
  const R az = q.zp - q.zm;
  const R dxy = q.xy_pp - q.xy_mm;
  const R dxmy = q.xy_pm - q.xy_mp;
  const R dxz = q.xz_pp - q.xz_mm;
  const R dxmz = q.xz_pm - q.xz_mp;
  const R dyz = q.yz_pp - q.yz_mm;
  const R dymz = q.yz_pm - q.yz_mp;
  const R sx = ax * R(1.0 / 18.0) + (dxy + dxmy + dxz + dxmz) * R(1.0 / 36.0);
  const R sy = ay * R(1.0 / 18.0) + (dxy - dxmy + dyz + dymz) * R(1.0 / 36.0);
  const R sz = az * R(1.0 / 18.0) + (dxz - dxmz + dyz - dymz) * R(1.0 / 36.0);
  const R gpsi = -G * q.c;
  Fx = gpsi * sx;
  Fy = gpsi * sy;
  Fz = gpsi * sz;
}

// ---------------------------------------------------------------- the step
// One work-group of NT threads owns the tile of columns [x0, x0 + bx) and
// rows [y0, y0 + by) (bx * by <= K NT) over planes [z0, z1); each thread
// carries K interior nodes (tile indices tid + k NT).  Iteration of plane z:
// pull plane z+1 (tile plus its one-node ring of halo nodes), publish
// psi(z+1) to LDS slot (k+2)%4, barrier, then force and collision of plane z
// from the populations kept in registers since the previous iteration.  Four
// psi slots make one barrier per iteration enough: the slot written at
// iteration k+1 was last read at iteration k-1.  An LDS psi plane is
// (by + 2) rows of (bx + 2) values; the halo ring is recomputed from its own
// 19 pulled loads (mostly cache hits: they are the neighbouring tiles'
// interior).
template <class T, int COLL, int FORC, int NT, int K>
__device__ inline void step_tile(const T* __restrict__ src, T* __restrict__ dst,
                                 const StepArgs& a, int txy, int zc, T* lds) {
  using R = T;
  const Phys<R> ph = make_phys<R>(a);
  const int nx = a.nx, ny = a.ny, nz = a.nz, plane = a.plane;
  const long long ps = a.ps;
  const int lw = a.bx + 2;
  const int lplane = (a.by + 2) * lw;
  const int tx = txy % a.ntiles_x, ty = txy / a.ntiles_x;
  const int x0 = tx * a.bx, y0 = ty * a.by;
  const int bxe = min(a.bx, nx - x0);
  const int bye = min(a.by, ny - y0);
  const int z0 = zc * a.zchunk;
  const int z1 = min(nz, z0 + a.zchunk);

  const int tid = threadIdx.x;
  int lx[K], ly[K], cx[K], cy[K];
  bool interior[K];
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const int i = tid + k * NT;
    lx[k] = i % a.bx;
    ly[k] = i / a.bx;
    interior[k] = ly[k] < bye && lx[k] < bxe;
    cx[k] = min(lx[k], bxe - 1);  // the node a thread past the edge stands in for
    cy[k] = min(ly[k], bye - 1);
  }
  // Halo ring: rows -1 and bye over columns -1..bxe, then columns -1 and bxe
  // over rows 0..bye-1.  A tile of whole rows has no halo columns of its own:
  // columns -1 and bxe are the row's last and first node, which the owners of
  // those nodes store a second time.
  const bool whole_rows = bxe == nx;
  const int hrow = whole_rows ? bxe : bxe + 2;
  const int nhalo = whole_rows ? 2 * bxe : 2 * hrow + 2 * bye;

  R cur[K][Q], nxt[K][Q];

  // psi of halo node h of plane z into its LDS row.
  auto halo_node = [&](int h, int z, R* lp) {
    int hl, hc;
    if (whole_rows) {
      hl = h < bxe ? -1 : bye;
      hc = h < bxe ? h : h - bxe;
    } else if (h < 2 * hrow) {
      hl = h < hrow ? -1 : bye;
      hc = (h < hrow ? h : h - hrow) - 1;
    } else {
      const int g = h - 2 * hrow;
      hc = g < bye ? -1 : bxe;
      hl = g < bye ? g : g - bye;
    }
    int hy = y0 + hl, hx = x0 + hc;
    hy = hy < 0 ? hy + ny : (hy >= ny ? hy - ny : hy);
    hx = hx < 0 ? hx + nx : (hx >= nx ? hx - nx : hx);
    const Nbr nb = neighbours(hx, hy, z, nx, ny, nz, plane);
    // All 19 loads are issued before the first add: left to itself, the
    // scheduler pairs each load with its add to save registers, which puts
    // 19 memory latencies in a row.
    R f[Q];
    pull<T, R>(src, ps, nb, f);
    __builtin_amdgcn_sched_barrier(0);
    R s = R(0);
#pragma unroll
    for (int q = 0; q < Q; ++q) s += f[q];
    const R v = psi_of(ph.rho_ref + s, ph.psi_rho0, ph.inv_psi_rho0);
    R* row = lp + (hl + 1) * lw;
    row[hc + 1] = v;
    if (whole_rows && hc == 0) row[bxe + 1] = v;
    if (whole_rows && hc == bxe - 1) row[0] = v;
  };

  // Pulls plane z: psi of the tile plus its halo ring into LDS slot `slot`;
  // interior populations into `keep`.  Threads past the tile's ragged edge
  // pull the clamped in-tile node (cx, cy) and store its psi a second time,
  // the same value to the same LDS word as its owner.  Loads and their uses
  // under a branch would leave the compiler unsure whether they have landed
  // at the end of the plane loop, and it would wait there for every
  // outstanding store before the next plane's loads.  The first round of the
  // halo ring is issued before the interior sums wait, so that both sets of
  // loads are in flight together.
  auto load_plane = [&](int z, int slot, R(&keep)[K][Q]) {
    R* lp = lds + slot * lplane;
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const Nbr nb = neighbours(x0 + cx[k], y0 + cy[k], z, nx, ny, nz, plane);
      pull<T, R>(src, ps, nb, keep[k]);
    }
    // float64: the halo loads wait for the interior sums (fewer registers
    // live at once; measured faster for the register-bound float64 kernel).
    constexpr bool halo_first = sizeof(T) < 8;
    if (halo_first && tid < nhalo) halo_node(tid, z, lp);
#pragma unroll
    for (int k = 0; k < K; ++k) {
      R s = R(0);
#pragma unroll
      for (int q = 0; q < Q; ++q) s += keep[k][q];
      const R v = psi_of(ph.rho_ref + s, ph.psi_rho0, ph.inv_psi_rho0);
      R* row = lp + (cy[k] + 1) * lw;
      row[cx[k] + 1] = v;
      if (whole_rows && cx[k] == 0) row[bxe + 1] = v;
      if (whole_rows && cx[k] == bxe - 1) row[0] = v;
    }
    if (!halo_first && tid < nhalo) halo_node(tid, z, lp);
    for (int h = tid + NT; h < nhalo; h += NT) halo_node(h, z, lp);
  };

  const int zprev = z0 == 0 ? nz - 1 : z0 - 1;
  load_plane(zprev, 0, nxt);
  load_plane(z0, 1, cur);

  for (int z = z0, it = 0; z < z1; ++z, ++it) {
    const int znext = z == nz - 1 ? 0 : z + 1;
    // The next plane's loads go out at raised wave priority, so that a
    // work-group issuing them is not held back by another's collision.
    __builtin_amdgcn_s_setprio(2);
    load_plane(znext, (it + 2) & 3, nxt);
    __builtin_amdgcn_s_setprio(0);
    __syncthreads();
    const R* pm = lds + (it & 3) * lplane;
    const R* pc = lds + ((it + 1) & 3) * lplane;
    const R* pp = lds + ((it + 2) & 3) * lplane;
#pragma unroll
    for (int k = 0; k < K; ++k) {
      if (!interior[k]) continue;
      const int x = lx[k] + 1;  // LDS column; x - 1 and x + 1 are in the ring
      const int xm = x - 1, xp = x + 1;
      const int rm = ly[k] * lw, rc = (ly[k] + 1) * lw, rp = (ly[k] + 2) * lw;
      Psi19<R> q;
      q.c = pc[rc + x];
      q.xp = pc[rc + xp];
      q.xm = pc[rc + xm];
      q.yp = pc[rp + x];
      q.ym = pc[rm + x];
      q.zp = pp[rc + x];
      q.zm = pm[rc + x];
      q.xy_pp = pc[rp + xp];
      q.xy_mm = pc[rm + xm];
      q.xy_pm = pc[rm + xp];
      q.xy_mp = pc[rp + xm];
      q.xz_pp = pp[rc + xp];
      q.xz_mm = pm[rc + xm];
      q.xz_pm = pm[rc + xp];
      q.xz_mp = pp[rc + xm];
      q.yz_pp = pp[rp + x];
      q.yz_mm = pm[rm + x];
      q.yz_pm = pm[rp + x];
      q.yz_mp = pp[rm + x];
      R Fx, Fy, Fz;
      sc_force<R>(q, ph.G, Fx, Fy, Fz);
      const unsigned idx =
          (unsigned)z * (unsigned)plane + (unsigned)((y0 + ly[k]) * nx + x0 + lx[k]);
      // The adjoint's recomputation keeps psi as the forces used it.
      if (a.psi_out) static_cast<T*>(a.psi_out)[idx] = q.c;
      collide<R, COLL, FORC>(cur[k], Fx, Fy, Fz, ph);
      // Written once and read only in the next step: non-temporal stores keep
      // them from evicting the rows the neighbouring tiles still re-read.
#pragma unroll
      for (int q = 0; q < Q; ++q)
        __builtin_nontemporal_store(T(cur[k][q]), &dst[lat_index<T>(q, idx, ps)]);
    }
#pragma unroll
    for (int k = 0; k < K; ++k)
#pragma unroll
      for (int q = 0; q < Q; ++q) cur[k][q] = nxt[k][q];
  }
}

// Single box: work-group b owns xy tile b mod (ntiles_x ntiles_y) of z chunk
// b div (ntiles_x ntiles_y).
template <class T, int COLL, int FORC, int NT, int K>
__global__ void __launch_bounds__(NT)
k_step(const T* __restrict__ src, T* __restrict__ dst, StepArgs a) {
  extern __shared__ __attribute__((aligned(16))) unsigned char smem_raw[];
  int b = blockIdx.x;
  if (a.xcd_remap) b = remap_xcd(b, gridDim.x);
  const int ntxy = a.ntiles_x * a.ntiles_y;
  step_tile<T, COLL, FORC, NT, K>(src, dst, a, b % ntxy, b / ntxy,
                                  reinterpret_cast<T*>(smem_raw));
}

// Two-kernel form of the step, the baseline the fused kernel is measured
// against: K1 pulls the populations of every node and writes psi to global
// memory; K2 pulls them again, reads the psi stencil from global memory and
// collides.  That moves 19 + 1 + 19 + 1 + 19 = 59 values per node (with
// perfect reuse of the psi stencil) instead of 38.  Same arithmetic as the
// fused kernel, so the results agree bitwise.
template <class T>
__global__ void __launch_bounds__(256)
k_density_psi(const T* __restrict__ src, T* __restrict__ psi, StepArgs a) {
  using R = T;
  const Phys<R> ph = make_phys<R>(a);
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < a.n;
       i += (long long)gridDim.x * blockDim.x) {
    const int x = (int)(i % a.nx), y = (int)((i / a.nx) % a.ny), z = (int)(i / a.plane);
    const Nbr nb = neighbours(x, y, z, a.nx, a.ny, a.nz, a.plane);
    R f[Q];
    pull<T, R>(src, a.ps, nb, f);
    R s = R(0);
#pragma unroll
    for (int q = 0; q < Q; ++q) s += f[q];
    psi[i] = T(psi_of(ph.rho_ref + s, ph.psi_rho0, ph.inv_psi_rho0));
  }
}

template <class T, int COLL, int FORC>
__global__ void __launch_bounds__(256)
k_step_psi(const T* __restrict__ src, const T* __restrict__ psi, T* __restrict__ dst,
           StepArgs a) {
  using R = T;
  const Phys<R> ph = make_phys<R>(a);
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < a.n;
       i += (long long)gridDim.x * blockDim.x) {
    const int x = (int)(i % a.nx), y = (int)((i / a.nx) % a.ny), z = (int)(i / a.plane);
    const Nbr b = neighbours(x, y, z, a.nx, a.ny, a.nz, a.plane);
    R f[Q];
    pull<T, R>(src, a.ps, b, f);
    Psi19<R> q;
    q.c = R(psi[b.zo[1] + b.yo[1] + b.xo[1]]);
    q.xp = R(psi[b.zo[1] + b.yo[1] + b.xo[2]]);
    q.xm = R(psi[b.zo[1] + b.yo[1] + b.xo[0]]);
    q.yp = R(psi[b.zo[1] + b.yo[2] + b.xo[1]]);
    q.ym = R(psi[b.zo[1] + b.yo[0] + b.xo[1]]);
    q.zp = R(psi[b.zo[2] + b.yo[1] + b.xo[1]]);
    q.zm = R(psi[b.zo[0] + b.yo[1] + b.xo[1]]);
    q.xy_pp = R(psi[b.zo[1] + b.yo[2] + b.xo[2]]);
    q.xy_mm = R(psi[b.zo[1] + b.yo[0] + b.xo[0]]);
    q.xy_pm = R(psi[b.zo[1] + b.yo[0] + b.xo[2]]);
    q.xy_mp = R(psi[b.zo[1] + b.yo[2] + b.xo[0]]);
    q.xz_pp = R(psi[b.zo[2] + b.yo[1] + b.xo[2]]);
    q.xz_mm = R(psi[b.zo[0] + b.yo[1] + b.xo[0]]);
    q.xz_pm = R(psi[b.zo[0] + b.yo[1] + b.xo[2]]);
    q.xz_mp = R(psi[b.zo[2] + b.yo[1] + b.xo[0]]);
    q.yz_pp = R(psi[b.zo[2] + b.yo[2] + b.xo[1]]);
    q.yz_mm = R(psi[b.zo[0] + b.yo[0] + b.xo[1]]);
    q.yz_pm = R(psi[b.zo[0] + b.yo[2] + b.xo[1]]);
    q.yz_mp = R(psi[b.zo[2] + b.yo[0] + b.xo[1]]);
    R Fx, Fy, Fz;
    sc_force<R>(q, ph.G, Fx, Fy, Fz);
    collide<R, COLL, FORC>(f, Fx, Fy, Fz, ph);
#pragma unroll
    for (int qq = 0; qq < Q; ++qq)
      __builtin_nontemporal_store(T(f[qq]), &dst[lat_index<T>(qq, (unsigned)i, a.ps)]);
  }
}

// Batch of boxes (uneven sizes and parameters), one step: the tile table
// lists (member, xy tile, z chunk) for every member; work-group b runs one
// entry.  Lattice `parity` of each member is the source.
template <class T, int COLL, int FORC, int NT, int K>
__global__ void __launch_bounds__(NT)
k_step_batch(const BatchMember* __restrict__ mem, const int4* __restrict__ tiles, int parity,
             int remap) {
  extern __shared__ __attribute__((aligned(16))) unsigned char smem_raw[];
  int b = blockIdx.x;
  if (remap) b = remap_xcd(b, gridDim.x);
  const int4 t = tiles[b];
  const StepArgs a = mem[t.x].a;
  step_tile<T, COLL, FORC, NT, K>((const T*)mem[t.x].lat[parity], (T*)mem[t.x].lat[parity ^ 1], a,
                                  t.y, t.z, reinterpret_cast<T*>(smem_raw));
}

// Grid-wide barrier for a cooperative launch (every work-group resident).
// Thread 0 arrives with an agent-scope release (its group's stores become
// visible to other XCDs) and waits with an agent-scope acquire.  The wait is
// bounded: after spin_limit polls, or as soon as another group has recorded
// a timeout, it records one in *err and the barrier returns false; callers
// then leave the kernel, so every work-group reaches its end.  The last group
// to arrive also clears *reset (the tile counter of the step just finished).
__device__ inline bool grid_barrier(unsigned* count, unsigned* gen, unsigned nblocks,
                                    unsigned* err, unsigned spin_limit, unsigned* reset) {
  __shared__ int ok;
  __syncthreads();
  if (threadIdx.x == 0) {
    ok = 1;
    const unsigned g = __hip_atomic_load(gen, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
    const unsigned arrived =
        __hip_atomic_fetch_add(count, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT) + 1u;
    if (arrived == nblocks) {
      __hip_atomic_store(count, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      if (reset) __hip_atomic_store(reset, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_fetch_add(gen, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    } else {
      unsigned spins = 0;
      while (__hip_atomic_load(gen, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) == g) {
        if (++spins > spin_limit ||
            __hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u) {
          __hip_atomic_fetch_or(err, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          ok = 0;
          break;
        }
        __builtin_amdgcn_s_sleep(8);
      }
    }
  }
  __syncthreads();
  return ok != 0;
}

// Batch, all steps in one cooperative launch.  Within a step, work-groups
// take tiles from a shared counter (tiles differ in size across members, so
// a dynamic queue balances them), then all groups meet at a grid barrier
// before the next step reads what this one wrote.  Two counters alternate
// between steps; the barrier clears the one just used.
// sync: [0] arrivals, [1] generation, [2] timeout flag, [3..4] tile counters.
template <class T, int COLL, int FORC, int NT, int K>
__global__ void __launch_bounds__(NT)
k_step_persistent(const BatchMember* __restrict__ mem, const int4* __restrict__ tiles,
                  int ntiles, int parity0, int nsteps, unsigned* sync, unsigned spin_limit) {
  extern __shared__ __attribute__((aligned(16))) unsigned char smem_raw[];
  __shared__ int next;
  for (int s = 0; s < nsteps; ++s) {
    const int parity = parity0 ^ (s & 1);
    unsigned* counter = sync + 3 + (s & 1);
    for (;;) {
      if (threadIdx.x == 0)
        next = (int)__hip_atomic_fetch_add(counter, 1u, __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_AGENT);
      __syncthreads();
      const int b = next;
      if (b >= ntiles) break;
      const int4 t = tiles[b];
      const StepArgs a = mem[t.x].a;
      step_tile<T, COLL, FORC, NT, K>((const T*)mem[t.x].lat[parity],
                                      (T*)mem[t.x].lat[parity ^ 1], a, t.y, t.z,
                                      reinterpret_cast<T*>(smem_raw));
      __syncthreads();  // the next tile reuses the LDS ring and `next`
    }
    if (!grid_barrier(sync, sync + 1, gridDim.x, sync + 2, spin_limit, counter)) return;
  }
}

// ------------------------------------------------------------ initial state
// Post-collision layout of the state f_a(x) = w_a rho0(x): lat[a][y] holds
// f_a(y + c_a) = w_a rho0(y + c_a), shifted by w_a rho_ref in float32.
template <class T>
__global__ void __launch_bounds__(256)
k_init(T* __restrict__ lat, const double* __restrict__ rho0, StepArgs a) {
  const long long n = a.n;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x) {
    const int x = (int)(i % a.nx);
    const int y = (int)((i / a.nx) % a.ny);
    const int z = (int)(i / a.plane);
    const Nbr nb = neighbours(x, y, z, a.nx, a.ny, a.nz, a.plane);
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      const unsigned src = nb.zo[1 + CZ[q]] + nb.yo[1 + CY[q]] + nb.xo[1 + CX[q]];
      lat[lat_index<T>(q, (unsigned)i, a.ps)] = T(weight<double>(q) * (rho0[src] - a.rho_ref));
    }
  }
}

// Post-streaming populations of every node into the plain arrays
// out[a * ps_out + x] (state export); ps_in is the lattice's own size.
template <class T>
__global__ void __launch_bounds__(256)
k_gather(const T* __restrict__ lat, long long ps_in, T* __restrict__ out, long long ps_out,
         StepArgs a) {
  const long long n = a.n;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x) {
    const int x = (int)(i % a.nx);
    const int y = (int)((i / a.nx) % a.ny);
    const int z = (int)(i / a.plane);
    const Nbr nb = neighbours(x, y, z, a.nx, a.ny, a.nz, a.plane);
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      const unsigned src = nb.zo[1 - CZ[q]] + nb.yo[1 - CY[q]] + nb.xo[1 - CX[q]];
      out[(long long)q * ps_out + i] = lat[lat_index<T>(q, src, ps_in)];
    }
  }
}

// Inverse of k_gather (state import) from plain arrays in[a * ps_in + x]:
// lat[a][y] = in[a][y + c_a]; ps_out is the lattice's own size.
template <class T>
__global__ void __launch_bounds__(256)
k_scatter(const T* __restrict__ in, long long ps_in, T* __restrict__ lat, long long ps_out,
          StepArgs a) {
  const long long n = a.n;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x) {
    const int x = (int)(i % a.nx);
    const int y = (int)((i / a.nx) % a.ny);
    const int z = (int)(i / a.plane);
    const Nbr nb = neighbours(x, y, z, a.nx, a.ny, a.nz, a.plane);
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      const unsigned src = nb.zo[1 + CZ[q]] + nb.yo[1 + CY[q]] + nb.xo[1 + CX[q]];
      lat[lat_index<T>(q, (unsigned)i, ps_out)] = in[(long long)q * ps_in + src];
    }
  }
}

// ------------------------------------------------------------------ moments
// Pass 1: rho and j of every node (float64).  j goes to u (later turned into
// u^b by pass 2) when u is given.
template <class T>
__global__ void __launch_bounds__(256)
k_moments1(const T* __restrict__ lat, double* __restrict__ rho, double* __restrict__ u,
           double* __restrict__ psi, StepArgs a) {
  const long long n = a.n;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x) {
    const int x = (int)(i % a.nx);
    const int y = (int)((i / a.nx) % a.ny);
    const int z = (int)(i / a.plane);
    const Nbr nb = neighbours(x, y, z, a.nx, a.ny, a.nz, a.plane);
    double f[Q];
    pull<T, double>(lat, a.ps, nb, f);
    double s = 0, jx = 0, jy = 0, jz = 0;
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      s += f[q];
      if (CX[q] != 0) jx += CX[q] * f[q];
      if (CY[q] != 0) jy += CY[q] * f[q];
      if (CZ[q] != 0) jz += CZ[q] * f[q];
    }
    const double r = a.rho_ref + s;
    rho[i] = r;
    psi[i] = psi_of(r, a.psi_rho0, 1.0 / a.psi_rho0);
    if (u) {
      u[i] = jx;
      u[n + i] = jy;
      u[2 * n + i] = jz;
    }
  }
}

// Shan-Chen force of node (x, y, z) from a float64 field of psi (computed
// once per node by the pass that wrote rho).
__device__ inline void force_from_psi(const double* __restrict__ psi, const Nbr& b,
                                      const StepArgs& a, double& Fx, double& Fy, double& Fz,
                                      double& psi_c) {
  double sx = 0, sy = 0, sz = 0;
#pragma unroll
  for (int q = 1; q < Q; ++q) {
    const unsigned idx = b.zo[1 + CZ[q]] + b.yo[1 + CY[q]] + b.xo[1 + CX[q]];
    const double wp = weight<double>(q) * psi[idx];
    if (CX[q] != 0) sx += CX[q] * wp;
    if (CY[q] != 0) sy += CY[q] * wp;
    if (CZ[q] != 0) sz += CZ[q] * wp;
  }
  psi_c = psi[b.zo[1] + b.yo[1] + b.xo[1]];
  Fx = -a.G * psi_c * sx;
  Fy = -a.G * psi_c * sy;
  Fz = -a.G * psi_c * sz;
}

// Pass 2: u^b = (j + F/2)/rho and the pressure of Eq. EOS_SC.
__global__ void __launch_bounds__(256)
k_moments2(const double* __restrict__ rho, const double* __restrict__ psi_f,
           double* __restrict__ u, double* __restrict__ p, StepArgs a) {
  const long long n = a.n;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x) {
    const int x = (int)(i % a.nx);
    const int y = (int)((i / a.nx) % a.ny);
    const int z = (int)(i / a.plane);
    const Nbr nb = neighbours(x, y, z, a.nx, a.ny, a.nz, a.plane);
    double Fx, Fy, Fz, psi;
    force_from_psi(psi_f, nb, a, Fx, Fy, Fz, psi);
    const double r = rho[i];
    if (u) {
      u[i] = (u[i] + 0.5 * Fx) / r;
      u[n + i] = (u[n + i] + 0.5 * Fy) / r;
      u[2 * n + i] = (u[2 * n + i] + 0.5 * Fz) / r;
    }
    if (p) p[i] = r / 3.0 + a.G * psi * psi / 6.0;
  }
}

// -------------------------------------------------------------- diagnostics
// Blocks of 256 threads own DIAG_CHUNK consecutive nodes of one z-slice, so a
// slice's liquid area is a sum of whole-block partials.  Each block writes 8
// partial sums: rho, jx, jy, jz, Fx, Fy, Fz, A.  Reductions run in a fixed
// order (per-thread serial, butterfly across the wavefront, waves in order),
// so results are bitwise reproducible.
constexpr int DIAG_CHUNK = 4096;
constexpr int DIAG_THREADS = 256;

__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

template <int NV>
__device__ inline void block_sums(double (&v)[NV], double* out) {
  __shared__ double red[DIAG_THREADS / 64][8];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < NV; ++k) v[k] = wave_sum(v[k]);
  if (lane == 0) {
#pragma unroll
    for (int k = 0; k < NV; ++k) red[wv][k] = v[k];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < NV; ++k) {
      double s = 0;
      for (int w = 0; w < DIAG_THREADS / 64; ++w) s += red[w][k];
      out[k] = s;
    }
  }
}

template <class T>
__global__ void __launch_bounds__(DIAG_THREADS)
k_diag1(const T* __restrict__ lat, double* __restrict__ rho, double* __restrict__ part,
        StepArgs a, int chunks_per_slice) {
  const int z = blockIdx.x / chunks_per_slice;
  const int c = blockIdx.x % chunks_per_slice;
  const int lo = c * DIAG_CHUNK, hi = min(a.plane, lo + DIAG_CHUNK);
  double v[4] = {0, 0, 0, 0};
  for (int i = lo + threadIdx.x; i < hi; i += DIAG_THREADS) {
    const int x = i % a.nx, y = i / a.nx;
    const Nbr nb = neighbours(x, y, z, a.nx, a.ny, a.nz, a.plane);
    double f[Q];
    pull<T, double>(lat, a.ps, nb, f);
    double s = 0, jx = 0, jy = 0, jz = 0;
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      s += f[q];
      if (CX[q] != 0) jx += CX[q] * f[q];
      if (CY[q] != 0) jy += CY[q] * f[q];
      if (CZ[q] != 0) jz += CZ[q] * f[q];
    }
    const double r = a.rho_ref + s;
    rho[(long long)z * a.plane + i] = r;
    rho[a.n + (long long)z * a.plane + i] = psi_of(r, a.psi_rho0, 1.0 / a.psi_rho0);
    v[0] += r;
    v[1] += jx;
    v[2] += jy;
    v[3] += jz;
  }
  block_sums<4>(v, part + (long long)blockIdx.x * 8);
}

__global__ void __launch_bounds__(DIAG_THREADS)
k_diag2(const double* __restrict__ rho, double* __restrict__ part, StepArgs a,
        int chunks_per_slice, double rho_v, double rho_l) {
  const int z = blockIdx.x / chunks_per_slice;
  const int c = blockIdx.x % chunks_per_slice;
  const int lo = c * DIAG_CHUNK, hi = min(a.plane, lo + DIAG_CHUNK);
  const double inv_dr = 1.0 / (rho_l - rho_v);
  double v[4] = {0, 0, 0, 0};
  for (int i = lo + threadIdx.x; i < hi; i += DIAG_THREADS) {
    const int x = i % a.nx, y = i / a.nx;
    const Nbr nb = neighbours(x, y, z, a.nx, a.ny, a.nz, a.plane);
    double Fx, Fy, Fz, psi;
    force_from_psi(rho + a.n, nb, a, Fx, Fy, Fz, psi);
    v[0] += Fx;
    v[1] += Fy;
    v[2] += Fz;
    const double fr = (rho[(long long)z * a.plane + i] - rho_v) * inv_dr;
    v[3] += fmin(fmax(fr, 0.0), 1.0);
  }
  block_sums<4>(v, part + (long long)blockIdx.x * 8 + 4);
}

// Final pass, one block: out[0] mass, out[1..3] momentum, out[4 + z] A(z).
__global__ void __launch_bounds__(DIAG_THREADS)
k_diag3(const double* __restrict__ part, double* __restrict__ out, int nz,
        int chunks_per_slice) {
  // A(z): one thread per slice, chunks in order.
  for (int z = threadIdx.x; z < nz; z += DIAG_THREADS) {
    double s = 0;
    for (int c = 0; c < chunks_per_slice; ++c) s += part[((long long)z * chunks_per_slice + c) * 8 + 7];
    out[4 + z] = s;
  }
  // Totals: each thread a strided serial sum over blocks, then the block tree.
  const long long nb = (long long)nz * chunks_per_slice;
  double v[7] = {0, 0, 0, 0, 0, 0, 0};
  for (long long b = threadIdx.x; b < nb; b += DIAG_THREADS) {
#pragma unroll
    for (int k = 0; k < 7; ++k) v[k] += part[b * 8 + k];
  }
  __shared__ double tot[8];
  block_sums<7>(v, tot);
  __syncthreads();
  if (threadIdx.x == 0) {
    out[0] = tot[0];
    out[1] = tot[1] + 0.5 * tot[4];
    out[2] = tot[2] + 0.5 * tot[5];
    out[3] = tot[3] + 0.5 * tot[6];
  }
}

int grid_for(long long n, int threads) {
  long long g = (n + threads - 1) / threads;
  if (g > 65536) g = 65536;
  if (g < 1) g = 1;
  return (int)g;
}

// ------------------------------------------------------------------ adjoint
// Reverse mode of one step.  Notation: B_n is the lattice written by step n
// (post-collision values at their own node), f_n(x)_a = B_{n-1}(x - c_a)_a the
// populations step n collides, rho_n their density.  The adjoint state between
// steps is (P, r) with dL/dB_n(y)_a = P(y + c_a)_a + r(y + c_a):
//   P(x)_a  adjoint of f_n(x)_a through the collision at x (incl. its
//           dependence on the moments rho(x), j(x));
//   r(x)    adjoint of rho_n(x) through psi, i.e. through the Shan-Chen
//           forces at x and at its 18 neighbours.
// Kernel A takes (P, r) of step n+1, forms dL/dB_n at every node, runs the
// collision backwards and writes P of step n and dL/dF; kernel B turns dL/dF
// into r of step n with the transposed force stencil.  Parameter gradients
// (dL/dG, dL/dtau and, for MRT, dL/ds_bulk, dL/ds_ghost) are accumulated per
// block in float64.

template <class T, int COLL>
__global__ void __launch_bounds__(256) k_adj_collide(AdjArgs g) {
  // float64 arithmetic for either storage type: the adjoint sums (the
  // equilibrium and source moments transposed, F-bar from sums of opposite
  // populations) cancel heavily, and in float32 their rounding alone moved
  // dL/dG of a 4000-step run by 1e-4 relative.
  using R = double;
  const StepArgs& a = g.a;
  const Phys<R> ph = make_phys<R>(a);
  const T* __restrict__ bprev = (const T*)g.bprev;
  const T* __restrict__ psi = (const T*)g.psi;
  const T* __restrict__ pn = (const T*)g.p_next;
  const T* __restrict__ rn = (const T*)g.r_next;
  T* __restrict__ po = (T*)g.p_out;
  T* __restrict__ pfb = (T*)g.psi_fbar;
  const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
  double dG = 0.0, dtau = 0.0, dbulk = 0.0, dghost = 0.0;
  if (i < a.n) {
    const int x = (int)(i % a.nx), y = (int)((i / a.nx) % a.ny), z = (int)(i / a.plane);
    const Nbr nb = neighbours(x, y, z, a.nx, a.ny, a.nz, a.plane);
    // The pulled populations stay in the storage type (exact; half the
    // registers for float32) and are widened where they are used.
    T f[Q];
    R gb[Q];
    pull<T, T>(bprev, a.ps, nb, f);
    // dL/dB_n(x)_b = P(x + c_b)_b + r(x + c_b)
    static_for<Q>([&](auto bc) {
      constexpr int b = decltype(bc)::value;
      const unsigned idx = nb.zo[1 + CZ[b]] + nb.yo[1 + CY[b]] + nb.xo[1 + CX[b]];
      gb[b] = R(pn[lat_index<T>(b, idx, a.ps)]) + R(rn[idx]);
    });
    // Shan-Chen force at x from the psi field of this step (as the forward
    // step computed it).
    R vx = R(0), vy = R(0), vz = R(0);
    static_for<Q - 1>([&](auto bc) {
      constexpr int b = decltype(bc)::value + 1;
      const unsigned idx = nb.zo[1 + CZ[b]] + nb.yo[1 + CY[b]] + nb.xo[1 + CX[b]];
      const R wp = weight<R>(b) * R(psi[idx]);
      if constexpr (CX[b] != 0) vx += R(CX[b]) * wp;
      if constexpr (CY[b] != 0) vy += R(CY[b]) * wp;
      if constexpr (CZ[b] != 0) vz += R(CZ[b]) * wp;
    });
    const R psi_c = R(psi[i]);
    const R gpsi = -ph.G * psi_c;
    const R Fx = gpsi * vx, Fy = gpsi * vy, Fz = gpsi * vz;
    // Forward moments (as in the collision).
    R s = R(0), jx = R(0), jy = R(0), jz = R(0);
    static_for<Q>([&](auto ac) {
      constexpr int q = decltype(ac)::value;
      s += R(f[q]);
      if constexpr (CX[q] != 0) jx += R(CX[q]) * R(f[q]);
      if constexpr (CY[q] != 0) jy += R(CY[q]) * R(f[q]);
      if constexpr (CZ[q] != 0) jz += R(CZ[q]) * R(f[q]);
    });
    const R rr = ph.rho_ref + s;
    const R inv = R(1) / rr;
    const R ux = (jx + R(0.5) * Fx) * inv, uy = (jy + R(0.5) * Fy) * inv,
            uz = (jz + R(0.5) * Fz) * inv;
    const R usq = ux * ux + uy * uy + uz * uz;
    const R uF = ux * Fx + uy * Fy + uz * Fz;
    // Adjoints of the collision inputs.
    R sb = R(0), rb = R(0), ubx = R(0), uby = R(0), ubz = R(0), Fbx = R(0), Fby = R(0),
      Fbz = R(0);
    R pout[Q];
    if constexpr (COLL == kBGK) {
      const R om = ph.omega, src = R(1) - R(0.5) * om;
      R T0 = R(0), T1x = R(0), T1y = R(0), T1z = R(0), Tcux = R(0), Tcuy = R(0), Tcuz = R(0),
        TcFx = R(0), TcFy = R(0), TcFz = R(0), Tq = R(0), dom = R(0);
      static_for<Q>([&](auto ac) {
        constexpr int q = decltype(ac)::value;
        const R w = weight<R>(q);
        R cu = R(0), cF = R(0);
        if constexpr (CX[q] != 0) { cu += R(CX[q]) * ux; cF += R(CX[q]) * Fx; }
        if constexpr (CY[q] != 0) { cu += R(CY[q]) * uy; cF += R(CY[q]) * Fy; }
        if constexpr (CZ[q] != 0) { cu += R(CZ[q]) * uz; cF += R(CZ[q]) * Fz; }
        const R t = w * gb[q];
        T0 += t;
        Tq += t * (R(3) * cu + R(4.5) * cu * cu);
        if constexpr (CX[q] != 0) { T1x += R(CX[q]) * t; Tcux += R(CX[q]) * t * cu; TcFx += R(CX[q]) * t * cF; }
        if constexpr (CY[q] != 0) { T1y += R(CY[q]) * t; Tcuy += R(CY[q]) * t * cu; TcFy += R(CY[q]) * t * cF; }
        if constexpr (CZ[q] != 0) { T1z += R(CZ[q]) * t; Tcuz += R(CZ[q]) * t * cu; TcFz += R(CZ[q]) * t * cF; }
        // d f*/d omega = (f_eq - f) - S / 2
        const R geq = w * s + w * rr * (R(3) * cu + R(4.5) * cu * cu - R(1.5) * usq);
        const R S = w * (R(3) * (cF - uF) + R(9) * cu * cF);
        dom += gb[q] * (geq - R(f[q]) - R(0.5) * S);
      });
      sb = om * T0;
      rb = om * (Tq - R(1.5) * usq * T0);
      ubx = om * rr * (R(3) * T1x + R(9) * Tcux - R(3) * ux * T0) + src * (R(9) * TcFx - R(3) * Fx * T0);
      uby = om * rr * (R(3) * T1y + R(9) * Tcuy - R(3) * uy * T0) + src * (R(9) * TcFy - R(3) * Fy * T0);
      ubz = om * rr * (R(3) * T1z + R(9) * Tcuz - R(3) * uz * T0) + src * (R(9) * TcFz - R(3) * Fz * T0);
      Fbx = src * (R(3) * T1x - R(3) * ux * T0 + R(9) * Tcux);
      Fby = src * (R(3) * T1y - R(3) * uy * T0 + R(9) * Tcuy);
      Fbz = src * (R(3) * T1z - R(3) * uz * T0 + R(9) * Tcuz);
      static_for<Q>([&](auto ac) { pout[decltype(ac)::value] = (R(1) - om) * gb[decltype(ac)::value]; });
      dtau = -double(dom) / (double(ph.tau) * double(ph.tau));
    } else {
      // Moments and closed-form equilibrium / source moments as in collide().
      const R ux2 = ux * ux, uy2 = uy * uy, uz2 = uz * uz;
      const R pxx = R(2) * ux2 - uy2 - uz2, pww = uy2 - uz2;
      const R sxx = R(2) * ux * Fx - uy * Fy - uz * Fz, sww = uy * Fy - uz * Fz;
      R meq[Q], msrc[Q];
      static_for<Q>([&](auto ic) { meq[decltype(ic)::value] = R(0); msrc[decltype(ic)::value] = R(0); });
      meq[1] = R(-11) * s + R(19) * rr * usq;  msrc[1] = R(38) * uF;
      meq[2] = R(3) * s - R(5.5) * rr * usq;   msrc[2] = R(-11) * uF;
      meq[4] = R(-2.0 / 3.0) * rr * ux;        msrc[4] = R(-2.0 / 3.0) * Fx;
      meq[6] = R(-2.0 / 3.0) * rr * uy;        msrc[6] = R(-2.0 / 3.0) * Fy;
      meq[8] = R(-2.0 / 3.0) * rr * uz;        msrc[8] = R(-2.0 / 3.0) * Fz;
      meq[9] = rr * pxx;                       msrc[9] = R(2) * sxx;
      meq[10] = R(-0.5) * rr * pxx;            msrc[10] = -sxx;
      meq[11] = rr * pww;                      msrc[11] = R(2) * sww;
      meq[12] = R(-0.5) * rr * pww;            msrc[12] = -sww;
      meq[13] = rr * ux * uy;                  msrc[13] = ux * Fy + uy * Fx;
      meq[14] = rr * uy * uz;                  msrc[14] = uy * Fz + uz * Fy;
      meq[15] = rr * ux * uz;                  msrc[15] = ux * Fz + uz * Fx;
      // kb_i = -sum_a M_ia gb_a; m_i = sum_b M_ib f_b
      R mb[Q], eqb[Q], srb[Q];
      R dlam = R(0), dlb = R(0), dlg = R(0);
      static_for<Q>([&](auto ic) {
        constexpr int ii = decltype(ic)::value;
        mb[ii] = R(0);
        eqb[ii] = R(0);
        srb[ii] = R(0);
        if constexpr (mrt_class(ii) != 0) {
          R kb = R(0), m = R(0);
          static_for<Q>([&](auto ac) {
            constexpr int q = decltype(ac)::value;
            if constexpr (mrt_entry(ii, q) != 0) {
              kb -= R(mrt_entry(ii, q)) * gb[q];
              m += R(mrt_entry(ii, q)) * R(f[q]);
            }
          });
          const R lam =
              mrt_class(ii) == 1 ? ph.s_bulk : (mrt_class(ii) == 2 ? ph.omega : ph.s_ghost);
          const R inv_d = R(1) / R(mrt_norm(ii));
          mb[ii] = kb * lam * inv_d;
          eqb[ii] = -kb * lam * inv_d;
          srb[ii] = -kb * (R(1) - R(0.5) * lam) * inv_d;
          // dm*_i / ds_i = -(m_i - meq_i) - msrc_i / 2, and dL/dm*_i = -kb_i / d_i.
          const R dls = kb * (m - meq[ii] + R(0.5) * msrc[ii]) * inv_d;
          if constexpr (mrt_class(ii) == 1) dlb += dls;
          if constexpr (mrt_class(ii) == 2) dlam += dls;
          if constexpr (mrt_class(ii) == 3) dlg += dls;
        }
      });
      dtau = -double(dlam) / (double(ph.tau) * double(ph.tau));
      dbulk = double(dlb);
      dghost = double(dlg);
      // F from the conserved momentum rows (D_a += 0.1 c_a . F)
      static_for<Q>([&](auto ac) {
        constexpr int q = decltype(ac)::value;
        if constexpr (CX[q] != 0) Fbx += R(0.1) * R(CX[q]) * gb[q];
        if constexpr (CY[q] != 0) Fby += R(0.1) * R(CY[q]) * gb[q];
        if constexpr (CZ[q] != 0) Fbz += R(0.1) * R(CZ[q]) * gb[q];
      });
      // Equilibrium moments back to (s, rho, u).
      sb += R(-11) * eqb[1] + R(3) * eqb[2];
      rb += usq * (R(19) * eqb[1] - R(5.5) * eqb[2]);
      const R eu = rr * (R(38) * eqb[1] - R(11) * eqb[2]);
      ubx += eu * ux;
      uby += eu * uy;
      ubz += eu * uz;
      rb += R(-2.0 / 3.0) * (ux * eqb[4] + uy * eqb[6] + uz * eqb[8]);
      ubx += R(-2.0 / 3.0) * rr * eqb[4];
      uby += R(-2.0 / 3.0) * rr * eqb[6];
      ubz += R(-2.0 / 3.0) * rr * eqb[8];
      const R e9 = eqb[9] - R(0.5) * eqb[10];
      rb += pxx * e9;
      ubx += rr * e9 * R(4) * ux;
      uby += rr * e9 * R(-2) * uy;
      ubz += rr * e9 * R(-2) * uz;
      const R e11 = eqb[11] - R(0.5) * eqb[12];
      rb += pww * e11;
      uby += rr * e11 * R(2) * uy;
      ubz += rr * e11 * R(-2) * uz;
      rb += ux * uy * eqb[13] + uy * uz * eqb[14] + ux * uz * eqb[15];
      ubx += rr * (uy * eqb[13] + uz * eqb[15]);
      uby += rr * (ux * eqb[13] + uz * eqb[14]);
      ubz += rr * (uy * eqb[14] + ux * eqb[15]);
      // Source moments back to (u, F).
      const R e1 = R(38) * srb[1] - R(11) * srb[2];
      ubx += e1 * Fx; uby += e1 * Fy; ubz += e1 * Fz;
      Fbx += e1 * ux; Fby += e1 * uy; Fbz += e1 * uz;
      Fbx += R(-2.0 / 3.0) * srb[4];
      Fby += R(-2.0 / 3.0) * srb[6];
      Fbz += R(-2.0 / 3.0) * srb[8];
      const R es = R(2) * srb[9] - srb[10];
      ubx += es * R(2) * Fx; uby -= es * Fy; ubz -= es * Fz;
      Fbx += es * R(2) * ux; Fby -= es * uy; Fbz -= es * uz;
      const R ew = R(2) * srb[11] - srb[12];
      uby += ew * Fy; ubz -= ew * Fz;
      Fby += ew * uy; Fbz -= ew * uz;
      ubx += srb[13] * Fy + srb[15] * Fz;
      uby += srb[13] * Fx + srb[14] * Fz;
      ubz += srb[14] * Fy + srb[15] * Fx;
      Fbx += srb[13] * uy + srb[15] * uz;
      Fby += srb[13] * ux + srb[14] * uz;
      Fbz += srb[14] * uy + srb[15] * ux;
      // Identity part plus M^T mb.
      static_for<Q>([&](auto ac) {
        constexpr int q = decltype(ac)::value;
        R acc = gb[q];
        static_for<Q>([&](auto ic) {
          constexpr int ii = decltype(ic)::value;
          if constexpr (mrt_class(ii) != 0 && mrt_entry(ii, q) != 0)
            acc += R(mrt_entry(ii, q)) * mb[ii];
        });
        pout[q] = acc;
      });
    }
    // u = (j + F/2) / rho, rho = rho_ref + s.
    const R jbx = ubx * inv, jby = uby * inv, jbz = ubz * inv;
    Fbx += R(0.5) * jbx;
    Fby += R(0.5) * jby;
    Fbz += R(0.5) * jbz;
    rb -= (ubx * ux + uby * uy + ubz * uz) * inv;
    sb += rb;
    static_for<Q>([&](auto ac) {
      constexpr int q = decltype(ac)::value;
      R v = pout[q] + sb;
      if constexpr (CX[q] != 0) v += R(CX[q]) * jbx;
      if constexpr (CY[q] != 0) v += R(CY[q]) * jby;
      if constexpr (CZ[q] != 0) v += R(CZ[q]) * jbz;
      po[lat_index<T>(q, (unsigned)i, a.ps)] = T(v);
    });
    // For kernel B: the local half of dL/dpsi(x) and the field its
    // transposed stencil gathers.
    static_cast<T*>(g.fbar_dot_v)[i] = T(Fbx * vx + Fby * vy + Fbz * vz);
    pfb[i] = T(psi_c * Fbx);
    pfb[a.n + i] = T(psi_c * Fby);
    pfb[2 * a.n + i] = T(psi_c * Fbz);
    // dL/dG: F is linear in G.
    if (a.G != 0.0)
      dG = (double(Fbx) * double(Fx) + double(Fby) * double(Fy) + double(Fbz) * double(Fz)) / a.G;
  }
  // This block's partials accumulate over every step of the backward pass and
  // are reduced once at its end (fixed order: steps, then blocks).
  double v[4] = {dG, dtau, dbulk, dghost};
  __shared__ double tot[4];
  block_sums<4>(v, tot);
  if (threadIdx.x == 0) {
    double* pp = g.partial + 4LL * blockIdx.x;
#pragma unroll
    for (int k = 0; k < 4; ++k) pp[k] += tot[k];
  }
}

// r(x) = psi'(rho(x)) * dL/dpsi(x), with
// dL/dpsi(x) = -G [ Fb(x) . sum_b w_b psi(x + c_b) c_b
//                   + sum_b w_b c_b . (psi Fb)(x - c_b) ].
// Kernel A stored the first term's dot product and the field psi Fb.
template <class T>
__global__ void __launch_bounds__(256) k_adj_psi(AdjArgs g) {
  using R = double;  // as in k_adj_collide
  const StepArgs& a = g.a;
  const Phys<R> ph = make_phys<R>(a);
  const T* __restrict__ psi = (const T*)g.psi;
  const T* __restrict__ t1v = (const T*)g.fbar_dot_v;
  const T* __restrict__ pfb = (const T*)g.psi_fbar;
  T* __restrict__ ro = (T*)g.r_out;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < a.n;
       i += (long long)gridDim.x * blockDim.x) {
    const int x = (int)(i % a.nx), y = (int)((i / a.nx) % a.ny), z = (int)(i / a.plane);
    const Nbr nb = neighbours(x, y, z, a.nx, a.ny, a.nz, a.plane);
    R t2 = R(0);
    static_for<Q - 1>([&](auto bc) {
      constexpr int b = decltype(bc)::value + 1;
      const unsigned im = nb.zo[1 - CZ[b]] + nb.yo[1 - CY[b]] + nb.xo[1 - CX[b]];
      R ch = R(0);
      if constexpr (CX[b] != 0) ch += R(CX[b]) * R(pfb[im]);
      if constexpr (CY[b] != 0) ch += R(CY[b]) * R(pfb[a.n + im]);
      if constexpr (CZ[b] != 0) ch += R(CZ[b]) * R(pfb[2 * a.n + im]);
      t2 += weight<R>(b) * ch;
    });
    // psi' = exp(-rho / rho0) = 1 - psi / rho0.
    const R dpsi = R(1) - R(psi[i]) * ph.inv_psi_rho0;
    ro[i] = T(-ph.G * (R(t1v[i]) + t2) * dpsi);
  }
}

// Terminal adjoint: P = 0, r = dL/drho of the final state.
template <class T>
__global__ void __launch_bounds__(256) k_adj_seed(AdjArgs g, const double* __restrict__ rhobar) {
  T* __restrict__ po = (T*)g.p_out;
  T* __restrict__ ro = (T*)g.r_out;
  const StepArgs& a = g.a;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < a.n;
       i += (long long)gridDim.x * blockDim.x) {
#pragma unroll
    for (int q = 0; q < Q; ++q) po[lat_index<T>(q, (unsigned)i, a.ps)] = T(0);
    ro[i] = T(rhobar[i]);
  }
}

// dL/drho0(x) = sum_a w_a P(x)_a + r(x)  (the initial state is f_a = w_a rho0).
template <class T>
__global__ void __launch_bounds__(256) k_adj_final(AdjArgs g, double* __restrict__ rho0bar) {
  const T* __restrict__ pn = (const T*)g.p_next;
  const T* __restrict__ rn = (const T*)g.r_next;
  const StepArgs& a = g.a;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < a.n;
       i += (long long)gridDim.x * blockDim.x) {
    double s = 0.0;
#pragma unroll
    for (int q = 0; q < Q; ++q)
      s += weight<double>(q) * double(pn[lat_index<T>(q, (unsigned)i, a.ps)]);
    rho0bar[i] = s + double(rn[i]);
  }
}

// acc[0..3] += sum of nb block partials (dL/dG, dL/dtau, dL/ds_bulk,
// dL/ds_ghost), in a fixed order.
__global__ void __launch_bounds__(256) k_adj_reduce(const double* __restrict__ part, int nb,
                                                    double* __restrict__ acc) {
  double v[4] = {0.0, 0.0, 0.0, 0.0};
  for (int b = threadIdx.x; b < nb; b += 256) {
#pragma unroll
    for (int k = 0; k < 4; ++k) v[k] += part[4LL * b + k];
  }
  __shared__ double tot[4];
  block_sums<4>(v, tot);
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < 4; ++k) acc[k] += tot[k];
  }
}

// Gradient of the minimum radius r_min = min_z sqrt(A(z)/pi) with respect to
// rho (field given in `rho`, overwritten): only the argmin slice, and only
// nodes strictly between rho_v and rho_l, carry 1 / (2 pi r_min (rho_l - rho_v)).
__global__ void __launch_bounds__(256) k_rmin_grad(double* __restrict__ rho, StepArgs a, int zstar,
                                                   double coef, double rho_v, double rho_l) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < a.n;
       i += (long long)gridDim.x * blockDim.x) {
    const int z = (int)(i / a.plane);
    const double r = rho[i];
    rho[i] = (z == zstar && r > rho_v && r < rho_l) ? coef : 0.0;
  }
}

}  // namespace

// ---------------------------------------------------------------- launchers
hipError_t launch_init(int prec, void* lat, const double* rho0, const StepArgs& a,
                       hipStream_t s) {
  const int g = grid_for(a.n, 256);
  if (prec == 0)
    hipLaunchKernelGGL(k_init<double>, dim3(g), dim3(256), 0, s, (double*)lat, rho0, a);
  else
    hipLaunchKernelGGL(k_init<float>, dim3(g), dim3(256), 0, s, (float*)lat, rho0, a);
  return hipGetLastError();
}

template <class T, int COLL, int FORC, int NT>
static void step_nt(int npt, int grid, size_t lds, const T* in, T* out, const StepArgs& a,
                    hipStream_t s) {
  if (npt == 2)
    hipLaunchKernelGGL((k_step<T, COLL, FORC, NT, 2>), dim3(grid), dim3(NT), lds, s, in, out, a);
  else
    hipLaunchKernelGGL((k_step<T, COLL, FORC, NT, 1>), dim3(grid), dim3(NT), lds, s, in, out, a);
}

template <class T, int COLL, int FORC>
static hipError_t step_t(int threads, int npt, const void* src, void* dst, const StepArgs& a,
                         hipStream_t s) {
  const int grid = a.ntiles_x * a.ntiles_y * ((a.nz + a.zchunk - 1) / a.zchunk);
  const size_t lds = (size_t)4 * (a.by + 2) * (a.bx + 2) * sizeof(T);
  if ((long long)a.by * a.bx > (long long)npt * threads) return hipErrorInvalidValue;
  const T* in = (const T*)src;
  T* out = (T*)dst;
  switch (threads) {
    case 256: step_nt<T, COLL, FORC, 256>(npt, grid, lds, in, out, a, s); break;
    case 512: step_nt<T, COLL, FORC, 512>(npt, grid, lds, in, out, a, s); break;
    default: step_nt<T, COLL, FORC, 1024>(npt, grid, lds, in, out, a, s); break;
  }
  return hipGetLastError();
}

template <class T, int COLL, int FORC>
static hipError_t step_two_t(const void* src, void* psi, void* dst, const StepArgs& a,
                             hipStream_t s) {
  const int g = grid_for(a.n, 256);
  hipLaunchKernelGGL(k_density_psi<T>, dim3(g), dim3(256), 0, s, (const T*)src, (T*)psi, a);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_step_psi<T, COLL, FORC>), dim3(g), dim3(256), 0, s, (const T*)src,
                     (const T*)psi, (T*)dst, a);
  return hipGetLastError();
}

hipError_t launch_step_two_kernel(int prec, int coll, int forc, const void* src, void* psi,
                                  void* dst, const StepArgs& a, hipStream_t s) {
  if (prec == 0) {
    if (coll == kMRT) return step_two_t<double, kMRT, kGuo>(src, psi, dst, a, s);
    if (forc == kShift) return step_two_t<double, kBGK, kShift>(src, psi, dst, a, s);
    return step_two_t<double, kBGK, kGuo>(src, psi, dst, a, s);
  }
  if (coll == kMRT) return step_two_t<float, kMRT, kGuo>(src, psi, dst, a, s);
  if (forc == kShift) return step_two_t<float, kBGK, kShift>(src, psi, dst, a, s);
  return step_two_t<float, kBGK, kGuo>(src, psi, dst, a, s);
}

hipError_t launch_step(int prec, int coll, int forc, int threads, int npt, const void* src,
                       void* dst, const StepArgs& a, hipStream_t s) {
  if (prec == 0) {
    if (coll == kMRT) return step_t<double, kMRT, kGuo>(threads, npt, src, dst, a, s);
    if (forc == kShift) return step_t<double, kBGK, kShift>(threads, npt, src, dst, a, s);
    return step_t<double, kBGK, kGuo>(threads, npt, src, dst, a, s);
  }
  if (coll == kMRT) return step_t<float, kMRT, kGuo>(threads, npt, src, dst, a, s);
  if (forc == kShift) return step_t<float, kBGK, kShift>(threads, npt, src, dst, a, s);
  return step_t<float, kBGK, kGuo>(threads, npt, src, dst, a, s);
}

template <class T, int COLL, int FORC, int NT, int K>
static hipError_t batch_nt_k(const BatchLaunch& L, hipStream_t s) {
  if (!L.persistent) {
    hipLaunchKernelGGL((k_step_batch<T, COLL, FORC, NT, K>), dim3(L.ntiles), dim3(NT), L.lds, s,
                       L.members, L.tiles, L.parity, L.remap);
    return hipGetLastError();
  }
  int per_cu = 0, cus = 0, dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (e == hipSuccess)
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
        &per_cu, reinterpret_cast<const void*>(&k_step_persistent<T, COLL, FORC, NT, K>), NT,
        L.lds);
  if (e != hipSuccess) return e;
  if (per_cu < 1) return hipErrorInvalidConfiguration;
  int grid = per_cu * cus;
  if (grid > L.ntiles) grid = L.ntiles;
  const BatchMember* mem = L.members;
  const int4* tiles = L.tiles;
  int ntiles = L.ntiles, parity = L.parity, nsteps = L.nsteps;
  unsigned* sync = L.sync;
  unsigned spin = L.spin_limit;
  void* args[] = {&mem, &tiles, &ntiles, &parity, &nsteps, &sync, &spin};
  return hipLaunchCooperativeKernel(
      reinterpret_cast<const void*>(&k_step_persistent<T, COLL, FORC, NT, K>), dim3(grid),
      dim3(NT), args, (unsigned)L.lds, s);
}

template <class T, int COLL, int FORC>
static hipError_t batch_t(const BatchLaunch& L, hipStream_t s) {
  if (L.npt == 2) {
    switch (L.threads) {
      case 256: return batch_nt_k<T, COLL, FORC, 256, 2>(L, s);
      case 512: return batch_nt_k<T, COLL, FORC, 512, 2>(L, s);
      default: return batch_nt_k<T, COLL, FORC, 1024, 2>(L, s);
    }
  }
  switch (L.threads) {
    case 256: return batch_nt_k<T, COLL, FORC, 256, 1>(L, s);
    case 512: return batch_nt_k<T, COLL, FORC, 512, 1>(L, s);
    default: return batch_nt_k<T, COLL, FORC, 1024, 1>(L, s);
  }
}

hipError_t launch_batch(const BatchLaunch& L, hipStream_t s) {
  if (L.prec == 0) {
    if (L.coll == kMRT) return batch_t<double, kMRT, kGuo>(L, s);
    if (L.forc == kShift) return batch_t<double, kBGK, kShift>(L, s);
    return batch_t<double, kBGK, kGuo>(L, s);
  }
  if (L.coll == kMRT) return batch_t<float, kMRT, kGuo>(L, s);
  if (L.forc == kShift) return batch_t<float, kBGK, kShift>(L, s);
  return batch_t<float, kBGK, kGuo>(L, s);
}

hipError_t launch_moments(int prec, const void* lat, double* rho, double* u, double* p,
                          double* psi_scratch, const StepArgs& a, hipStream_t s) {
  const int g = grid_for(a.n, 256);
  if (prec == 0)
    hipLaunchKernelGGL(k_moments1<double>, dim3(g), dim3(256), 0, s, (const double*)lat, rho, u,
                       psi_scratch, a);
  else
    hipLaunchKernelGGL(k_moments1<float>, dim3(g), dim3(256), 0, s, (const float*)lat, rho, u,
                       psi_scratch, a);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (u || p) {
    hipLaunchKernelGGL(k_moments2, dim3(g), dim3(256), 0, s, (const double*)rho,
                       (const double*)psi_scratch, u, p, a);
    e = hipGetLastError();
  }
  return e;
}

int diag_blocks(const StepArgs& a) {
  const int cps = (a.plane + DIAG_CHUNK - 1) / DIAG_CHUNK;
  return cps * a.nz;
}

hipError_t launch_diagnostics(int prec, const void* lat, double* rho_scratch, double* part,
                              double* out, double rho_v, double rho_l, const StepArgs& a,
                              hipStream_t s) {
  const int cps = (a.plane + DIAG_CHUNK - 1) / DIAG_CHUNK;
  const int nb = cps * a.nz;
  if (prec == 0)
    hipLaunchKernelGGL(k_diag1<double>, dim3(nb), dim3(DIAG_THREADS), 0, s, (const double*)lat,
                       rho_scratch, part, a, cps);
  else
    hipLaunchKernelGGL(k_diag1<float>, dim3(nb), dim3(DIAG_THREADS), 0, s, (const float*)lat,
                       rho_scratch, part, a, cps);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_diag2, dim3(nb), dim3(DIAG_THREADS), 0, s, (const double*)rho_scratch,
                     part, a, cps, rho_v, rho_l);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_diag3, dim3(1), dim3(DIAG_THREADS), 0, s, (const double*)part, out, a.nz,
                     cps);
  return hipGetLastError();
}

hipError_t launch_gather(int prec, const void* lat, long long ps_in, void* out, long long ps_out,
                         const StepArgs& a, hipStream_t s) {
  const int g = grid_for(a.n, 256);
  if (prec == 0)
    hipLaunchKernelGGL(k_gather<double>, dim3(g), dim3(256), 0, s, (const double*)lat, ps_in,
                       (double*)out, ps_out, a);
  else
    hipLaunchKernelGGL(k_gather<float>, dim3(g), dim3(256), 0, s, (const float*)lat, ps_in,
                       (float*)out, ps_out, a);
  return hipGetLastError();
}

hipError_t launch_scatter(int prec, const void* in, long long ps_in, void* lat, long long ps_out,
                          const StepArgs& a, hipStream_t s) {
  const int g = grid_for(a.n, 256);
  if (prec == 0)
    hipLaunchKernelGGL(k_scatter<double>, dim3(g), dim3(256), 0, s, (const double*)in, ps_in,
                       (double*)lat, ps_out, a);
  else
    hipLaunchKernelGGL(k_scatter<float>, dim3(g), dim3(256), 0, s, (const float*)in, ps_in,
                       (float*)lat, ps_out, a);
  return hipGetLastError();
}

int adj_blocks(const StepArgs& a) { return (int)((a.n + 255) / 256); }

hipError_t launch_adjoint_reduce(const AdjArgs& g, double* acc, hipStream_t s) {
  hipLaunchKernelGGL(k_adj_reduce, dim3(1), dim3(256), 0, s, (const double*)g.partial,
                     adj_blocks(g.a), acc);
  return hipGetLastError();
}

hipError_t launch_adjoint_step(int prec, int coll, const AdjArgs& g, hipStream_t s) {
  const int nb = adj_blocks(g.a);
  if (prec == 0) {
    if (coll == kMRT)
      hipLaunchKernelGGL((k_adj_collide<double, kMRT>), dim3(nb), dim3(256), 0, s, g);
    else
      hipLaunchKernelGGL((k_adj_collide<double, kBGK>), dim3(nb), dim3(256), 0, s, g);
  } else {
    if (coll == kMRT)
      hipLaunchKernelGGL((k_adj_collide<float, kMRT>), dim3(nb), dim3(256), 0, s, g);
    else
      hipLaunchKernelGGL((k_adj_collide<float, kBGK>), dim3(nb), dim3(256), 0, s, g);
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int gp = grid_for(g.a.n, 256);
  if (prec == 0)
    hipLaunchKernelGGL(k_adj_psi<double>, dim3(gp), dim3(256), 0, s, g);
  else
    hipLaunchKernelGGL(k_adj_psi<float>, dim3(gp), dim3(256), 0, s, g);
  return hipGetLastError();
}

hipError_t launch_adjoint_seed(int prec, const AdjArgs& g, const double* rhobar, hipStream_t s) {
  const int gp = grid_for(g.a.n, 256);
  if (prec == 0)
    hipLaunchKernelGGL(k_adj_seed<double>, dim3(gp), dim3(256), 0, s, g, rhobar);
  else
    hipLaunchKernelGGL(k_adj_seed<float>, dim3(gp), dim3(256), 0, s, g, rhobar);
  return hipGetLastError();
}

hipError_t launch_adjoint_final(int prec, const AdjArgs& g, double* rho0bar, hipStream_t s) {
  const int gp = grid_for(g.a.n, 256);
  if (prec == 0)
    hipLaunchKernelGGL(k_adj_final<double>, dim3(gp), dim3(256), 0, s, g, rho0bar);
  else
    hipLaunchKernelGGL(k_adj_final<float>, dim3(gp), dim3(256), 0, s, g, rho0bar);
  return hipGetLastError();
}

hipError_t launch_rmin_grad(double* rho, const StepArgs& a, int zstar, double coef, double rho_v,
                            double rho_l, hipStream_t s) {
  hipLaunchKernelGGL(k_rmin_grad, dim3(grid_for(a.n, 256)), dim3(256), 0, s, rho, a, zstar, coef,
                     rho_v, rho_l);
  return hipGetLastError();
}

void lattice_tables(int32_t* c, double* w) {
  for (int q = 0; q < Q; ++q) {
    if (c) {
      c[3 * q + 0] = CX[q];
      c[3 * q + 1] = CY[q];
      c[3 * q + 2] = CZ[q];
    }
    if (w) w[q] = weight<double>(q);
  }
}

}  // namespace lbsc
