// Windowed direct sum of eq. (2.10): every packet evaluated at every grid
// point within its window, on gfx950.
//
// Pipeline (all on the caller's stream):
//   1. ds_key      per packet: its spatial bin (from its nearest grid index);
//   2. positions   counting sort of the bins (sort.hip), then ds_prep writes
//                  each packet's record straight to its sorted position: the
//                  nearest grid index and offset, the phase at that point and
//                  its per-step increment (revolutions, FP64, reduced mod 1),
//                  and log|scale a|;
//   3. ds_kernel   gather: a workgroup owns a tile of output points and walks
//                  the packets of the bins its tile can see.  Packet records
//                  are wave-uniform and are read into scalar registers through
//                  the scalar cache; each lane owns four points and accumulates
//                  their sums.  Per point: the Gaussian and the window test in
//                  FP32 with v_exp_f32, the phase from FP64 (one FMA per
//                  dimension and v_fract_f64), then v_sin_f32 / v_cos_f32 on
//                  the reduced revolution count; FP32 partial sums of at most 32
//                  packets are flushed into FP64 accumulators.  The FP64 variant
//                  does the same arithmetic in FP64 (OCML exp, sincospi).
//   4. ds_reduce   sum of the per-chunk partial grids, conversion to the
//                  output precision.
#include "common.h"

namespace fggc {
namespace {

constexpr int kBlock = 256;  // 4 waves
constexpr int kFlush = 32;   // packets per FP32 partial sum

__device__ __forceinline__ int64_t floordiv(int64_t a, int64_t b) {
  int64_t q = a / b;
  return (a % b != 0 && ((a < 0) != (b < 0))) ? q - 1 : q;
}
__device__ __forceinline__ int64_t imod(int64_t a, int64_t m) {
  int64_t r = a % m;
  return r < 0 ? r + m : r;
}

struct PrepParams {
  int d;
  int64_t N;
  const double *Q, *P, *S, *a;
  double eps, scale;
  int64_t n[3];
  double dx[3];
  int64_t binw[3], nbin[3];
};

// nearest grid index of coordinate q (position from x_0 = -pi wrapped into
// [0, 2 pi)) and the offset Q - x_m, |offset| <= dx/2
__device__ __forceinline__ int64_t nearest_index(double q, double dx, int64_t n, double &delta) {
  const double t = (q + kPi) - kTwoPi * floor((q + kPi) / kTwoPi);
  const double m = rint(t / dx);
  delta = fma(-m, dx, t);
  int64_t mi = (int64_t)m;
  if (mi >= n) mi -= n;
  return mi;
}

__global__ void ds_key_kernel(PrepParams p, uint32_t *__restrict__ key) {
  const int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (j >= p.N) return;
  uint32_t bin = 0;
  for (int k = 0; k < p.d; ++k) {
    double delta;
    const int64_t mi = nearest_index(p.Q[k * p.N + j], p.dx[k], p.n[k], delta);
    bin = bin * (uint32_t)p.nbin[k] + (uint32_t)(mi / p.binw[k]);
  }
  key[j] = bin;
}

__global__ void ds_prep_kernel(PrepParams p, const uint32_t *__restrict__ pos, DsRec *__restrict__ rec) {
  const int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (j >= p.N) return;
  DsRec r;
  r.pad = 0;
  for (int k = 0; k < 3; ++k) {
    r.deltaf[k] = 0.0f;
    r.mq[k] = 0;
    r.delta[k] = 0.0;
    r.omega[k] = 0.0;
  }
  double pdelta = 0.0;
  for (int k = 0; k < p.d; ++k) {
    double delta;
    const int64_t mi = nearest_index(p.Q[k * p.N + j], p.dx[k], p.n[k], delta);
    r.mq[k] = (int32_t)mi;
    r.delta[k] = delta;
    r.deltaf[k] = (float)delta;
    const double Pk = p.P[k * p.N + j];
    pdelta = fma(Pk, delta, pdelta);
    const double w = Pk / (p.eps * (double)p.n[k]);  // P dx / (2 pi eps)
    r.omega[k] = w - floor(w);
  }
  const double are = p.scale * p.a[2 * j], aim = p.scale * p.a[2 * j + 1];
  r.lnamp = log(hypot(are, aim));
  r.la2 = (float)(r.lnamp * 1.4426950408889634);
  const double ph = (p.S[j] - pdelta) / (kTwoPi * p.eps) + atan2(aim, are) * (1.0 / kTwoPi);
  r.phi0 = ph - floor(ph);
  rec[pos[j]] = r;
}

// Lane / sub-tile / wave layout of a workgroup tile for each dimension count.
// Each lane owns 4 points (sub-tiles); a wave covers L*S points per
// dimension, a workgroup (4 waves) L*S*V.
template <int D> struct Shape;
template <> struct Shape<1> {
  static constexpr int L[3] = {64, 1, 1}, S[3] = {4, 1, 1}, V[3] = {4, 1, 1};
};
template <> struct Shape<2> {
  static constexpr int L[3] = {8, 8, 1}, S[3] = {2, 2, 1}, V[3] = {2, 2, 1};
};
template <> struct Shape<3> {
  static constexpr int L[3] = {4, 4, 4}, S[3] = {1, 2, 2}, V[3] = {4, 1, 1};
};

struct DsParams {
  const DsRec *rec;        // sorted by bin
  const int64_t *start;    // [nbins + 1]
  int64_t n[3], binw[3], nbin[3];
  int64_t box_lo[3], box_n[3];
  int64_t ntile[3];        // tiles per dimension over the box
  int64_t W[3];            // window half-width in grid steps per dimension
  double dx[3];
  double R2;               // window radius squared
  double gauss;            // -1/(2 eps)
  int nchunk;
  int lanewrap;            // grid too small for a wave span: wrap every lane
  double *partial;         // [nchunk][prod box_n] complex FP64
};

// WRAP: grids too small for a wave's span, where every lane takes its own
// minimum image (a separate instantiation keeps that path's registers out of
// the common one)
template <int D, bool F64, bool WRAP>
__global__ __launch_bounds__(kBlock) void ds_kernel(DsParams p) {
  using Sh = Shape<D>;
  const int lane = threadIdx.x & 63;
  // the wave index is uniform across the wave: keep it (and all that derives
  // from it) in scalar registers so that window tests branch on the SALU
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);

  // tile and chunk of this workgroup
  int64_t tile = blockIdx.x, torg[3] = {0, 0, 0};
  for (int k = D - 1; k >= 0; --k) {
    torg[k] = p.box_lo[k] + (tile % p.ntile[k]) * (Sh::L[k] * Sh::S[k] * Sh::V[k]);
    tile /= p.ntile[k];
  }
  int lw[3], ll[3];
  {
    int w = wave, l = lane;
    for (int k = D - 1; k >= 0; --k) {
      lw[k] = w % Sh::V[k];
      w /= Sh::V[k];
      ll[k] = l % Sh::L[k];
      l /= Sh::L[k];
    }
  }
  int64_t worg[3] = {0, 0, 0};  // wave origin (grid index)
  for (int k = 0; k < D; ++k) worg[k] = torg[k] + lw[k] * (Sh::L[k] * Sh::S[k]);

  // per-lane offsets of the 4 owned points from the wave origin, and the
  // (wave-uniform) offsets of the 4 sub-tiles
  float offf[4][3];
  double offd[4][3];
  int subo[4][3];
  for (int s = 0; s < 4; ++s) {
    int ss = s;
    for (int k = D - 1; k >= 0; --k) {
      int sk = ss % Sh::S[k];
      ss /= Sh::S[k];
      subo[s][k] = sk * Sh::L[k];
      int o = sk * Sh::L[k] + ll[k];
      offf[s][k] = (float)o;
      offd[s][k] = (double)o;
    }
  }
  int nn[3], hh[3], Wi[3];
  for (int k = 0; k < 3; ++k) {
    nn[k] = (int)p.n[k];
    hh[k] = nn[k] / 2;
    Wi[k] = (int)p.W[k];
  }

  // bins visible from the tile: grid points [torg - W, torg + span - 1 + W]
  // per dimension, taken modulo n, as at most two bin intervals
  int64_t ia[3][2], ic[3][2], ilen[3][2], bcount[3];
  int nint[3];
  for (int k = 0; k < 3; ++k) {
    nint[k] = 1;
    ia[k][0] = ic[k][0] = 0;
    ilen[k][0] = 1;
    ilen[k][1] = 0;
    bcount[k] = 1;
  }
  for (int k = 0; k < D; ++k) {
    const int64_t span = Sh::L[k] * Sh::S[k] * Sh::V[k];
    const int64_t lo = torg[k] - p.W[k], hi = torg[k] + span - 1 + p.W[k];
    const int64_t nk = p.n[k], nb = p.nbin[k], bw = p.binw[k];
    if (hi - lo + 1 >= nk) {
      nint[k] = 1;
      ia[k][0] = 0;
      ic[k][0] = nb - 1;
    } else {
      const int64_t lm = imod(lo, nk), hm = imod(hi, nk);
      if (lm <= hm) {
        nint[k] = 1;
        ia[k][0] = lm / bw;
        ic[k][0] = hm / bw;
      } else if (hm / bw + 1 >= lm / bw) {
        nint[k] = 1;  // the two pieces touch: every bin
        ia[k][0] = 0;
        ic[k][0] = nb - 1;
      } else {
        nint[k] = 2;
        ia[k][0] = lm / bw;
        ic[k][0] = nb - 1;
        ia[k][1] = 0;
        ic[k][1] = hm / bw;
      }
    }
    ilen[k][0] = ic[k][0] - ia[k][0] + 1;
    ilen[k][1] = nint[k] == 2 ? ic[k][1] - ia[k][1] + 1 : 0;
    bcount[k] = ilen[k][0] + ilen[k][1];
  }
  // visible bins form rows (all but the last dimension), each holding at most
  // two contiguous runs in bin order; count packets, then take this chunk.
  int64_t nrows = 1;
  for (int k = 0; k < D - 1; ++k) nrows *= bcount[k];
  const int kl = D - 1;
  int64_t total = 0;
  auto row_base = [&](int64_t row) {
    int64_t rr = row, idx[3] = {0, 0, 0};
    for (int k = D - 2; k >= 0; --k) {
      const int64_t r = rr % bcount[k];
      rr /= bcount[k];
      idx[k] = r < ilen[k][0] ? ia[k][0] + r : ia[k][1] + (r - ilen[k][0]);
    }
    int64_t b = 0;
    for (int k = 0; k < D - 1; ++k) b = b * p.nbin[k] + idx[k];
    return b * p.nbin[kl];
  };
  for (int64_t row = 0; row < nrows; ++row) {
    const int64_t base = row_base(row);
    for (int run = 0; run < nint[kl]; ++run)
      total += p.start[base + ic[kl][run] + 1] - p.start[base + ia[kl][run]];
  }
  const int64_t v0 = total * blockIdx.y / p.nchunk, v1 = total * (blockIdx.y + 1) / p.nchunk;

  // accumulators
  float a32r[4] = {0, 0, 0, 0}, a32i[4] = {0, 0, 0, 0};
  double a64r[4] = {0, 0, 0, 0}, a64i[4] = {0, 0, 0, 0};
  int pending = 0;

  const float R2f = (float)p.R2;
  const float gl2 = (float)(p.gauss * 1.4426950408889634);  // -log2(e) / (2 eps)
  float dxf[3];
  for (int k = 0; k < 3; ++k) dxf[k] = (float)p.dx[k];

  int64_t vbase = 0;
  for (int64_t row = 0; row < nrows && vbase < v1; ++row) {
    const int64_t base = row_base(row);
    for (int run = 0; run < nint[kl]; ++run) {
      const int64_t ca = ia[kl][run], cb = ic[kl][run] + 1;
      const int64_t sa = p.start[base + ca], sb = p.start[base + cb];
      const int64_t len = sb - sa;
      int64_t lo = v0 - vbase, hi = v1 - vbase;
      if (lo < 0) lo = 0;
      if (hi > len) hi = len;
      if (lo >= hi) {
        vbase += len;
        continue;
      }
      // software pipeline: the next record is requested before this one is used
      DsRec nxt = p.rec[sa + lo];
      for (int64_t v = lo; v < hi; ++v) {
        const DsRec r = nxt;
        nxt = p.rec[sa + (v + 1 < hi ? v + 1 : v)];
        // displacement (in grid steps) of the wave origin from the packet, minimum image
        int kb[3];
        bool vis = true;
        for (int k = 0; k < D; ++k) {
          int kv = (int)(worg[k] - r.mq[k]);  // in (-n, n + span)
          if constexpr (WRAP) {
            while (kv >= nn[k] - hh[k]) kv -= nn[k];
            while (kv < -hh[k]) kv += nn[k];
          } else {
            // grids at least twice (tile span + window) wide: one correction suffices
            if (kv < -hh[k]) kv += nn[k];
            else if (kv >= nn[k] - hh[k]) kv -= nn[k];
          }
          kb[k] = kv;
          const int span = Sh::L[k] * Sh::S[k];
          vis = vis && (unsigned)(kv + span - 1 + Wi[k]) < (unsigned)(2 * Wi[k] + span);
        }
        if constexpr (WRAP) {
          // small grids: a wave span can wrap around the torus and come back
          // inside the window, so every lane takes its own minimum image
          for (int s = 0; s < 4; ++s) {
            double y2 = 0.0, th = r.phi0;
            for (int k = 0; k < D; ++k) {
              int kk = kb[k] + subo[s][k] + ll[k];
              if (kk >= nn[k] - hh[k]) kk -= nn[k];
              const double y = fma((double)kk, p.dx[k], -r.delta[k]);
              y2 = fma(y, y, y2);
              th = fma((double)kk, r.omega[k], th);
            }
            if (y2 <= p.R2) {
              const double g = exp(fma(y2, p.gauss, r.lnamp));
              double sn, cs;
              sincospi(2.0 * __builtin_amdgcn_fract(th), &sn, &cs);
              a64r[s] = fma(g, cs, a64r[s]);
              a64i[s] = fma(g, sn, a64i[s]);
            }
          }
          continue;
        }
        if (!vis) continue;
        double thb = r.phi0;
        for (int k = 0; k < D; ++k) thb = fma((double)kb[k], r.omega[k], thb);
        if (F64) {
          for (int s = 0; s < 4; ++s) {
            bool sv = true;
            for (int k = 0; k < D; ++k)
              sv = sv && (unsigned)(kb[k] + subo[s][k] + Sh::L[k] - 1 + Wi[k]) < (unsigned)(2 * Wi[k] + Sh::L[k]);
            if (!sv) continue;
            double y2 = 0.0, th = thb;
            for (int k = 0; k < D; ++k) {
              const double y = fma((double)kb[k] + offd[s][k], p.dx[k], -r.delta[k]);
              y2 = fma(y, y, y2);
              th = fma(offd[s][k], r.omega[k], th);
            }
            if (y2 <= p.R2) {
              const double g = exp(fma(y2, p.gauss, r.lnamp));
              double sn, cs;
              sincospi(2.0 * __builtin_amdgcn_fract(th), &sn, &cs);
              a64r[s] = fma(g, cs, a64r[s]);
              a64i[s] = fma(g, sn, a64i[s]);
            }
          }
        } else {
          float kbf[3];
          for (int k = 0; k < D; ++k) kbf[k] = (float)kb[k];
          for (int s = 0; s < 4; ++s) {
            bool sv = true;
            for (int k = 0; k < D; ++k)
              sv = sv && (unsigned)(kb[k] + subo[s][k] + Sh::L[k] - 1 + Wi[k]) < (unsigned)(2 * Wi[k] + Sh::L[k]);
            if (!sv) continue;
            float y2 = 0.0f;
            double th = thb;
            for (int k = 0; k < D; ++k) {
              const float y = fmaf(kbf[k] + offf[s][k], dxf[k], -r.deltaf[k]);
              y2 = fmaf(y, y, y2);
              th = fma(offd[s][k], r.omega[k], th);
            }
            float g = __builtin_amdgcn_exp2f(fmaf(y2, gl2, r.la2));
            g = (y2 <= R2f) ? g : 0.0f;
            const float rv = (float)__builtin_amdgcn_fract(th);
            a32r[s] = fmaf(g, __builtin_amdgcn_cosf(rv), a32r[s]);
            a32i[s] = fmaf(g, __builtin_amdgcn_sinf(rv), a32i[s]);
          }
          if (++pending == kFlush) {
            pending = 0;
            for (int s = 0; s < 4; ++s) {
              a64r[s] += (double)a32r[s];
              a64i[s] += (double)a32i[s];
              a32r[s] = 0.0f;
              a32i[s] = 0.0f;
            }
          }
        }
      }
      vbase += len;
    }
  }
  if (!F64) {
    for (int s = 0; s < 4; ++s) {
      a64r[s] += (double)a32r[s];
      a64i[s] += (double)a32i[s];
    }
  }
  // write this chunk's partial sums for the owned points inside the box
  int64_t npts = 1;
  for (int k = 0; k < D; ++k) npts *= p.box_n[k];
  double *out = p.partial + 2 * (int64_t)blockIdx.y * npts;
  for (int s = 0; s < 4; ++s) {
    bool inside = true;
    int64_t flat = 0;
    for (int k = 0; k < D; ++k) {
      const int64_t rel = worg[k] + (int64_t)offd[s][k] - p.box_lo[k];
      inside = inside && rel < p.box_n[k];
      flat = flat * p.box_n[k] + rel;
    }
    if (inside) {
      out[2 * flat] = a64r[s];
      out[2 * flat + 1] = a64i[s];
    }
  }
}

// ---------------------------------------------------------------------------
// Separable direct sum on the matrix cores (box window, d = 2, FP32).
//
// With the window |y_k| <= R taken per dimension, a packet's term at grid
// point (m_0, m_1) factors: it is A_j(m_0) B_j(m_1) with
//   A_j(m_0) = |scale a_j| e^{-y_0^2/(2 eps)} e^{2 pi i (phi0_j + k_0 omega_0j)} [|y_0| <= R],
//   B_j(m_1) = e^{-y_1^2/(2 eps)} e^{2 pi i k_1 omega_1j} [|y_1| <= R],
// k_d the minimum-image grid offset of m_d from the packet's nearest grid
// index and y_d = k_d dx_d - delta_d.  A 32 x 32 tile of u is then
// sum_j A_j B_j^T: a product of a 32 x J and a J x 32 complex matrix over the
// J packets that reach the tile.  One wave owns a tile.  The packets of the
// visible bins are tested 64 at a time (one per lane) and the visible ones
// are taken in pairs: lane l evaluates A of packet l/32 at row l%32 and B of
// packet l/32 at column l%32, which is the operand layout of
// v_mfma_f32_32x32x2_f32 (K = 2), and four MFMAs add the complex product.
// FP32 sums over 16 pairs are flushed into FP64 accumulators.
typedef float f32x16 __attribute__((ext_vector_type(16)));

constexpr int kSepTile = 32;
constexpr int kSepFlush = 16;  // packet pairs per FP32 partial sum

struct SepParams {
  const DsRec *rec;      // sorted by bin
  const int64_t *start;  // [nbins + 1]
  int64_t n[2], binw[2], nbin[2], ntile[2];
  int W[2];              // window half-width in grid steps, rounded up
  float dxf[2], Rf, gl2;  // gl2 = -log2(e) / (2 eps)
  int nchunk;
  int allvis;            // grid too small for the interval visibility test
  double *partial;       // [nchunk][n0 n1] complex FP64
};

__device__ __forceinline__ int min_image(int k, int n) {
  const int h = n >> 1;
  return k >= n - h ? k - n : (k < -h ? k + n : k);
}

__global__ __launch_bounds__(64) void ds_sep2_kernel(SepParams p) {
  const int lane = threadIdx.x;
  const int row = lane & 31;
  const int64_t torg0 = ((int64_t)blockIdx.x / p.ntile[1]) * kSepTile;
  const int64_t torg1 = ((int64_t)blockIdx.x % p.ntile[1]) * kSepTile;
  const int64_t torg[2] = {torg0, torg1};
  const int n0 = (int)p.n[0], n1 = (int)p.n[1];

  // bins visible from the tile: grid points [torg - W, torg + 31 + W] per
  // dimension, modulo n, as at most two bin intervals
  int64_t ia[2][2], ic[2][2], ilen[2][2], bcount[2];
  int nint[2];
  for (int k = 0; k < 2; ++k) {
    const int64_t lo = torg[k] - p.W[k], hi = torg[k] + kSepTile - 1 + p.W[k];
    const int64_t nk = p.n[k], nb = p.nbin[k], bw = p.binw[k];
    ia[k][1] = ic[k][1] = 0;
    if (hi - lo + 1 >= nk) {
      nint[k] = 1;
      ia[k][0] = 0;
      ic[k][0] = nb - 1;
    } else {
      const int64_t lm = imod(lo, nk), hm = imod(hi, nk);
      if (lm <= hm) {
        nint[k] = 1;
        ia[k][0] = lm / bw;
        ic[k][0] = hm / bw;
      } else if (hm / bw + 1 >= lm / bw) {
        nint[k] = 1;
        ia[k][0] = 0;
        ic[k][0] = nb - 1;
      } else {
        nint[k] = 2;
        ia[k][0] = lm / bw;
        ic[k][0] = nb - 1;
        ia[k][1] = 0;
        ic[k][1] = hm / bw;
      }
    }
    ilen[k][0] = ic[k][0] - ia[k][0] + 1;
    ilen[k][1] = nint[k] == 2 ? ic[k][1] - ia[k][1] + 1 : 0;
    bcount[k] = ilen[k][0] + ilen[k][1];
  }
  auto row_base = [&](int64_t r) {
    const int64_t b0 = r < ilen[0][0] ? ia[0][0] + r : ia[0][1] + (r - ilen[0][0]);
    return b0 * p.nbin[1];
  };
  int64_t total = 0;
  for (int64_t r = 0; r < bcount[0]; ++r) {
    const int64_t base = row_base(r);
    for (int run = 0; run < nint[1]; ++run)
      total += p.start[base + ic[1][run] + 1] - p.start[base + ia[1][run]];
  }
  const int64_t v0 = total * blockIdx.y / p.nchunk, v1 = total * (blockIdx.y + 1) / p.nchunk;

  f32x16 cr, ci;
  for (int r = 0; r < 16; ++r) cr[r] = ci[r] = 0.0f;
  double sr[16], si[16];
  for (int r = 0; r < 16; ++r) sr[r] = si[r] = 0.0;
  int pend = 0;
  const int m0 = (int)torg0 + row, m1 = (int)torg1 + row;  // this lane's row (A) and column (B)

  int64_t vbase = 0;
  for (int64_t rr = 0; rr < bcount[0] && vbase < v1; ++rr) {
    const int64_t base = row_base(rr);
    for (int run = 0; run < nint[1]; ++run) {
      const int64_t sa = p.start[base + ia[1][run]], sb = p.start[base + ic[1][run] + 1];
      const int64_t len = sb - sa;
      int64_t lo = v0 - vbase, hi = v1 - vbase;
      if (lo < 0) lo = 0;
      if (hi > len) hi = len;
      vbase += len;
      for (int64_t b = lo; b < hi; b += 64) {
        // one candidate record per lane, and whether its window reaches the tile
        const int64_t v = b + lane;
        int mq0 = 0, mq1 = 0;
        float la2 = 0.0f, d0 = 0.0f, d1 = 0.0f;
        double om0 = 0.0, om1 = 0.0, ph = 0.0;
        bool vis = false;
        if (v < hi) {
          const DsRec &r = p.rec[sa + v];
          mq0 = r.mq[0];
          mq1 = r.mq[1];
          la2 = r.la2;
          d0 = r.deltaf[0];
          d1 = r.deltaf[1];
          om0 = r.omega[0];
          om1 = r.omega[1];
          ph = r.phi0;
          const int kv0 = min_image((int)torg0 - mq0, n0), kv1 = min_image((int)torg1 - mq1, n1);
          vis = p.allvis || (kv0 + kSepTile - 1 >= -p.W[0] && kv0 <= p.W[0] && kv1 + kSepTile - 1 >= -p.W[1] &&
                             kv1 <= p.W[1]);
        }
        uint64_t mask = __ballot(vis);
        while (mask) {
          const int j0 = __builtin_ctzll(mask);
          mask &= mask - 1;
          int j1 = -1;
          if (mask) {
            j1 = __builtin_ctzll(mask);
            mask &= mask - 1;
          }
          const bool live = lane < 32 || j1 >= 0;
          const int src = lane < 32 || j1 < 0 ? j0 : j1;
          const int smq0 = __shfl(mq0, src), smq1 = __shfl(mq1, src);
          const float sla2 = __shfl(la2, src), sd0 = __shfl(d0, src), sd1 = __shfl(d1, src);
          const double som0 = __shfl(om0, src), som1 = __shfl(om1, src), sph = __shfl(ph, src);
          // A at row m0 (carries the amplitude and the packet's phase)
          const int k0 = min_image(m0 - smq0, n0);
          const float y0 = fmaf((float)k0, p.dxf[0], -sd0);
          float g0 = __builtin_amdgcn_exp2f(fmaf(y0 * y0, p.gl2, sla2));
          g0 = (live && fabsf(y0) <= p.Rf) ? g0 : 0.0f;
          const float r0 = (float)__builtin_amdgcn_fract(fma((double)k0, som0, sph));
          const float ar = g0 * __builtin_amdgcn_cosf(r0), ai = g0 * __builtin_amdgcn_sinf(r0);
          // B at column m1
          const int k1 = min_image(m1 - smq1, n1);
          const float y1 = fmaf((float)k1, p.dxf[1], -sd1);
          float g1 = __builtin_amdgcn_exp2f(y1 * y1 * p.gl2);
          g1 = (live && fabsf(y1) <= p.Rf) ? g1 : 0.0f;
          const float r1 = (float)__builtin_amdgcn_fract((double)k1 * som1);
          const float br = g1 * __builtin_amdgcn_cosf(r1), bi = g1 * __builtin_amdgcn_sinf(r1);
          cr = __builtin_amdgcn_mfma_f32_32x32x2f32(ar, br, cr, 0, 0, 0);
          cr = __builtin_amdgcn_mfma_f32_32x32x2f32(-ai, bi, cr, 0, 0, 0);
          ci = __builtin_amdgcn_mfma_f32_32x32x2f32(ar, bi, ci, 0, 0, 0);
          ci = __builtin_amdgcn_mfma_f32_32x32x2f32(ai, br, ci, 0, 0, 0);
          if (++pend == kSepFlush) {
            pend = 0;
            for (int r = 0; r < 16; ++r) {
              sr[r] += (double)cr[r];
              si[r] += (double)ci[r];
              cr[r] = ci[r] = 0.0f;
            }
          }
        }
      }
    }
  }
  for (int r = 0; r < 16; ++r) {
    sr[r] += (double)cr[r];
    si[r] += (double)ci[r];
  }
  // result layout of the 32x32 MFMA: lane l, register r holds row
  // 8 (r / 4) + 4 (l / 32) + r % 4 and column l % 32
  double *out = p.partial + 2 * (int64_t)blockIdx.y * p.n[0] * p.n[1];
  const int64_t col = torg1 + (lane & 31);
  for (int r = 0; r < 16; ++r) {
    const int64_t m = torg0 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
    if (m < p.n[0] && col < p.n[1]) {
      const int64_t flat = m * p.n[1] + col;
      out[2 * flat] = sr[r];
      out[2 * flat + 1] = si[r];
    }
  }
}

template <bool F64>
__global__ void ds_reduce_kernel(int64_t npts, int nchunk, const double *__restrict__ partial,
                                 void *__restrict__ u) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= npts) return;
  double re = 0.0, im = 0.0;
  for (int c = 0; c < nchunk; ++c) {
    re += partial[2 * (c * npts + i)];
    im += partial[2 * (c * npts + i) + 1];
  }
  if (F64) {
    reinterpret_cast<double2 *>(u)[i] = make_double2(re, im);
  } else {
    reinterpret_cast<float2 *>(u)[i] = make_float2((float)re, (float)im);
  }
}

// layout of one direct-sum call's workspace
struct DsLayout {
  int D;
  int64_t span[3], binw[3], nbin[3], ntile[3], W[3];
  int64_t nbins, ntiles, npts;
  int nchunk;
  size_t off_rec, off_keys, off_pos, off_start, off_part, off_sort, total;
};

DsLayout ds_layout(const DirectArgs &a) {
  DsLayout L{};
  const int D = a.g.d;
  L.D = D;
  static const int sp1[3] = {1024, 1, 1}, sp2[3] = {32, 32, 1}, sp3[3] = {16, 8, 8};
  const int *sp = D == 1 ? sp1 : (D == 2 ? sp2 : sp3);
  L.nbins = 1;
  L.ntiles = 1;
  L.npts = 1;
  for (int k = 0; k < 3; ++k) {
    L.span[k] = k < D ? sp[k] : 1;
    L.binw[k] = k < D ? std::max<int64_t>(1, L.span[k] / 2) : 1;
    L.nbin[k] = k < D ? (a.g.n[k] + L.binw[k] - 1) / L.binw[k] : 1;
    L.ntile[k] = k < D ? (a.box.n[k] + L.span[k] - 1) / L.span[k] : 1;
    L.W[k] = k < D ? (int64_t)std::floor(a.R / a.g.dx[k]) + 1 : 0;
    L.nbins *= L.nbin[k];
    L.ntiles *= L.ntile[k];
    L.npts *= k < D ? a.box.n[k] : 1;
  }
  // chunks: aim for >= 2048 workgroups, and >= ~512 candidate packets per chunk
  double cand = (double)a.pk->N;
  for (int k = 0; k < D; ++k)
    cand *= std::min(1.0, (double)(L.span[k] + 2 * L.W[k] + 2 * L.binw[k]) / (double)a.g.n[k]);
  // chunks: aim for ~8 waves per SIMD, >= ~256 candidate packets per chunk, and
  // a partial-sum buffer of at most ~32 MB.  The separable kernel runs one
  // wave per workgroup and wants ~16 per SIMD to overlap its matrix-core and
  // vector work: 16384 workgroups, a buffer of up to ~256 MB.
  const bool sep = a.box_window != 0;
  int nc = (int)std::ceil((sep ? 16384.0 : 8192.0) / (double)L.ntiles);
  nc = std::min(nc, (int)std::max(1.0, cand / (sep ? 128.0 : 256.0)));
  nc = std::min<int64_t>(nc, std::max<int64_t>(1, ((int64_t)(sep ? 256 : 32) << 20) / (L.npts * 16)));
  L.nchunk = std::max(1, std::min(nc, 512));
  const int64_t N = std::max<int64_t>(a.pk->N, 1);
  size_t o = 0;
  auto put = [&](size_t bytes) {
    size_t at = o;
    o = align_up(o + bytes, 256);
    return at;
  };
  L.off_rec = put(N * sizeof(DsRec));
  L.off_keys = put(N * 4);
  L.off_pos = put(N * 4);
  L.off_start = put((L.nbins + 1) * 8);
  L.off_part = put((size_t)L.nchunk * L.npts * 16);
  L.off_sort = put(bucket_positions_bytes(a.pk->N, L.nbins));
  L.total = o;
  return L;
}

}  // namespace

size_t direct_workspace_bytes(const DirectArgs &a) { return ds_layout(a).total; }

bool direct_graph_safe(const DirectArgs &a) {
  const DsLayout L = ds_layout(a);
  return bucket_positions_graph_safe(a.pk->N, L.nbins);
}

void launch_direct(const DirectArgs &a, Workspace &ws, hipStream_t s) {
  const DsLayout L = ds_layout(a);
  const bool f64 = a.precision == FGGC_FP64;
  char *base = (char *)ws.take(L.total);
  DsRec *rec = (DsRec *)(base + L.off_rec);
  uint32_t *keys = (uint32_t *)(base + L.off_keys), *pos = (uint32_t *)(base + L.off_pos);
  int64_t *start = (int64_t *)(base + L.off_start);
  double *part = (double *)(base + L.off_part);
  const int64_t N = a.pk->N;
  if (N > 0) {
    PrepParams pp{};
    pp.d = L.D;
    pp.N = N;
    pp.Q = a.pk->Q;
    pp.P = a.pk->P;
    pp.S = a.pk->S;
    pp.a = a.pk->a;
    pp.eps = a.eps;
    pp.scale = a.scale;
    for (int k = 0; k < 3; ++k) {
      pp.n[k] = k < L.D ? a.g.n[k] : 1;
      pp.dx[k] = k < L.D ? a.g.dx[k] : 1.0;
      pp.binw[k] = L.binw[k];
      pp.nbin[k] = L.nbin[k];
    }
    const dim3 g((unsigned)((N + 255) / 256)), b(256);
    {
      StageScope sc_sort(a.prof, "ds_sort", s);
      ds_key_kernel<<<g, b, 0, s>>>(pp, keys);
      FGGC_HIP(hipGetLastError());
      bucket_positions(keys, N, L.nbins, pos, start, base + L.off_sort, s);
    }
    StageScope sc(a.prof, "ds_prep", s);
    ds_prep_kernel<<<g, b, 0, s>>>(pp, pos, rec);
    FGGC_HIP(hipGetLastError());
  }
  if (N > 0 && a.box_window) {
    SepParams p{};
    p.rec = rec;
    p.start = start;
    for (int k = 0; k < 2; ++k) {
      p.n[k] = a.g.n[k];
      p.binw[k] = L.binw[k];
      p.nbin[k] = L.nbin[k];
      p.ntile[k] = L.ntile[k];
      p.W[k] = (int)L.W[k];
      p.dxf[k] = (float)a.g.dx[k];
      if (a.g.n[k] < 2 * (L.W[k] + kSepTile) + 2) p.allvis = 1;
    }
    p.Rf = (float)a.R;
    p.gl2 = (float)(-1.4426950408889634 / (2.0 * a.eps));
    p.nchunk = L.nchunk;
    p.partial = part;
    {
      StageScope sc(a.prof, "ds_kernel", s);
      ds_sep2_kernel<<<dim3((unsigned)L.ntiles, (unsigned)L.nchunk), dim3(64), 0, s>>>(p);
      FGGC_HIP(hipGetLastError());
    }
    StageScope sr(a.prof, "ds_reduce", s);
    ds_reduce_kernel<false><<<dim3((unsigned)((L.npts + 255) / 256)), dim3(256), 0, s>>>(L.npts, L.nchunk,
                                                                                        part, a.u);
    FGGC_HIP(hipGetLastError());
  } else if (N > 0) {
    DsParams p{};
    p.rec = rec;
    p.start = start;
    for (int k = 0; k < 3; ++k) {
      p.n[k] = k < L.D ? a.g.n[k] : 1;
      p.binw[k] = L.binw[k];
      p.nbin[k] = L.nbin[k];
      p.box_lo[k] = k < L.D ? a.box.lo[k] : 0;
      p.box_n[k] = k < L.D ? a.box.n[k] : 1;
      p.ntile[k] = L.ntile[k];
      p.W[k] = L.W[k];
      p.dx[k] = k < L.D ? a.g.dx[k] : 1.0;
    }
    p.R2 = a.R * a.R;
    p.gauss = -1.0 / (2.0 * a.eps);
    p.nchunk = L.nchunk;
    p.partial = part;
    p.lanewrap = 0;
    for (int k = 0; k < L.D; ++k)
      if (a.g.n[k] < 2 * (L.W[k] + L.span[k]) + 2) p.lanewrap = 1;
    dim3 grid((unsigned)L.ntiles, (unsigned)L.nchunk);
    {
    StageScope sc(a.prof, "ds_kernel", s);
#define FGGC_DS(DD)                                                                    \
  if (f64 && p.lanewrap) ds_kernel<DD, true, true><<<grid, dim3(kBlock), 0, s>>>(p);  \
  else if (f64) ds_kernel<DD, true, false><<<grid, dim3(kBlock), 0, s>>>(p);         \
  else if (p.lanewrap) ds_kernel<DD, false, true><<<grid, dim3(kBlock), 0, s>>>(p);  \
  else ds_kernel<DD, false, false><<<grid, dim3(kBlock), 0, s>>>(p);
    if (L.D == 1) { FGGC_DS(1) }
    else if (L.D == 2) { FGGC_DS(2) }
    else { FGGC_DS(3) }
#undef FGGC_DS
    FGGC_HIP(hipGetLastError());
    }
    StageScope sr(a.prof, "ds_reduce", s);
    if (f64) ds_reduce_kernel<true><<<dim3((unsigned)((L.npts + 255) / 256)), dim3(256), 0, s>>>(
        L.npts, L.nchunk, part, a.u);
    else ds_reduce_kernel<false><<<dim3((unsigned)((L.npts + 255) / 256)), dim3(256), 0, s>>>(
        L.npts, L.nchunk, part, a.u);
    FGGC_HIP(hipGetLastError());
  } else {
    launch_zero(a.u, (size_t)L.npts * (f64 ? 16 : 8), s);
  }
}

}  // namespace fggc
