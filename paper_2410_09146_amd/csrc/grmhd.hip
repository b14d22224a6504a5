// libgrmhd.so: host side of the C ABI declared in include/grmhd.h, plus the
// gfx950 kernels (kernels.h).  The host builds, once per pack, everything the
// kernels need as flat device tables: block descriptors, 1-D coordinate
// tables, ghost-zone gather maps and tile / chunk work lists, all placed in
// the caller's workspace.  Each public call then only enqueues kernels on
// the pack's stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <type_traits>
#include <utility>
#include <unordered_map>
#include <vector>

#include "../../include/grmhd.h"
#include "kernels.h"
#include "m1.h"
#include "amr.h"

using namespace grmhd;

namespace {

thread_local std::string g_err;

constexpr size_t ALIGN = 256;
// reduction result block in the workspace: 16 doubles written by the fold
// (dt first); slot RES_NFAIL holds the device counter of failed inversions
// (every con2prim adds its failures; zeroed once, at pack creation)
constexpr int RES_SLOTS = 32;
constexpr int RES_NFAIL = 24;
constexpr size_t align_up(size_t x) { return (x + ALIGN - 1) / ALIGN * ALIGN; }

// Everything derived from a descriptor on the host.
struct Plan {
  int nb = 0, ng = 4;
  long long nct = 0;
  std::vector<long long> off;
  std::vector<BlockInfo> blocks;
  std::vector<double> rc, rf, sc, cc, sf, cf;
  std::vector<int4> tiles[3][NSHAPE];
  // fused stage: tiles along D at stride TD - 1 over the faces ng .. ng + n
  // (the block's upper face included), for single-level packs
  std::vector<int4> tilesF[3][NSHAPE];
  // persistent streaming tiles (k_flux_pf): as tiles, but for D = x2, x3 the
  // columns start at an even x1 (ng - 2) so that cell pairs are 16-byte aligned
  std::vector<int4> tilesP[3][NSHAPE];
  std::vector<int2> planes;       // (3 block + D, first face), 64 faces each
  std::vector<int2> ch_int, ch_ext, ch_bcc;
  std::vector<GhostP> gP;
  std::vector<GhostB> gB;
  std::vector<GhostR> gR;          // two-level meshes: restriction + staging
  std::vector<GhostPro> gPro;      // prolongation of P into fine ghosts
  std::vector<GhostBR> gBR;
  std::vector<GhostBPro> gBPro;
  long long nsP = 0, nsB = 0;      // staged coarse-view cells / faces
  std::vector<FixF> fixF;          // level-boundary corrections (two-level meshes)
  std::vector<FixE> fixE;
  int maxlev = 0;
  // host copies of the layout (regrid / remap)
  std::vector<int> lev, lloc;     // per block; lloc in cells of the block's level
  int root_nx[3] = {0, 0, 0};
  int bc[6] = {0, 0, 0, 0, 0, 0};
  int active[3] = {1, 1, 1};
  double dxmin = 0.0;
  // workspace carve-up (byte offsets)
  size_t o_F, o_Bcc, o_flags, o_iters, o_blocks, o_tab, o_planes, o_chi, o_che,
      o_flr, o_chb, o_gP, o_gB, o_gR, o_gPro, o_gBR, o_gBPro, o_SP, o_SB, o_E, o_fixF, o_fixE, o_part, o_res,
      o_mlpw, o_mlpf, total;
  size_t o_tl[3][NSHAPE], o_tlF[3][NSHAPE], o_tlP[3][NSHAPE];
};

int fail(const std::string &m, int code)
{
  g_err = m;
  return code;
}

int validate(const grmhd_pack_desc *d)
{
  if (!d) return fail("null descriptor", GRMHD_E_INVALID);
  if (d->nblocks < 1 || d->nblocks > (1 << 20)) return fail("nblocks out of range", GRMHD_E_INVALID);
  if (d->ng != 4) return fail("ng must be 4", GRMHD_E_UNSUPPORTED);
  if (d->recon < 0 || d->recon > 4) return fail("bad recon", GRMHD_E_INVALID);
  if (d->riemann < 0 || d->riemann > 1) return fail("bad riemann", GRMHD_E_INVALID);
  if (d->precision != GRMHD_PREC_FP64 && d->precision != GRMHD_PREC_MIXED)
    return fail("bad precision", GRMHD_E_INVALID);
  if (d->nscalar < 0 || d->nscalar > 1) return fail("nscalar must be 0 or 1", GRMHD_E_INVALID);
  if (d->nscalar && d->precision != GRMHD_PREC_FP64)
    return fail("the passive scalar needs FP64 precision", GRMHD_E_UNSUPPORTED);
  if (!d->nx || !d->lloc) return fail("null nx/lloc", GRMHD_E_INVALID);
  for (int s = 0; s < 6; ++s)
    if (d->bc[s] < 0 || d->bc[s] > 3) return fail("bad boundary kind", GRMHD_E_INVALID);
  for (int dd = 0; dd < 3; ++dd) {
    if (d->root_nx[dd] < 1) return fail("root_nx < 1", GRMHD_E_SHAPE);
    if (!(d->xmax[dd] > d->xmin[dd])) return fail("xmax <= xmin", GRMHD_E_SHAPE);
    if ((d->bc[2 * dd] == GRMHD_BC_PERIODIC) != (d->bc[2 * dd + 1] == GRMHD_BC_PERIODIC))
      return fail("periodic must pair", GRMHD_E_INVALID);
  }
  if ((d->bc[0] == GRMHD_BC_POLAR) || (d->bc[1] == GRMHD_BC_POLAR) ||
      (d->bc[4] == GRMHD_BC_POLAR) || (d->bc[5] == GRMHD_BC_POLAR))
    return fail("polar boundaries only along x2", GRMHD_E_UNSUPPORTED);
  int maxlev = 0;
  for (int b = 0; b < d->nblocks; ++b) {
    const int lev = d->level ? d->level[b] : 0;
    if (lev < 0 || lev > 1) return fail("levels 0 and 1 only", GRMHD_E_UNSUPPORTED);
    maxlev = std::max(maxlev, lev);
    for (int dd = 0; dd < 3; ++dd) {
      const int n = d->nx[3 * b + dd], l = d->lloc[3 * b + dd], N = d->root_nx[dd] << lev;
      if (n < 1 || n > 4096) return fail("block size out of range", GRMHD_E_SHAPE);
      if (l < 0 || l + n > N) return fail("block outside the domain", GRMHD_E_SHAPE);
      if (n < d->ng && N != n) return fail("split blocks need n >= ng", GRMHD_E_SHAPE);
      if (lev == 1 && ((n | l) & 1)) return fail("level-1 blocks need even size and offset", GRMHD_E_SHAPE);
    }
  }
  if (maxlev > 0 && d->nscalar)
    return fail("two-level meshes carry no passive scalar", GRMHD_E_UNSUPPORTED);
  if (maxlev > 0)
    for (int dd = 0; dd < 3; ++dd)
      if (d->root_nx[dd] < 2 * d->ng) return fail("two-level meshes need root_nx >= 2 ng", GRMHD_E_SHAPE);
  // blocks must tile the domain exactly once (volume in level-1 cells)
  long long vol = 0;
  for (int b = 0; b < d->nblocks; ++b) {
    const int lev = d->level ? d->level[b] : 0;
    vol += ((long long)d->nx[3 * b] * d->nx[3 * b + 1] * d->nx[3 * b + 2]) << (3 * (1 - lev));
  }
  if (vol != 8LL * d->root_nx[0] * d->root_nx[1] * d->root_nx[2])
    return fail("blocks do not cover the domain", GRMHD_E_SHAPE);
  return GRMHD_OK;
}

void layout(const grmhd_pack_desc *d, std::vector<long long> &off, long long &nct)
{
  off.resize(d->nblocks);
  long long o = 0;
  for (int b = 0; b < d->nblocks; ++b) {
    off[b] = o;
    long long c = 1;
    for (int dd = 0; dd < 3; ++dd) c *= d->nx[3 * b + dd] + 2 * d->ng;
    o += (c + 31) / 32 * 32;
  }
  nct = o;
}

// owner lookup over level-0 cells at a granularity of g cells; a level-l
// cell is looked up through its level-0 ancestor
struct Owner {
  int g[3], dims[3];
  std::vector<int> id;
  int at(int l, const int c[3]) const
  {
    const int x = (c[0] >> l) / g[0], y = (c[1] >> l) / g[1], z = (c[2] >> l) / g[2];
    return id[x + (size_t)dims[0] * (y + (size_t)dims[1] * z)];
  }
};

int gcd(int a, int b) { return b ? gcd(b, a % b) : a; }

int build_plan(const grmhd_pack_desc *d, Plan &p)
{
  int rc = validate(d);
  if (rc) return rc;
  p.nb = d->nblocks;
  p.ng = d->ng;
  const int ng = d->ng;
  layout(d, p.off, p.nct);
  auto lev_of = [&](int b) { return d->level ? d->level[b] : 0; };
  for (int b = 0; b < p.nb; ++b) p.maxlev = std::max(p.maxlev, lev_of(b));
  double dx[3];
  for (int dd = 0; dd < 3; ++dd) dx[dd] = (d->xmax[dd] - d->xmin[dd]) / d->root_nx[dd];
  p.dxmin = 1e300;
  for (int dd = 0; dd < 3; ++dd) {
    p.active[dd] = d->root_nx[dd] > 1;
    if (p.active[dd]) p.dxmin = std::min(p.dxmin, dx[dd] / (1 << p.maxlev));
  }
  if (p.dxmin == 1e300) p.dxmin = dx[0] / (1 << p.maxlev);

  // owner grid (level-0 cells; level-1 blocks are aligned to them)
  Owner own;
  for (int dd = 0; dd < 3; ++dd) {
    int g = d->root_nx[dd];
    for (int b = 0; b < p.nb; ++b)
      g = gcd(g, gcd(d->nx[3 * b + dd] >> lev_of(b), d->lloc[3 * b + dd] >> lev_of(b)));
    own.g[dd] = g;
    own.dims[dd] = d->root_nx[dd] / g;
  }
  own.id.assign((size_t)own.dims[0] * own.dims[1] * own.dims[2], -1);
  for (int b = 0; b < p.nb; ++b) {
    int lo[3], hi[3];
    for (int dd = 0; dd < 3; ++dd) {
      lo[dd] = (d->lloc[3 * b + dd] >> lev_of(b)) / own.g[dd];
      hi[dd] = ((d->lloc[3 * b + dd] + d->nx[3 * b + dd]) >> lev_of(b)) / own.g[dd];
    }
    for (int z = lo[2]; z < hi[2]; ++z)
      for (int y = lo[1]; y < hi[1]; ++y)
        for (int x = lo[0]; x < hi[0]; ++x) {
          int &o = own.id[x + (size_t)own.dims[0] * (y + (size_t)own.dims[1] * z)];
          if (o >= 0) return fail("blocks overlap", GRMHD_E_SHAPE);
          o = b;
        }
  }

  p.lev.resize(p.nb);
  p.lloc.resize(3 * (size_t)p.nb);
  for (int b = 0; b < p.nb; ++b) {
    p.lev[b] = lev_of(b);
    for (int dd = 0; dd < 3; ++dd) p.lloc[3 * b + dd] = d->lloc[3 * b + dd];
  }
  for (int dd = 0; dd < 3; ++dd) p.root_nx[dd] = d->root_nx[dd];
  for (int q = 0; q < 6; ++q) p.bc[q] = d->bc[q];

  // blocks and coordinate tables
  p.blocks.resize(p.nb);
  const bool plo = d->bc[2] == GRMHD_BC_POLAR, phi = d->bc[3] == GRMHD_BC_POLAR;
  for (int b = 0; b < p.nb; ++b) {
    BlockInfo &bi = p.blocks[b];
    std::memset(&bi, 0, sizeof bi);
    const int lev = lev_of(b);
    double dxl[3];
    for (int dd = 0; dd < 3; ++dd) {
      dxl[dd] = dx[dd] / (1 << lev);
      bi.n[dd] = d->nx[3 * b + dd];
      bi.s[dd] = bi.n[dd] + 2 * ng;
      bi.dx[dd] = dxl[dd];
    }
    const int N2 = d->root_nx[1] << lev;
    bi.off = p.off[b];
    bi.tab1 = (int)p.rc.size();
    bi.tab2 = (int)p.sc.size();
    for (int i = 0; i < bi.s[0]; ++i) {
      const int g = d->lloc[3 * b] + i - ng;
      p.rc.push_back(std::exp(d->xmin[0] + ((double)g + 0.5) * dxl[0]));
      p.rf.push_back(std::exp(d->xmin[0] + ((double)g) * dxl[0]));
    }
    bi.pole_lo = bi.pole_hi = -1;
    for (int j = 0; j < bi.s[1]; ++j) {
      int g = d->lloc[3 * b + 1] + j - ng;
      if (plo && g < 0) g = -1 - g;
      if (phi && g >= N2) g = 2 * N2 - 1 - g;
      const double th = d->xmin[1] + ((double)g + 0.5) * dxl[1];
      p.sc.push_back(std::sin(th));
      p.cc.push_back(std::cos(th));
      int gf = d->lloc[3 * b + 1] + j - ng;
      if (plo && gf < 0) gf = -gf;
      if (phi && gf > N2) gf = 2 * N2 - gf;
      const double tf = d->xmin[1] + ((double)gf) * dxl[1];
      const bool pole = (plo && gf == 0) || (phi && gf == N2);
      p.sf.push_back(pole ? 0.0 : std::sin(tf));
      p.cf.push_back(std::cos(tf));
      if (plo && d->lloc[3 * b + 1] + j - ng == 0) bi.pole_lo = j;
      if (phi && d->lloc[3 * b + 1] + j - ng == N2) bi.pole_hi = j;
    }
  }

  // work lists
  for (int b = 0; b < p.nb; ++b) {
    const BlockInfo &bi = p.blocks[b];
    for (int D = 0; D < 3; ++D) {
      const int AX = D == 0 ? 1 : 0, BX = D == 2 ? 1 : 2;
      for (int sh = 0; sh < NSHAPE; ++sh) {
        const int td = shape_td(sh), ta = shape_ta(sh);
        for (int kb = ng - 1; kb <= ng + bi.n[BX]; ++kb)
          for (int a0 = ng - 1; a0 <= ng + bi.n[AX]; a0 += ta)
            for (int f0 = ng; f0 < ng + bi.n[D]; f0 += td) {
              int o[3];
              o[D] = f0; o[AX] = a0; o[BX] = kb;
              p.tiles[D][sh].push_back(make_int4(b, o[0], o[1], o[2]));
            }
        {
          const int a_lo = AX == 0 ? ng - 2 : ng - 1;
          for (int kb = ng - 1; kb <= ng + bi.n[BX]; ++kb)
            for (int a0 = a_lo; a0 <= ng + bi.n[AX]; a0 += ta)
              for (int f0 = ng; f0 < ng + bi.n[D]; f0 += td) {
                int o[3];
                o[D] = f0; o[AX] = a0; o[BX] = kb;
                p.tilesP[D][sh].push_back(make_int4(b, o[0], o[1], o[2]));
              }
        }
        if (p.maxlev == 0 && !d->nscalar)
          for (int kb = ng - 1; kb <= ng + bi.n[BX]; ++kb)
            for (int a0 = ng - 1; a0 <= ng + bi.n[AX]; a0 += ta)
              for (int f0 = ng; f0 < ng + bi.n[D]; f0 += td - 1) {
                int o[3];
                o[D] = f0; o[AX] = a0; o[BX] = kb;
                p.tilesF[D][sh].push_back(make_int4(b, o[0], o[1], o[2]));
              }
      }
    }
  }
  // XCD-aware order of the flux tile lists: workgroups are dealt round-robin
  // over the 8 XCDs (workgroup w to XCD w % 8), so the natural, spatially
  // ordered list is cut into 8 contiguous runs (the first n % 8 one entry
  // longer) and workgroup w takes entry w / 8 of run w % 8.  Each XCD then
  // sweeps one contiguous eighth of the tiles and reuses the stencil halos in
  // its own L2.  (The cell-chunk lists keep the natural order: the same
  // permutation of them measured slower for the update and the cell-centred
  // field.)
  auto xcd_order = [](auto &L) {
    const size_t n = L.size(), base = n / 8, rem = n % 8;
    std::remove_reference_t<decltype(L)> out(n);
    for (size_t w = 0; w < n; ++w) {
      const size_t x = w % 8;
      out[w] = L[x * base + std::min(x, rem) + w / 8];
    }
    L.swap(out);
  };
  for (int D = 0; D < 3; ++D)
    for (int sh = 0; sh < NSHAPE; ++sh) {
      xcd_order(p.tiles[D][sh]);
      xcd_order(p.tilesF[D][sh]);
      xcd_order(p.tilesP[D][sh]);
    }
  for (int b = 0; b < p.nb; ++b) {
    const BlockInfo &bi = p.blocks[b];
    for (int D = 0; D < 3; ++D) {
      const int AX = D == 0 ? 1 : 0, BX = D == 2 ? 1 : 2;
      const int np = (bi.n[AX] + 2) * (bi.n[BX] + 2);
      for (int s = 0; s < np; s += 64) p.planes.push_back(make_int2(3 * b + D, s));
    }
    const long long ni = (long long)bi.n[0] * bi.n[1] * bi.n[2];
    for (long long s = 0; s < ni; s += 256) p.ch_int.push_back(make_int2(b, (int)s));
    const long long ne = (long long)(bi.n[0] + 1) * (bi.n[1] + 1) * (bi.n[2] + 1);
    for (long long s = 0; s < ne; s += 256) p.ch_ext.push_back(make_int2(b, (int)s));
    const long long nbc = (long long)(bi.s[0] - 1) * (bi.s[1] - 1) * (bi.s[2] - 1);
    for (long long s = 0; s < nbc; s += 256) p.ch_bcc.push_back(make_int2(b, (int)s));
  }


  // ghost maps.  Per axis at level l: global index -> (source global index,
  // flags); returns 0 interior, 1 mapped, -1 fixed (leave).
  auto map_axis = [&](int l, int dd, int g, bool normal, int &src, int &flip, int &ofl) -> int {
    const int N = d->root_nx[dd] << l;
    const int hiN = normal ? N : N - 1;
    flip = 0; ofl = 0;
    if (g >= 0 && g <= hiN) { src = g; return 0; }
    const bool low = g < 0;
    const int bc = d->bc[2 * dd + (low ? 0 : 1)];
    switch (bc) {
      case GRMHD_BC_PERIODIC: src = ((g % N) + N) % N; return 1;   // face N is face 0
      case GRMHD_BC_OUTFLOW: src = low ? 0 : hiN; ofl = low ? 1 : 2; return 1;
      case GRMHD_BC_POLAR:
        src = normal ? (low ? -g : 2 * N - g) : (low ? -1 - g : 2 * N - 1 - g);
        flip = 1;
        return 1;
      default: return -1;
    }
  };
  // linear index of level-l global index X inside block ob (same level)
  auto lin_in = [&](int ob, const int X[3]) -> long long {
    const BlockInfo &sb = p.blocks[ob];
    long long lin = 0, mul = 1;
    for (int dd = 0; dd < 3; ++dd) {
      lin += mul * (X[dd] - d->lloc[3 * ob + dd] + ng);
      mul *= sb.s[dd];
    }
    return sb.off + lin;
  };
  // owner of a level-l face (the cell above it, or below at the upper edge)
  // owner of a level-l face: the cell above it (below at the upper domain
  // edge); where the two cells beside the face lie on different levels, the
  // finer one, whose frame may then name the face N instead of 0 (or 0
  // instead of N) across a periodic boundary
  auto face_owner = [&](int l, int comp, int F[3]) -> int {
    const int N = d->root_nx[comp] << l;
    int C[3] = {F[0], F[1], F[2]};
    C[comp] = std::min(C[comp], N - 1);
    int ob = own.at(l, C);
    int A[3] = {F[0], F[1], F[2]}, alt = -1;
    const bool per = d->bc[2 * comp] == GRMHD_BC_PERIODIC;
    if (F[comp] > 0 && F[comp] < N) { A[comp] = F[comp] - 1; alt = F[comp]; }
    else if (F[comp] == N && per) { A[comp] = 0; alt = 0; }
    else if (F[comp] == 0 && per) { A[comp] = N - 1; alt = N; }
    if (alt >= 0) {
      const int oa = own.at(l, A);
      if (lev_of(oa) > lev_of(ob)) { ob = oa; F[comp] = alt; }
    }
    return ob;
  };
  // staged level-0 views: cells keyed by (mapped index, flags), faces by
  // (component, index)
  std::unordered_map<long long, int> stP, stB;
  auto key3 = [&](int l, const int X[3]) -> long long {
    const long long N0 = (long long)(d->root_nx[0] << l) + 1, N1 = (long long)(d->root_nx[1] << l) + 1;
    return X[0] + N0 * (X[1] + N1 * (long long)X[2]);
  };
  // coarse-view staging row of level-0 cell C (any index); -1 beyond a fixed
  // boundary
  auto stage_cell = [&](const int Cin[3]) -> int {
    int C[3], flags = 0;
    for (int dd = 0; dd < 3; ++dd) {
      int fl, ofl;
      if (map_axis(0, dd, Cin[dd], false, C[dd], fl, ofl) < 0) return -1;
      if (fl) flags |= 1 << dd;
      if (ofl & 1) flags |= 8 << (2 * dd);
      if (ofl & 2) flags |= 16 << (2 * dd);
    }
    const long long key = key3(0, C) * 512 + flags;
    auto it = stP.find(key);
    if (it != stP.end()) return it->second;
    const int idx = (int)p.nsP++;
    stP.emplace(key, idx);
    const int ob = own.at(0, C);
    GhostR r{};
    r.dst = idx; r.flags = flags; r.tgt = 1;
    if (lev_of(ob) == 0) {
      r.src = lin_in(ob, C); r.n = 1;
    } else {
      const int X[3] = {2 * C[0], 2 * C[1], 2 * C[2]};
      r.src = lin_in(ob, X); r.n = 8;
      r.sj = p.blocks[ob].s[0]; r.sk = (long long)p.blocks[ob].s[0] * p.blocks[ob].s[1];
    }
    p.gR.push_back(r);
    return idx;
  };
  // mean of the 4 level-1 child faces of level-0 face Q, as a GhostBR
  auto child_faces = [&](int ob, int comp, const int Q[3], GhostBR &r) {
    const int t1 = (comp + 1) % 3, t2 = (comp + 2) % 3;
    const int X[3] = {2 * Q[0], 2 * Q[1], 2 * Q[2]};
    const long long str[3] = {1, p.blocks[ob].s[0], (long long)p.blocks[ob].s[0] * p.blocks[ob].s[1]};
    r.src = lin_in(ob, X); r.n = 4; r.st1 = str[t1]; r.st2 = str[t2];
  };
  // staging row of level-0 face Q (inside the domain)
  auto stage_face = [&](int comp, const int Qin[3]) -> int {
    const long long key = key3(0, Qin) * 3 + comp;
    auto it = stB.find(key);
    if (it != stB.end()) return it->second;
    const int idx = (int)p.nsB++;
    stB.emplace(key, idx);
    int Q[3] = {Qin[0], Qin[1], Qin[2]};
    const int ob = face_owner(0, comp, Q);
    GhostBR r{};
    r.dst = idx; r.comp = comp; r.flip = 0; r.tgt = 1;
    if (lev_of(ob) == 0) { r.src = lin_in(ob, Q); r.n = 1; }
    else child_faces(ob, comp, Q, r);
    p.gBR.push_back(r);
    return idx;
  };
  for (int b = 0; b < p.nb; ++b) {
    const BlockInfo &bi = p.blocks[b];
    const int *ll = &d->lloc[3 * b];
    const int l = lev_of(b);
    for (int comp = -1; comp < 3; ++comp) {   // -1: cell-centred P
      for (int k = 0; k < bi.s[2]; ++k)
        for (int j = 0; j < bi.s[1]; ++j)
          for (int i = 0; i < bi.s[0]; ++i) {
            const int idx[3] = {i, j, k};
            bool ghost = false;
            for (int dd = 0; dd < 3; ++dd) {
              const int hi = (comp == dd) ? ng + bi.n[dd] : ng + bi.n[dd] - 1;
              if (idx[dd] < ng || idx[dd] > hi) ghost = true;
            }
            if (!ghost) continue;
            int src[3], flags = 0, flipn = 0;
            bool fixed = false;
            for (int dd = 0; dd < 3; ++dd) {
              int fl, ofl;
              const int g = ll[dd] + idx[dd] - ng;
              const int r = map_axis(l, dd, g, comp == dd, src[dd], fl, ofl);
              if (r < 0) fixed = true;
              if (fl) { flags |= 1 << dd; if (comp == dd) flipn = 1; }
              if (ofl & 1) flags |= 8 << (2 * dd);
              if (ofl & 2) flags |= 16 << (2 * dd);
            }
            if (fixed) continue;
            const long long dst = bi.off + i + (long long)bi.s[0] * (j + (long long)bi.s[1] * k);
            const int ob = comp < 0 ? own.at(l, src) : face_owner(l, comp, src);
            if (ob < 0) return fail("ghost source not covered", GRMHD_E_SHAPE);
            const int lo = lev_of(ob);
            if (lo == l) {
              if (comp < 0) p.gP.push_back(GhostP{dst, lin_in(ob, src), flags, 0});
              else p.gB.push_back(GhostB{dst, lin_in(ob, src), comp, flipn});
            } else if (comp < 0 && lo < l) {          // prolongation from level 0
              GhostPro g{};
              g.dst = dst; g.flags = flags;
              const int C[3] = {src[0] >> 1, src[1] >> 1, src[2] >> 1};
              g.s[0] = stage_cell(C);
              if (g.s[0] < 0) return fail("internal: parent beyond a fixed boundary", GRMHD_E_SHAPE);
              for (int dd = 0; dd < 3; ++dd) {
                int Q[3] = {C[0], C[1], C[2]};
                Q[dd] = C[dd] - 1;
                const int sm = stage_cell(Q);
                Q[dd] = C[dd] + 1;
                const int sp = stage_cell(Q);
                g.s[1 + 2 * dd] = sm < 0 ? g.s[0] : sm;
                g.s[2 + 2 * dd] = sp < 0 ? g.s[0] : sp;
                g.oct |= (src[dd] & 1) << dd;
              }
              p.gPro.push_back(g);
            } else if (comp < 0) {                     // restriction from level 1
              GhostR r{};
              const int X[3] = {2 * src[0], 2 * src[1], 2 * src[2]};
              r.dst = dst; r.src = lin_in(ob, X); r.n = 8; r.flags = flags; r.tgt = 0;
              r.sj = p.blocks[ob].s[0]; r.sk = (long long)p.blocks[ob].s[0] * p.blocks[ob].s[1];
              p.gR.push_back(r);
            } else if (lo < l) {                       // face prolongation
              GhostBPro g{};
              g.dst = dst; g.comp = comp; g.flip = flipn;
              int Q[3] = {src[0] >> 1, src[1] >> 1, src[2] >> 1};
              if ((src[comp] & 1) == 0) {
                Q[comp] = src[comp] / 2;
                g.sa = stage_face(comp, Q); g.sb = -1;
              } else {
                Q[comp] = (src[comp] - 1) / 2;
                g.sa = stage_face(comp, Q);
                Q[comp] = (src[comp] + 1) / 2;
                g.sb = stage_face(comp, Q);
              }
              p.gBPro.push_back(g);
            } else {                                   // face restriction
              GhostBR r{};
              r.dst = dst; r.comp = comp; r.flip = flipn; r.tgt = 0;
              child_faces(ob, comp, src, r);
              p.gBR.push_back(r);
            }
          }
    }
  }

  // level-boundary corrections of every level-0 block (the fine fluxes and
  // EMFs are authoritative): faces whose other side is a level-1 block, and
  // own edges that coincide with two edges of a level-1 block (the first such
  // block in block order)
  if (p.maxlev > 0) {
    auto wrap0 = [&](int dd, int g, int &out) -> bool {
      const int N = d->root_nx[dd];
      if (g >= 0 && g < N) { out = g; return true; }
      if (d->bc[2 * dd] != GRMHD_BC_PERIODIC) return false;
      out = ((g % N) + N) % N;
      return true;
    };
    auto str_of = [&](int b, int dd) -> long long {
      return dd == 0 ? 1 : dd == 1 ? (long long)p.blocks[b].s[0]
                                   : (long long)p.blocks[b].s[0] * p.blocks[b].s[1];
    };
    // does fine block f own the fine edge along e at cell fe, faces (fa, fb)?
    // (periodic faces N and 0 are the same face)
    auto owns_edge = [&](int f, int e, const int want[3], int X[3]) -> bool {
      const int ax[3] = {e, (e + 1) % 3, (e + 2) % 3};
      int cand[3][2], nc[3];
      for (int q = 0; q < 3; ++q) {
        const int dd = ax[q], N = d->root_nx[dd] << 1;
        nc[q] = 1;
        cand[q][0] = want[q];
        if (q > 0 && d->bc[2 * dd] == GRMHD_BC_PERIODIC) {
          if (want[q] == 0) cand[q][nc[q]++] = N;
          else if (want[q] == N) cand[q][nc[q]++] = 0;
        }
      }
      for (int x = 0; x < nc[0]; ++x)
        for (int y = 0; y < nc[1]; ++y)
          for (int z = 0; z < nc[2]; ++z) {
            const int v[3] = {cand[0][x], cand[1][y], cand[2][z]};
            bool ok = true;
            for (int q = 0; q < 3; ++q) {
              const int dd = ax[q], lo = d->lloc[3 * f + dd];
              const int hi = lo + d->nx[3 * f + dd] - (q == 0 ? 1 : 0);
              if (v[q] < lo || v[q] > hi) ok = false;
              X[dd] = v[q];
            }
            if (ok) return true;
          }
      return false;
    };
    for (int c = 0; c < p.nb; ++c) {
      if (lev_of(c) != 0) continue;
      const int *llc = &d->lloc[3 * c], *nxc = &d->nx[3 * c];
      for (int D = 0; D < 3; ++D) {
        const int t1 = (D + 1) % 3, t2 = (D + 2) % 3;
        for (int side = 0; side < 2; ++side) {
          int oc;
          if (!wrap0(D, side ? llc[D] + nxc[D] : llc[D] - 1, oc)) continue;
          for (int u2 = 0; u2 < nxc[t2]; ++u2)
            for (int u1 = 0; u1 < nxc[t1]; ++u1) {
              int C0[3];
              C0[D] = oc; C0[t1] = llc[t1] + u1; C0[t2] = llc[t2] + u2;
              const int f = own.at(0, C0);
              if (lev_of(f) != 1) continue;
              int X[3], G[3];
              X[D] = side ? 2 * oc : 2 * (oc + 1);
              X[t1] = 2 * C0[t1]; X[t2] = 2 * C0[t2];
              G[D] = llc[D] + (side ? nxc[D] : 0); G[t1] = C0[t1]; G[t2] = C0[t2];
              p.fixF.push_back(FixF{lin_in(c, G), lin_in(f, X), str_of(f, t1), str_of(f, t2), D, 0});
            }
        }
      }
      for (int e = 0; e < 3; ++e) {
        const int a = (e + 1) % 3, bx = (e + 2) % 3;
        for (int kb = 0; kb <= nxc[bx]; ++kb)
          for (int ka = 0; ka <= nxc[a]; ++ka) {
            if (!(ka == 0 || ka == nxc[a] || kb == 0 || kb == nxc[bx])) continue;
            for (int ie = 0; ie < nxc[e]; ++ie) {
              const int want[3] = {2 * (llc[e] + ie), 2 * (llc[a] + ka), 2 * (llc[bx] + kb)};
              // candidate fine blocks: owners of the fine cells beside the edge
              int best = -1, BX[3] = {0, 0, 0};
              for (int sa = -1; sa <= 0; ++sa)
                for (int sb = -1; sb <= 0; ++sb) {
                  int cell[3];
                  cell[e] = want[0];
                  const int ca = want[1] + sa, cb = want[2] + sb;
                  const int Na = d->root_nx[a] << 1, Nb = d->root_nx[bx] << 1;
                  if ((ca < 0 || ca >= Na) && d->bc[2 * a] != GRMHD_BC_PERIODIC) continue;
                  if ((cb < 0 || cb >= Nb) && d->bc[2 * bx] != GRMHD_BC_PERIODIC) continue;
                  cell[a] = ((ca % Na) + Na) % Na;
                  cell[bx] = ((cb % Nb) + Nb) % Nb;
                  const int q = own.at(1, cell);
                  if (lev_of(q) != 1 || (best >= 0 && q >= best)) continue;
                  int X[3];
                  if (owns_edge(q, e, want, X)) { best = q; BX[0] = X[0]; BX[1] = X[1]; BX[2] = X[2]; }
                }
              if (best < 0) continue;
              int G[3];
              G[e] = llc[e] + ie; G[a] = llc[a] + ka; G[bx] = llc[bx] + kb;
              p.fixE.push_back(FixE{lin_in(c, G), lin_in(best, BX), str_of(best, e), e, 0});
            }
          }
      }
    }
  }

  // every gather index must stay inside the pack's planes
  for (const GhostP &g : p.gP)
    if (g.dst < 0 || g.dst >= p.nct || g.src < 0 || g.src >= p.nct)
      return fail("internal: ghost map out of range", GRMHD_E_SHAPE);
  for (const GhostB &g : p.gB)
    if (g.dst < 0 || g.dst >= p.nct || g.src < 0 || g.src >= p.nct || g.comp < 0 || g.comp > 2)
      return fail("internal: face ghost map out of range", GRMHD_E_SHAPE);
  for (const GhostR &g : p.gR) {
    const long long last = g.n == 1 ? g.src : g.src + 1 + g.sj + g.sk;
    const long long lim = g.tgt ? p.nsP : p.nct;
    if (g.dst < 0 || g.dst >= lim || g.src < 0 || last >= p.nct || (g.n != 1 && g.n != 8))
      return fail("internal: restriction map out of range", GRMHD_E_SHAPE);
  }
  for (const GhostPro &g : p.gPro) {
    if (g.dst < 0 || g.dst >= p.nct) return fail("internal: prolongation map out of range", GRMHD_E_SHAPE);
    for (int q = 0; q < 7; ++q)
      if (g.s[q] < 0 || g.s[q] >= p.nsP) return fail("internal: prolongation stencil out of range", GRMHD_E_SHAPE);
  }
  for (const GhostBR &g : p.gBR) {
    const long long last = g.n == 1 ? g.src : g.src + g.st1 + g.st2;
    const long long lim = g.tgt ? p.nsB : p.nct;
    if (g.dst < 0 || g.dst >= lim || g.src < 0 || last >= p.nct || g.comp < 0 || g.comp > 2 ||
        (g.n != 1 && g.n != 4))
      return fail("internal: face restriction map out of range", GRMHD_E_SHAPE);
  }
  for (const FixF &f : p.fixF)
    if (f.dst < 0 || f.dst >= p.nct || f.src < 0 || f.src + f.st1 + f.st2 >= p.nct || f.D < 0 || f.D > 2)
      return fail("internal: flux correction map out of range", GRMHD_E_SHAPE);
  for (const FixE &f : p.fixE)
    if (f.dst < 0 || f.dst >= p.nct || f.src < 0 || f.src + f.st >= p.nct || f.e < 0 || f.e > 2)
      return fail("internal: EMF correction map out of range", GRMHD_E_SHAPE);
  for (const GhostBPro &g : p.gBPro)
    if (g.dst < 0 || g.dst >= p.nct || g.comp < 0 || g.comp > 2 || g.sa < 0 || g.sa >= p.nsB ||
        g.sb >= p.nsB)
      return fail("internal: face prolongation map out of range", GRMHD_E_SHAPE);

  // workspace carve-up
  size_t o = 0;
  auto take = [&](size_t bytes) { size_t r = o; o += align_up(bytes); return r; };
  p.o_F = take(sizeof(double) * 24 * (size_t)p.nct);
  p.o_Bcc = take(sizeof(double) * 3 * (size_t)p.nct);
  p.o_flags = take((size_t)p.nct);
  p.o_iters = take((size_t)p.nct);
  p.o_blocks = take(sizeof(BlockInfo) * p.nb);
  p.o_tab = take(sizeof(double) * (2 * p.rc.size() + 4 * p.sc.size()));
  p.o_flr = take(sizeof(double) * 4 * p.rc.size());   // two tables (see floor_table)
  for (int D = 0; D < 3; ++D)
    for (int sh = 0; sh < NSHAPE; ++sh) {
      p.o_tl[D][sh] = take(sizeof(int4) * p.tiles[D][sh].size());
      p.o_tlF[D][sh] = take(sizeof(int4) * p.tilesF[D][sh].size());
      p.o_tlP[D][sh] = take(sizeof(int4) * p.tilesP[D][sh].size());
    }
  p.o_planes = take(sizeof(int2) * p.planes.size());
  p.o_chi = take(sizeof(int2) * p.ch_int.size());
  p.o_che = take(sizeof(int2) * p.ch_ext.size());
  p.o_chb = take(sizeof(int2) * p.ch_bcc.size());
  p.o_gP = take(sizeof(GhostP) * std::max<size_t>(p.gP.size(), 1));
  p.o_gB = take(sizeof(GhostB) * std::max<size_t>(p.gB.size(), 1));
  p.o_gR = take(sizeof(GhostR) * p.gR.size());
  p.o_gPro = take(sizeof(GhostPro) * p.gPro.size());
  p.o_gBR = take(sizeof(GhostBR) * p.gBR.size());
  p.o_gBPro = take(sizeof(GhostBPro) * p.gBPro.size());
  p.o_SP = take(sizeof(double) * 5 * (size_t)p.nsP);
  p.o_SB = take(sizeof(double) * (size_t)p.nsB);
  p.o_E = take(p.maxlev > 0 ? sizeof(double) * 3 * (size_t)p.nct : 0);
  p.o_fixF = take(sizeof(FixF) * p.fixF.size());
  p.o_fixE = take(sizeof(FixE) * p.fixE.size());
  p.o_part = take(sizeof(double) * NPART * p.ch_int.size());
  p.o_res = take(sizeof(double) * RES_SLOTS);
  p.o_mlpw = take(sizeof(unsigned short) * MLPB_N);
  p.o_mlpf = take(sizeof(float) * MLPF_N);
  p.total = o;
  return GRMHD_OK;
}

}  // namespace

struct grmhd_pack {
  Plan plan;
  grmhd_pack_desc desc;
  grmhd_state_ptrs st;
  hipStream_t stream;
  char *ws;
  std::string err;
  bool mlp_bound = false;
  // optional per-kernel-family timing with events on the pack's stream
  bool prof = false;
  int shape[3] = {0, 0, 0};     // face-tile shape per direction (autotuned)
  int tune_sh = -1;             // >= 0 while the autotuner times one shape
  int tune_dir = -1;            // direction being timed (-1: all)
  int persist = 0;              // > 0: persistent flux grid of this many workgroups
  bool dt_ready = false;        // a reduction fold has written the device dt
  // fused stage (optional; single-level packs without the scalar): the flux
  // tiles do the hydro divergence, sources and RK update, the update kernel
  // keeps CT only
  bool fused = false;
  RkArgs rk{};                  // the stage being launched (fused tiles)
  // concurrent flux launches: auxiliary streams (default priority) and the
  // fork / join events; ls = the stream a tile launch goes to (null: stream)
  bool concurrent = true;
  hipStream_t aux[3] = {nullptr, nullptr, nullptr};
  hipEvent_t ev_fork = nullptr, ev_join[3] = {nullptr, nullptr, nullptr};
  hipStream_t ls = nullptr;
  // grmhd_step without a copy of its base: the first stage writes its result
  // over U0 / Bf0 (to_base), the first inversion and ghost fill and the second
  // stage then see U0 / Bf0 as the current state (swap), and the second stage
  // writes the combination over U / Bf
  bool to_base = false, swap = false;
  // the floors the radial floor table holds (Kerr-Schild packs), and whether
  // a step graph is being captured (the table is then brought up to date
  // before the capture and before each replay, never inside the graph)
  double flr_key[4] = {0.0, 0.0, 0.0, 0.0};
  bool flr_ok = false, capturing = false;
  ~grmhd_pack()
  {
    for (int k = 0; k < 3; ++k) {
      if (aux[k]) { (void)hipStreamSynchronize(aux[k]); (void)hipStreamDestroy(aux[k]); }
      if (ev_join[k]) (void)hipEventDestroy(ev_join[k]);
    }
    if (ev_fork) (void)hipEventDestroy(ev_fork);
  }
  // captured SSPRK2 step (dt read on the device)
  hipGraphExec_t gexec = nullptr;
  int g_guess = -1;
  double g_cfl = 0.0;
  grmhd_metric g_metric{};
  grmhd_eos g_eos{};
  grmhd_eos_table g_tab{};
  std::vector<hipEvent_t> ev_free;
  std::vector<std::tuple<int, hipEvent_t, hipEvent_t>> ev_rec;
  KArgs args() const
  {
    KArgs a;
    a.P = (double *)st.P; a.Bf = (double *)st.Bf; a.U = (double *)st.U;
    a.U0 = (double *)st.U0; a.Bf0 = (double *)st.Bf0;
    if (swap) { std::swap(a.U, a.U0); std::swap(a.Bf, a.Bf0); }
    a.F = (double *)(ws + plan.o_F);
    a.Bcc = (double *)(ws + plan.o_Bcc);
    a.flags = (int8_t *)(ws + plan.o_flags);
    a.iters = (uint8_t *)(ws + plan.o_iters);
    a.blocks = (const BlockInfo *)(ws + plan.o_blocks);
    const double *t = (const double *)(ws + plan.o_tab);
    const size_t n1 = plan.rc.size(), n2 = plan.sc.size();
    a.tab.rc = t; a.tab.rf = t + n1;
    a.tab.sc = t + 2 * n1; a.tab.cc = t + 2 * n1 + n2;
    a.tab.sf = t + 2 * n1 + 2 * n2; a.tab.cf = t + 2 * n1 + 3 * n2;
    a.flr_rho = (double *)(ws + plan.o_flr);
    a.flr_u = a.flr_rho + n1;
    a.met.M = 1.0; a.met.a = 0.0;
    std::memset(&a.eos, 0, sizeof a.eos);
    a.nct = plan.nct;
    a.ng = plan.ng;
    for (int d = 0; d < 3; ++d) a.active[d] = plan.active[d];
    a.SP = (double *)(ws + plan.o_SP);
    a.SB = (double *)(ws + plan.o_SB);
    a.nsp = plan.nsP;
    a.E = (double *)(ws + plan.o_E);
    std::memset(&a.et, 0, sizeof a.et);
    a.npv = 5 + desc.nscalar;
    a.nfail = (unsigned long long *)(ws + plan.o_res) + RES_NFAIL;
    return a;
  }
};

namespace {

int perr(grmhd_pack *p, const std::string &m, int code)
{
  if (p) p->err = m;
  g_err = m;
  return code;
}

// RAII event pair around the launches of one kernel family
struct Prof {
  grmhd_pack *p;
  int fam;
  hipEvent_t a = nullptr, b = nullptr;
  hipEvent_t take()
  {
    hipEvent_t e = nullptr;
    if (!p->ev_free.empty()) { e = p->ev_free.back(); p->ev_free.pop_back(); }
    else if (hipEventCreate(&e) != hipSuccess) e = nullptr;
    return e;
  }
  Prof(grmhd_pack *pp, int f) : p(pp), fam(f)
  {
    if (!p->prof) return;
    a = take(); b = take();
    if (a) (void)hipEventRecord(a, p->stream);
  }
  ~Prof()
  {
    if (!p->prof || !a || !b) return;
    (void)hipEventRecord(b, p->stream);
    p->ev_rec.emplace_back(fam, a, b);
  }
};

#define HIPCHK(p, x)                                                                  \
  do {                                                                                \
    hipError_t e_ = (x);                                                              \
    if (e_ != hipSuccess)                                                             \
      return perr(p, std::string(#x ": ") + hipGetErrorString(e_), GRMHD_E_HIP);      \
  } while (0)

#define LAUNCHCHK(p)                                                                  \
  do {                                                                                \
    hipError_t e_ = hipGetLastError();                                                \
    if (e_ != hipSuccess)                                                             \
      return perr(p, std::string("launch: ") + hipGetErrorString(e_), GRMHD_E_HIP);   \
  } while (0)

int check_metric(grmhd_pack *p, const grmhd_metric *m)
{
  if (!m) return perr(p, "null metric", GRMHD_E_INVALID);
  if (m->kind != GRMHD_METRIC_MINKOWSKI && m->kind != GRMHD_METRIC_KS_LOGSPH)
    return perr(p, "bad metric kind", GRMHD_E_INVALID);
  if (m->kind == GRMHD_METRIC_KS_LOGSPH && !(std::fabs(m->a) < m->M))
    return perr(p, "need |a| < M", GRMHD_E_INVALID);
  return 0;
}

void fill_eos(KArgs &a, const grmhd_eos *e)
{
  a.eos.gam = e->gamma;
  a.eos.rho_flr0 = e->rho_flr0; a.eos.rho_flr_pow = e->rho_flr_pow;
  a.eos.u_flr0 = e->u_flr0; a.eos.u_flr_pow = e->u_flr_pow;
  a.eos.W_max = e->W_max;
  a.eos.tol = e->c2p_tol > 0 ? e->c2p_tol : 1e-14;
  a.eos.max_iter = e->c2p_max_iter > 0 ? e->c2p_max_iter : 40;
  std::memset(&a.et, 0, sizeof a.et);
  if (const grmhd_eos_table *t = e->table) {
    a.et.d = (const double2 *)t->data;
    a.et.nx = t->n[0]; a.et.ny = t->n[1]; a.et.nz = t->n[2];
    for (int d = 0; d < 3; ++d) {
      a.et.lo[d] = t->lo[d];
      a.et.hi[d] = t->hi[d];
      a.et.ih[d] = (double)(t->n[d] - 1) / (t->hi[d] - t->lo[d]);
    }
    a.et.rho_min = std::exp(t->lo[0]); a.et.rho_max = std::exp(t->hi[0]);
    a.et.eps_min = std::exp(t->lo[1]); a.et.eps_max = std::exp(t->hi[1]);
  }
}

int check_eos(grmhd_pack *p, const grmhd_eos *e)
{
  if (!e) return perr(p, "null eos", GRMHD_E_INVALID);
  if (!e->table && !(e->gamma > 1.0)) return perr(p, "gamma must exceed 1", GRMHD_E_INVALID);
  if (!(e->W_max > 1.0)) return perr(p, "W_max must exceed 1", GRMHD_E_INVALID);
  if (const grmhd_eos_table *t = e->table) {
    if (!p->desc.nscalar) return perr(p, "a table needs the Y_e scalar (nscalar = 1)", GRMHD_E_INVALID);
    if (!t->data) return perr(p, "null table data", GRMHD_E_INVALID);
    for (int d = 0; d < 3; ++d) {
      if (t->n[d] < 2 || t->n[d] > (1 << 16)) return perr(p, "table axes need 2..65536 nodes", GRMHD_E_SHAPE);
      if (!std::isfinite(t->lo[d]) || !std::isfinite(t->hi[d]) || !(t->hi[d] > t->lo[d]))
        return perr(p, "table axis needs finite lo < hi", GRMHD_E_INVALID);
    }
    if ((long long)t->n[0] * t->n[1] * t->n[2] > (1LL << 30))
      return perr(p, "table too large", GRMHD_E_SHAPE);
    if (!(std::exp(t->lo[0]) > 0.0) || !(std::exp(t->lo[1]) > 0.0) ||
        !std::isfinite(std::exp(t->hi[0])) || !std::isfinite(std::exp(t->hi[1])))
      return perr(p, "table density / energy range out of double range", GRMHD_E_INVALID);
  }
  return 0;
}

template <typename T>
const T *dptr(const grmhd_pack *p, size_t off) { return (const T *)(p->ws + off); }

// ---- templated launch helpers (host dispatch over compile-time options)

template <int MK, int D, int RC, int FV, int RS, typename T, int SH, int NSC>
void launch_tiles(grmhd_pack *p, const KArgs &a)
{
  const Plan &pl = p->plan;
  const bool fz = p->fused && NSC == 0;
  const auto &L = fz ? pl.tilesF[D][SH] : pl.tiles[D][SH];
  if (L.empty()) return;
  Prof t(p, GRMHD_PROF_FLUX_X1 + D);
  const hipStream_t st = p->ls ? p->ls : p->stream;
  const int nt = (int)L.size();
  const int grid = p->persist > 0 ? std::min(nt, p->persist) : nt;
  if constexpr (NSC == 0) {
    if (fz) {
      hipLaunchKernelGGL((k_flux<MK, D, RC, FV, RS, T, SH, 0, 1>), dim3(grid), dim3(256), 0,
                         st, a, dptr<int4>(p, pl.o_tlF[D][SH]), nt, p->rk);
      return;
    }
    if constexpr (std::is_same<T, double>::value) {
      if (p->persist > 0) {
        // persistent grid: each workgroup streams its next stencil window
        // into LDS while it solves the current tile
        const int np = (int)pl.tilesP[D][SH].size();
        hipLaunchKernelGGL((k_flux_pf<MK, D, RC, FV, RS, SH>), dim3(std::min(np, p->persist)),
                           dim3(256), 0, st, a, dptr<int4>(p, pl.o_tlP[D][SH]), np);
        return;
      }
    }
  }
  hipLaunchKernelGGL((k_flux<MK, D, RC, FV, RS, T, SH, NSC, 0>), dim3(grid), dim3(256), 0,
                     st, a, dptr<int4>(p, pl.o_tl[D][SH]), nt, p->rk);
}

// Every shape is instantiated for the WENO5-Z-AOAH point-value path (the
// production reconstruction; with the passive scalar, for LLF); the other
// reconstructions and combinations use 16 x 16 tiles.
template <int RC, int FV, int RS, int NSC>
constexpr bool all_shapes() { return RC == RC_WENO && FV == 0 && (NSC == 0 || RS == RS_LLF); }

template <int MK, int D, int RC, int FV, int RS, typename T, int NSC>
void launch_tiles_sh(grmhd_pack *p, const KArgs &a, int sh)
{
  if constexpr (all_shapes<RC, FV, RS, NSC>()) {
    switch (sh) {
      case 1: launch_tiles<MK, D, RC, FV, RS, T, 1, NSC>(p, a); return;
      case 2: launch_tiles<MK, D, RC, FV, RS, T, 2, NSC>(p, a); return;
      case 3: launch_tiles<MK, D, RC, FV, RS, T, 3, NSC>(p, a); return;
      case 4: launch_tiles<MK, D, RC, FV, RS, T, 4, NSC>(p, a); return;
      default: break;
    }
  }
  launch_tiles<MK, D, RC, FV, RS, T, 0, NSC>(p, a);
}

template <int MK, int D, int RC, int FV, int RS, typename T, int NSC>
void launch_flux(grmhd_pack *p, const KArgs &a)
{
  launch_tiles_sh<MK, D, RC, FV, RS, T, NSC>(p, a, p->tune_sh >= 0 ? p->tune_sh : p->shape[D]);
}

template <int MK, int RC, int FV, int RS, typename T, int NSC>
void launch_flux3(grmhd_pack *p, const KArgs &a)
{
  // The three directions' tiles and the boundary planes write disjoint face
  // fluxes: with concurrency on, x2, x3 and the planes run on streams of their
  // own (forked from and joined back into the pack's stream, so a captured
  // step graph holds them as parallel branches) and fill one another's tails.
  // Per-family timing and autotuning keep everything on the pack's stream;
  // the fused stage's directions depend on one another.
  const Plan &pl = p->plan;
  const bool planes = p->tune_sh < 0 && !pl.planes.empty() && !p->fused;
  const bool conc = p->concurrent && p->aux[0] && !p->prof && p->tune_sh < 0 &&
                    p->tune_dir < 0 && !p->fused;
  if (conc) {
    (void)hipEventRecord(p->ev_fork, p->stream);
    for (int k = 0; k < 3; ++k) (void)hipStreamWaitEvent(p->aux[k], p->ev_fork, 0);
  }
  if (p->tune_dir < 0 || p->tune_dir == 0) launch_flux<MK, 0, RC, FV, RS, T, NSC>(p, a);
  p->ls = conc ? p->aux[0] : nullptr;
  if (p->tune_dir < 0 || p->tune_dir == 1) launch_flux<MK, 1, RC, FV, RS, T, NSC>(p, a);
  p->ls = conc ? p->aux[1] : nullptr;
  if (p->tune_dir < 0 || p->tune_dir == 2) launch_flux<MK, 2, RC, FV, RS, T, NSC>(p, a);
  p->ls = nullptr;
  if (planes) {
    Prof t(p, GRMHD_PROF_FLUX_PLANE);
    hipLaunchKernelGGL((k_flux_planes<MK, RC, FV, RS, T, NSC>), dim3(pl.planes.size()), dim3(64), 0,
                       conc ? p->aux[2] : p->stream, a, dptr<int2>(p, pl.o_planes));
  }
  if (conc) {
    for (int k = 0; k < 3; ++k) {
      (void)hipEventRecord(p->ev_join[k], p->aux[k]);
      (void)hipStreamWaitEvent(p->stream, p->ev_join[k], 0);
    }
  }
}

template <int MK, int RC, int FV, typename T, int NSC>
void launch_flux_rs(grmhd_pack *p, const KArgs &a, int rs)
{
  if (rs == RS_HLL) launch_flux3<MK, RC, FV, RS_HLL, T, NSC>(p, a);
  else launch_flux3<MK, RC, FV, RS_LLF, T, NSC>(p, a);
}

template <int MK, typename T, int NSC>
void launch_flux_rc(grmhd_pack *p, const KArgs &a, int rc, int fv, int rs)
{
  switch (rc) {
    case RC_CONST: launch_flux_rs<MK, RC_CONST, 0, T, NSC>(p, a, rs); break;
    case RC_PLM_MC: launch_flux_rs<MK, RC_PLM_MC, 0, T, NSC>(p, a, rs); break;
    case RC_PLM_MINMOD: launch_flux_rs<MK, RC_PLM_MINMOD, 0, T, NSC>(p, a, rs); break;
    case RC_MP5:
      if (fv) launch_flux_rs<MK, RC_MP5, 1, T, NSC>(p, a, rs);
      else launch_flux_rs<MK, RC_MP5, 0, T, NSC>(p, a, rs);
      break;
    default:
      if (fv) launch_flux_rs<MK, RC_WENO, 1, T, NSC>(p, a, rs);
      else launch_flux_rs<MK, RC_WENO, 0, T, NSC>(p, a, rs);
  }
}

template <int MK>
void launch_flux_all(grmhd_pack *p, const KArgs &a, int rc, int fv, int rs, int prec)
{
  if (p->desc.nscalar) launch_flux_rc<MK, double, 1>(p, a, rc, fv, rs);
  else if (prec == GRMHD_PREC_MIXED) launch_flux_rc<MK, float, 0>(p, a, rc, fv, rs);
  else launch_flux_rc<MK, double, 0>(p, a, rc, fv, rs);
}

// ---- refinement: block lookups over a plan and the remap maps

Owner owner_of(const Plan &P)
{
  Owner o;
  for (int d = 0; d < 3; ++d) {
    int g = P.root_nx[d];
    for (int b = 0; b < P.nb; ++b)
      g = gcd(g, gcd(P.blocks[b].n[d] >> P.lev[b], P.lloc[3 * b + d] >> P.lev[b]));
    o.g[d] = g;
    o.dims[d] = P.root_nx[d] / g;
  }
  o.id.assign((size_t)o.dims[0] * o.dims[1] * o.dims[2], -1);
  for (int b = 0; b < P.nb; ++b) {
    int lo[3], hi[3];
    for (int d = 0; d < 3; ++d) {
      lo[d] = (P.lloc[3 * b + d] >> P.lev[b]) / o.g[d];
      hi[d] = ((P.lloc[3 * b + d] + P.blocks[b].n[d]) >> P.lev[b]) / o.g[d];
    }
    for (int z = lo[2]; z < hi[2]; ++z)
      for (int y = lo[1]; y < hi[1]; ++y)
        for (int x = lo[0]; x < hi[0]; ++x) o.id[x + (size_t)o.dims[0] * (y + (size_t)o.dims[1] * z)] = b;
  }
  return o;
}

// cell index of the level-lev(b) cell c (global, in the block's level units) in block b
long long cell_at(const Plan &P, int b, const int c[3])
{
  const BlockInfo &bi = P.blocks[b];
  long long i[3];
  for (int d = 0; d < 3; ++d) i[d] = c[d] - P.lloc[3 * b + d] + P.ng;
  return bi.off + i[0] + (long long)bi.s[0] * (i[1] + (long long)bi.s[1] * i[2]);
}

long long stride_of(const Plan &P, int b, int d)
{
  const BlockInfo &bi = P.blocks[b];
  return d == 0 ? 1 : d == 1 ? (long long)bi.s[0] : (long long)bi.s[0] * bi.s[1];
}

struct RemapPlan {
  std::vector<std::pair<int, int>> copies;   // (dst block, src block) identical
  std::vector<RemapC> cells;
  std::vector<RemapF> faces;
  std::vector<RemapP> parents;
  double M[96];
  double id[3];
  size_t o_cells = 0, o_faces = 0, o_par = 0, o_M = 0, total = 0;
};

// Minimum-norm operator of the 8 children's divergence constraints.
void div_operator(const double id[3], double M[96])
{
  double D[8][12] = {{0}};
  for (int c = 0; c < 2; ++c)
    for (int b = 0; b < 2; ++b)
      for (int a = 0; a < 2; ++a) {
        const int r = a + 2 * b + 4 * c;
        D[r][b + 2 * c] = a ? -id[0] : id[0];
        D[r][4 + a + 2 * c] = b ? -id[1] : id[1];
        D[r][8 + a + 2 * b] = c ? -id[2] : id[2];
      }
  double A[8][16];
  for (int i = 0; i < 8; ++i)
    for (int j = 0; j < 8; ++j) {
      double s = 1.0;
      for (int k = 0; k < 12; ++k) s += D[i][k] * D[j][k];
      A[i][j] = s;
      A[i][8 + j] = i == j ? 1.0 : 0.0;
    }
  for (int c = 0; c < 8; ++c) {            // Gauss-Jordan (A is symmetric positive definite)
    const double piv = A[c][c];
    for (int k = 0; k < 16; ++k) A[c][k] /= piv;
    for (int r = 0; r < 8; ++r)
      if (r != c) {
        const double f = A[r][c];
        for (int k = 0; k < 16; ++k) A[r][k] -= f * A[c][k];
      }
  }
  for (int u = 0; u < 12; ++u)
    for (int v = 0; v < 8; ++v) {
      double s = 0.0;
      for (int k = 0; k < 8; ++k) s += D[k][u] * A[k][8 + v];
      M[u * 8 + v] = s;
    }
}

int build_remap(const Plan &Dp, const Plan &Sp, RemapPlan &R)
{
  for (int d = 0; d < 3; ++d)
    if (Dp.root_nx[d] != Sp.root_nx[d]) return fail("remap needs the same root grid", GRMHD_E_SHAPE);
  for (int q = 0; q < 6; ++q)
    if (Dp.bc[q] != Sp.bc[q]) return fail("remap needs the same boundaries", GRMHD_E_SHAPE);
  if (Dp.ng != Sp.ng) return fail("remap needs the same ghost depth", GRMHD_E_SHAPE);
  const Owner so = owner_of(Sp);
  const int ng = Dp.ng;
  auto sblk = [&](int l, const int c[3]) -> int {
    int c0[3];
    for (int d = 0; d < 3; ++d) {
      if (c[d] < 0 || c[d] >= (Sp.root_nx[d] << l)) return -1;
      c0[d] = c[d];
    }
    return so.at(l, c0);
  };
  R.id[0] = R.id[1] = R.id[2] = 0.0;
  for (int b = 0; b < Dp.nb; ++b)
    if (Dp.lev[b] == 1) {
      for (int d = 0; d < 3; ++d) R.id[d] = 1.0 / Dp.blocks[b].dx[d];
      break;
    }
  for (int b = 0; b < Dp.nb; ++b) {
    const BlockInfo &bi = Dp.blocks[b];
    const int l = Dp.lev[b];
    const int *L = &Dp.lloc[3 * b];
    {
      const int bs = sblk(l, L);
      if (bs >= 0 && Sp.lev[bs] == l && Sp.lloc[3 * bs] == L[0] && Sp.lloc[3 * bs + 1] == L[1] &&
          Sp.lloc[3 * bs + 2] == L[2] && Sp.blocks[bs].n[0] == bi.n[0] &&
          Sp.blocks[bs].n[1] == bi.n[1] && Sp.blocks[bs].n[2] == bi.n[2]) {
        R.copies.emplace_back(b, bs);
        continue;
      }
    }
    // cells
    for (int k = 0; k < bi.n[2]; ++k)
      for (int j = 0; j < bi.n[1]; ++j)
        for (int i = 0; i < bi.n[0]; ++i) {
          const int c[3] = {L[0] + i, L[1] + j, L[2] + k};
          const int bs = sblk(l, c);
          if (bs < 0) return fail("remap: a cell has no source block", GRMHD_E_SHAPE);
          RemapC m{};
          m.dst = cell_at(Dp, b, c);
          m.sj = (int)stride_of(Sp, bs, 1);
          m.sk = (int)stride_of(Sp, bs, 2);
          if (Sp.lev[bs] == l) {
            m.op = 0;
            m.src = cell_at(Sp, bs, c);
          } else if (l == 0) {
            const int c2[3] = {2 * c[0], 2 * c[1], 2 * c[2]};
            m.op = 2;
            m.src = cell_at(Sp, bs, c2);
          } else {
            const int pc[3] = {c[0] >> 1, c[1] >> 1, c[2] >> 1};
            m.op = 1;
            m.src = cell_at(Sp, bs, pc);
            m.oct = (c[0] & 1) | ((c[1] & 1) << 1) | ((c[2] & 1) << 2);
            for (int d = 0; d < 3; ++d) {
              const int li = pc[d] - Sp.lloc[3 * bs + d];       // interior position
              if (li > 0) m.inb |= 1 << (2 * d);
              if (li < Sp.blocks[bs].n[d] - 1) m.inb |= 1 << (2 * d + 1);
            }
            // the neighbours of the parent are in the source block's ghosts
            if (m.src - m.sk < Sp.blocks[bs].off ||
                m.src + m.sk >= Sp.blocks[bs].off + (long long)m.sk * Sp.blocks[bs].s[2])
              return fail("remap: prolongation stencil outside its block", GRMHD_E_SHAPE);
          }
          R.cells.push_back(m);
          if (l == 1 && Sp.lev[bs] == 0 && !(c[0] & 1) && !(c[1] & 1) && !(c[2] & 1))
            R.parents.push_back(RemapP{m.dst, m.src, (int)stride_of(Dp, b, 1), (int)stride_of(Dp, b, 2)});
        }
    // faces: along d the lower faces of the cells and the upper boundary face
    for (int d = 0; d < 3; ++d) {
      const int t1 = d == 0 ? 1 : 0, t2 = d == 2 ? 1 : 2;
      const int N = Dp.root_nx[d] << l;
      const bool per = Dp.bc[2 * d] == GRMHD_BC_PERIODIC;
      for (int k = 0; k < bi.n[2] + (d == 2); ++k)
        for (int j = 0; j < bi.n[1] + (d == 1); ++j)
          for (int i = 0; i < bi.n[0] + (d == 0); ++i) {
            int cu[3] = {L[0] + i, L[1] + j, L[2] + k};      // cell above the face
            int cl[3] = {cu[0], cu[1], cu[2]};
            cl[d] -= 1;                                       // cell below
            const bool upin = cu[d] < N;
            const int *cs = upin ? cu : cl;                   // the in-domain cell looked up
            const int bs = sblk(l, cs);
            if (bs < 0) return fail("remap: a face has no source block", GRMHD_E_SHAPE);
            RemapF f{};
            f.comp = d;
            f.dst = upin ? cell_at(Dp, b, cu) : cell_at(Dp, b, cl) + stride_of(Dp, b, d);
            // lower face index of (this level's) cell cu in block bb, or the
            // upper face of cl
            auto face_in = [&](const Plan &P, int bb, const int *cup, const int *clo, bool up) {
              return up ? cell_at(P, bb, cup) : cell_at(P, bb, clo) + stride_of(P, bb, d);
            };
            if (Sp.lev[bs] == l) {
              f.op = 0;
              f.src = face_in(Sp, bs, cu, cl, upin);
            } else if (l == 0) {
              // restriction: fine face 2 cu (or above fine cell 2 cl + e_d)
              int fu[3] = {2 * cu[0], 2 * cu[1], 2 * cu[2]};
              int fl[3] = {2 * cl[0], 2 * cl[1], 2 * cl[2]};
              fl[d] += 1;
              f.op = 1;
              f.src = face_in(Sp, bs, fu, fl, upin);
              f.st1 = stride_of(Sp, bs, t1);
              f.st2 = stride_of(Sp, bs, t2);
            } else {
              if (cu[d] & 1) continue;                        // inside a parent: k_remap_div
              // across the face: an existing fine cell gives its face
              int co[3] = {upin ? cl[0] : cu[0], upin ? cl[1] : cu[1], upin ? cl[2] : cu[2]};
              bool ok = true;
              if (co[d] < 0 || co[d] >= N) {
                if (per) co[d] = (co[d] + N) % N;
                else ok = false;
              }
              const int bo = ok ? sblk(1, co) : -1;
              if (bo >= 0 && Sp.lev[bo] == 1) {
                f.op = 0;
                // co is below the face when the looked-up cell is above it
                f.src = upin ? cell_at(Sp, bo, co) + stride_of(Sp, bo, d) : cell_at(Sp, bo, co);
              } else {
                const int pu[3] = {cu[0] >> 1, cu[1] >> 1, cu[2] >> 1};
                const int pl[3] = {cl[0] >> 1, cl[1] >> 1, cl[2] >> 1};
                f.op = 0;
                f.src = face_in(Sp, bs, pu, pl, upin);
              }
            }
            R.faces.push_back(f);
          }
    }
  }
  div_operator(R.id, R.M);
  size_t o = 0;
  auto take = [&](size_t bytes) { const size_t at = o; o += align_up(bytes); return at; };
  R.o_cells = take(sizeof(RemapC) * R.cells.size());
  R.o_faces = take(sizeof(RemapF) * R.faces.size());
  R.o_par = take(sizeof(RemapP) * R.parents.size());
  R.o_M = take(sizeof(double) * 96);
  R.total = o;
  return GRMHD_OK;
}

}  // namespace

extern "C" {

int grmhd_abi_version(void) { return GRMHD_ABI_VERSION; }

int grmhd_layout(const grmhd_pack_desc *desc, long long *offsets, long long *ncell_total)
{
  int rc = validate(desc);
  if (rc) return rc;
  std::vector<long long> off;
  long long n;
  layout(desc, off, n);
  if (offsets)
    for (int b = 0; b < desc->nblocks; ++b) offsets[b] = off[b];
  if (ncell_total) *ncell_total = n;
  return GRMHD_OK;
}

size_t grmhd_pack_workspace_bytes(const grmhd_pack_desc *desc)
{
  Plan p;
  if (build_plan(desc, p)) return 0;
  return p.total;
}

int grmhd_pack_create(const grmhd_pack_desc *desc, const grmhd_state_ptrs *state,
                      void *workspace, size_t ws_bytes, void *hip_stream, grmhd_pack **out)
{
  if (!out) return fail("null out", GRMHD_E_INVALID);
  *out = nullptr;
  if (!state || !state->P || !state->Bf || !state->U || !state->U0 || !state->Bf0)
    return fail("null state pointer", GRMHD_E_INVALID);
  if (!workspace || ((uintptr_t)workspace % ALIGN)) return fail("workspace null or unaligned", GRMHD_E_INVALID);
  grmhd_pack *p = new grmhd_pack();
  int rc = build_plan(desc, p->plan);
  if (rc) { delete p; return rc; }
  if (ws_bytes < p->plan.total) { delete p; return fail("workspace too small", GRMHD_E_SHAPE); }
  p->desc = *desc;
  p->desc.nx = p->desc.level = p->desc.lloc = nullptr;
  p->st = *state;
  p->stream = (hipStream_t)hip_stream;
  p->ws = (char *)workspace;
  const Plan &pl = p->plan;
  auto up = [&](size_t off, const void *src, size_t bytes) -> hipError_t {
    if (!bytes) return hipSuccess;
    return hipMemcpyAsync(p->ws + off, src, bytes, hipMemcpyHostToDevice, p->stream);
  };
  std::vector<double> tab;
  tab.insert(tab.end(), pl.rc.begin(), pl.rc.end());
  tab.insert(tab.end(), pl.rf.begin(), pl.rf.end());
  tab.insert(tab.end(), pl.sc.begin(), pl.sc.end());
  tab.insert(tab.end(), pl.cc.begin(), pl.cc.end());
  tab.insert(tab.end(), pl.sf.begin(), pl.sf.end());
  tab.insert(tab.end(), pl.cf.begin(), pl.cf.end());
  hipError_t e = hipSuccess;
  if (!e) e = up(pl.o_blocks, pl.blocks.data(), sizeof(BlockInfo) * pl.blocks.size());
  if (!e) e = up(pl.o_tab, tab.data(), sizeof(double) * tab.size());
  for (int D = 0; D < 3; ++D)
    for (int sh = 0; sh < NSHAPE; ++sh)
    {
      if (!e) e = up(pl.o_tl[D][sh], pl.tiles[D][sh].data(), sizeof(int4) * pl.tiles[D][sh].size());
      if (!e) e = up(pl.o_tlF[D][sh], pl.tilesF[D][sh].data(), sizeof(int4) * pl.tilesF[D][sh].size());
      if (!e) e = up(pl.o_tlP[D][sh], pl.tilesP[D][sh].data(), sizeof(int4) * pl.tilesP[D][sh].size());
    }
  if (!e) e = up(pl.o_planes, pl.planes.data(), sizeof(int2) * pl.planes.size());
  if (!e) e = up(pl.o_chi, pl.ch_int.data(), sizeof(int2) * pl.ch_int.size());
  if (!e) e = up(pl.o_che, pl.ch_ext.data(), sizeof(int2) * pl.ch_ext.size());
  if (!e) e = up(pl.o_chb, pl.ch_bcc.data(), sizeof(int2) * pl.ch_bcc.size());
  if (!e) e = up(pl.o_gP, pl.gP.data(), sizeof(GhostP) * pl.gP.size());
  if (!e) e = up(pl.o_gB, pl.gB.data(), sizeof(GhostB) * pl.gB.size());
  if (!e) e = up(pl.o_gR, pl.gR.data(), sizeof(GhostR) * pl.gR.size());
  if (!e) e = up(pl.o_gPro, pl.gPro.data(), sizeof(GhostPro) * pl.gPro.size());
  if (!e) e = up(pl.o_gBR, pl.gBR.data(), sizeof(GhostBR) * pl.gBR.size());
  if (!e) e = up(pl.o_gBPro, pl.gBPro.data(), sizeof(GhostBPro) * pl.gBPro.size());
  if (!e) e = up(pl.o_fixF, pl.fixF.data(), sizeof(FixF) * pl.fixF.size());
  if (!e) e = up(pl.o_fixE, pl.fixE.data(), sizeof(FixE) * pl.fixE.size());
  // flags / iteration counters / flux scratch start defined
  if (!e) e = hipMemsetAsync(p->ws + pl.o_flags, 0, 2 * align_up(pl.nct), p->stream);
  if (!e) e = hipMemsetAsync(p->ws + pl.o_F, 0, sizeof(double) * 24 * (size_t)pl.nct, p->stream);
  // reduction results (dt = 0 until the first fold) and the failure counter
  if (!e) e = hipMemsetAsync(p->ws + pl.o_res, 0, sizeof(double) * RES_SLOTS, p->stream);
  // host vectors must outlive the async copies
  if (!e) e = hipStreamSynchronize(p->stream);
  for (int k = 0; k < 3 && !e; ++k) e = hipStreamCreateWithFlags(&p->aux[k], hipStreamNonBlocking);
  if (!e) e = hipEventCreateWithFlags(&p->ev_fork, hipEventDisableTiming);
  for (int k = 0; k < 3 && !e; ++k) e = hipEventCreateWithFlags(&p->ev_join[k], hipEventDisableTiming);
  if (e) {
    std::string m = std::string("upload: ") + hipGetErrorString(e);
    delete p;
    return fail(m, GRMHD_E_HIP);
  }
  *out = p;
  return GRMHD_OK;
}

int grmhd_pack_destroy(grmhd_pack *p)
{
  if (!p) return GRMHD_E_INVALID;
  (void)hipStreamSynchronize(p->stream);
  for (auto &r : p->ev_rec) {
    (void)hipEventDestroy(std::get<1>(r));
    (void)hipEventDestroy(std::get<2>(r));
  }
  for (hipEvent_t e : p->ev_free) (void)hipEventDestroy(e);
  if (p->gexec) (void)hipGraphExecDestroy(p->gexec);
  delete p;
  return GRMHD_OK;
}

int grmhd_bind_state(grmhd_pack *p, const grmhd_state_ptrs *state)
{
  if (!p || !state || !state->P || !state->Bf || !state->U || !state->U0 || !state->Bf0)
    return perr(p, "null pointer", GRMHD_E_INVALID);
  p->st = *state;
  if (p->gexec) { (void)hipGraphExecDestroy(p->gexec); p->gexec = nullptr; }
  return GRMHD_OK;
}

int grmhd_fill_ghosts(grmhd_pack *p, const grmhd_metric *m)
{
  if (!p) return GRMHD_E_INVALID;
  if (int rc = check_metric(p, m)) return rc;
  KArgs a = p->args();
  a.met.M = m->M; a.met.a = m->a;
  const Plan &pl = p->plan;
  {
  Prof t(p, GRMHD_PROF_GHOST);
  if (!pl.gP.empty())
    hipLaunchKernelGGL(k_ghost_P, dim3((pl.gP.size() + 255) / 256), dim3(256), 0, p->stream, a,
                       dptr<GhostP>(p, pl.o_gP), (int)pl.gP.size());
  if (!pl.gB.empty())
    hipLaunchKernelGGL(k_ghost_B, dim3((pl.gB.size() + 255) / 256), dim3(256), 0, p->stream, a,
                       dptr<GhostB>(p, pl.o_gB), (int)pl.gB.size());
  // two-level meshes: restriction + coarse-view staging, then prolongation
  // (every gather above reads block interiors only)
  if (!pl.gR.empty())
    hipLaunchKernelGGL(k_ghost_avg, dim3((pl.gR.size() + 255) / 256), dim3(256), 0, p->stream, a,
                       dptr<GhostR>(p, pl.o_gR), (int)pl.gR.size());
  if (!pl.gBR.empty())
    hipLaunchKernelGGL(k_ghost_bavg, dim3((pl.gBR.size() + 255) / 256), dim3(256), 0, p->stream,
                       a, dptr<GhostBR>(p, pl.o_gBR), (int)pl.gBR.size());
  if (!pl.gPro.empty())
    hipLaunchKernelGGL(k_prolong_P, dim3((pl.gPro.size() + 255) / 256), dim3(256), 0, p->stream,
                       a, dptr<GhostPro>(p, pl.o_gPro), (int)pl.gPro.size());
  if (!pl.gBPro.empty())
    hipLaunchKernelGGL(k_prolong_B, dim3((pl.gBPro.size() + 255) / 256), dim3(256), 0, p->stream,
                       a, dptr<GhostBPro>(p, pl.o_gBPro), (int)pl.gBPro.size());
  }
  {
  Prof tb(p, GRMHD_PROF_BCC);
  if (m->kind == GRMHD_METRIC_KS_LOGSPH)
    hipLaunchKernelGGL(k_bcc<MK_KS>, dim3(pl.ch_bcc.size()), dim3(256), 0, p->stream, a,
                       dptr<int2>(p, pl.o_chb));
  else
    hipLaunchKernelGGL(k_bcc<MK_MINK>, dim3(pl.ch_bcc.size()), dim3(256), 0, p->stream, a,
                       dptr<int2>(p, pl.o_chb));
  }
  LAUNCHCHK(p);
  return GRMHD_OK;
}

int grmhd_stage(grmhd_pack *p, const grmhd_metric *m, const grmhd_eos *eos, double dt,
                const double rk[3])
{
  if (!p) return GRMHD_E_INVALID;
  if (int rc = check_metric(p, m)) return rc;
  if (int rc = check_eos(p, eos)) return rc;
  if (!rk) return perr(p, "null rk_coeffs", GRMHD_E_INVALID);
  if (!(dt > 0.0) && !p->dt_ready)
    return perr(p, "dt <= 0 asks for the device-resident dt, but no reduction has written one "
                   "(call grmhd_reductions or a grmhd_step with cfl > 0 first)", GRMHD_E_INVALID);
  KArgs a = p->args();
  a.met.M = m->M; a.met.a = m->a;
  fill_eos(a, eos);
  const Plan &pl = p->plan;
  const int rc = p->desc.recon, rs = p->desc.riemann, fv = p->desc.weno_fv;
  const int prec = p->desc.precision;
  const double *dtd = dptr<double>(p, pl.o_res);
  const int save = rk[1] == 0.0;
  p->rk = RkArgs{dt, dtd, rk[0], rk[1], rk[2], save};
  // update mode (rk_value): save or combine, result in the current arrays or
  // over the base arrays
  const int mode = p->to_base ? (save ? 2 : 3) : save;
  if (m->kind == GRMHD_METRIC_KS_LOGSPH) launch_flux_all<MK_KS>(p, a, rc, fv, rs, prec);
  else launch_flux_all<MK_MINK>(p, a, rc, fv, rs, prec);
  LAUNCHCHK(p);
  Prof t(p, GRMHD_PROF_UPDATE);
  const bool ks = m->kind == GRMHD_METRIC_KS_LOGSPH;
  if (pl.maxlev > 0) {
    // two levels: the fine fluxes and EMFs replace the coarse ones on level
    // boundaries (conservation and one interface field), then the update
    // reads the corrected edge arrays
    if (!pl.fixF.empty())
      hipLaunchKernelGGL(k_flux_fix, dim3((pl.fixF.size() + 255) / 256), dim3(256), 0, p->stream,
                         a, dptr<FixF>(p, pl.o_fixF), (int)pl.fixF.size());
    hipLaunchKernelGGL(k_emf, dim3(pl.ch_ext.size()), dim3(256), 0, p->stream, a,
                       dptr<int2>(p, pl.o_che));
    if (!pl.fixE.empty())
      hipLaunchKernelGGL(k_emf_fix, dim3((pl.fixE.size() + 255) / 256), dim3(256), 0, p->stream,
                         a, dptr<FixE>(p, pl.o_fixE), (int)pl.fixE.size());
    if (ks) hipLaunchKernelGGL((k_update<MK_KS, 1>), dim3(pl.ch_ext.size()), dim3(256), 0,
                               p->stream, a, dptr<int2>(p, pl.o_che), dt, dtd, rk[0], rk[1], rk[2], mode);
    else hipLaunchKernelGGL((k_update<MK_MINK, 1>), dim3(pl.ch_ext.size()), dim3(256), 0,
                            p->stream, a, dptr<int2>(p, pl.o_che), dt, dtd, rk[0], rk[1], rk[2], mode);
  } else if (p->desc.nscalar) {
    if (ks) hipLaunchKernelGGL((k_update<MK_KS, 0, 1>), dim3(pl.ch_ext.size()), dim3(256), 0,
                               p->stream, a, dptr<int2>(p, pl.o_che), dt, dtd, rk[0], rk[1], rk[2], mode);
    else hipLaunchKernelGGL((k_update<MK_MINK, 0, 1>), dim3(pl.ch_ext.size()), dim3(256), 0,
                            p->stream, a, dptr<int2>(p, pl.o_che), dt, dtd, rk[0], rk[1], rk[2], mode);
  } else if (p->fused) {
    // the flux tiles did the hydro update: constrained transport only
    if (ks) hipLaunchKernelGGL((k_update<MK_KS, 0, 0, 0>), dim3(pl.ch_ext.size()), dim3(256), 0,
                               p->stream, a, dptr<int2>(p, pl.o_che), dt, dtd, rk[0], rk[1], rk[2], mode);
    else hipLaunchKernelGGL((k_update<MK_MINK, 0, 0, 0>), dim3(pl.ch_ext.size()), dim3(256), 0,
                            p->stream, a, dptr<int2>(p, pl.o_che), dt, dtd, rk[0], rk[1], rk[2], mode);
  } else if (ks) {
    hipLaunchKernelGGL((k_update<MK_KS, 0>), dim3(pl.ch_ext.size()), dim3(256), 0, p->stream, a,
                       dptr<int2>(p, pl.o_che), dt, dtd, rk[0], rk[1], rk[2], mode);
  } else {
    hipLaunchKernelGGL((k_update<MK_MINK, 0>), dim3(pl.ch_ext.size()), dim3(256), 0, p->stream, a,
                       dptr<int2>(p, pl.o_che), dt, dtd, rk[0], rk[1], rk[2], mode);
  }
  LAUNCHCHK(p);
  return GRMHD_OK;
}

}  // extern "C"

namespace {

template <int MK, int RED, int NSC>
void launch_c2p_n(grmhd_pack *p, const KArgs &a, int guess, dim3 g, const int2 *ch,
                  const MlpDev &mlp, double *part)
{
  if (guess == 0) hipLaunchKernelGGL((k_c2p<MK, 0, RED, NSC>), g, dim3(256), 0, p->stream, a, ch, mlp, part);
  else if (guess == 1) hipLaunchKernelGGL((k_c2p<MK, 1, RED, NSC>), g, dim3(256), 0, p->stream, a, ch, mlp, part);
  else hipLaunchKernelGGL((k_c2p<MK, 2, RED, NSC>), g, dim3(256), 0, p->stream, a, ch, mlp, part);
}

template <int MK, int RED>
void launch_c2p(grmhd_pack *p, const KArgs &a, int guess, dim3 g, const int2 *ch,
                const MlpDev &mlp, double *part)
{
  if (p->desc.nscalar) launch_c2p_n<MK, RED, 1>(p, a, guess, g, ch, mlp, part);
  else launch_c2p_n<MK, RED, 0>(p, a, guess, g, ch, mlp, part);
}

// The radial floor table for the floors of eos (a few hundred entries),
// rewritten only when they differ from the ones it holds.  Inside a capture
// that the caller started (not grmhd_step_graph's own, which brings the table
// up to date outside its graph) the inversion uses a second table whose
// rewrite is always recorded, so each replay writes the floors it was
// captured with and the first table, which the host keeps track of, is never
// touched by a replay.
void floor_table(grmhd_pack *p, KArgs &a, const grmhd_eos *eos)
{
  const int nr = (int)p->plan.rc.size();
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(p->stream, &cs) != hipSuccess) cs = hipStreamCaptureStatusNone;
  if (cs == hipStreamCaptureStatusActive) {
    a.flr_rho += 2 * nr;
    a.flr_u += 2 * nr;
    if (nr > 0)
      hipLaunchKernelGGL(k_floor_tab, dim3((nr + 255) / 256), dim3(256), 0, p->stream, a, nr);
    return;
  }
  const double key[4] = {eos->rho_flr0, eos->rho_flr_pow, eos->u_flr0, eos->u_flr_pow};
  if (p->flr_ok && !std::memcmp(key, p->flr_key, sizeof key)) return;
  if (nr > 0)
    hipLaunchKernelGGL(k_floor_tab, dim3((nr + 255) / 256), dim3(256), 0, p->stream, a, nr);
  std::memcpy(p->flr_key, key, sizeof key);
  p->flr_ok = true;
}

// part != nullptr: the inversion also writes the reduction partials, and the
// final fold runs right after it (the reductions of grmhd_reductions).
int con2prim_impl(grmhd_pack *p, const grmhd_metric *m, const grmhd_eos *eos, int guess,
                  double cfl, bool reduce)
{
  if (!p) return GRMHD_E_INVALID;
  if (int rc = check_metric(p, m)) return rc;
  if (int rc = check_eos(p, eos)) return rc;
  if (guess < 0 || guess > 2) return perr(p, "bad guess kind", GRMHD_E_INVALID);
  if (guess == GRMHD_GUESS_MLP && !p->mlp_bound)
    return perr(p, "no learned guess bound", GRMHD_E_INVALID);
  KArgs a = p->args();
  a.met.M = m->M; a.met.a = m->a;
  fill_eos(a, eos);
  const Plan &pl = p->plan;
  const dim3 g(pl.ch_int.size());
  const int2 *ch = dptr<int2>(p, pl.o_chi);
  // the learned guess is evaluated inside the inversion kernel
  const MlpDev mlp{dptr<unsigned short>(p, pl.o_mlpw), dptr<float>(p, pl.o_mlpf)};
  double *part = (double *)(p->ws + pl.o_part);
  {
  Prof t(p, GRMHD_PROF_C2P);
  const bool ks = m->kind == GRMHD_METRIC_KS_LOGSPH;
  if (ks && !p->capturing) floor_table(p, a, eos);
  if (reduce) {
    if (ks) launch_c2p<MK_KS, 1>(p, a, guess, g, ch, mlp, part);
    else launch_c2p<MK_MINK, 1>(p, a, guess, g, ch, mlp, part);
  } else {
    if (ks) launch_c2p<MK_KS, 0>(p, a, guess, g, ch, mlp, part);
    else launch_c2p<MK_MINK, 0>(p, a, guess, g, ch, mlp, part);
  }
  }
  if (reduce) {
    p->dt_ready = true;
    Prof t(p, GRMHD_PROF_REDUCE);
    hipLaunchKernelGGL(k_reduce_fin, dim3(1), dim3(256), 0, p->stream, (const double *)part,
                       (int)pl.ch_int.size(), cfl, pl.dxmin, (double *)(p->ws + pl.o_res));
  }
  LAUNCHCHK(p);
  return GRMHD_OK;
}

}  // namespace

extern "C" {

int grmhd_con2prim(grmhd_pack *p, const grmhd_metric *m, const grmhd_eos *eos, int guess)
{
  return con2prim_impl(p, m, eos, guess, 0.0, false);
}

int grmhd_prim_to_cons(grmhd_pack *p, const grmhd_metric *m, const grmhd_eos *eos)
{
  if (!p) return GRMHD_E_INVALID;
  if (int rc = check_metric(p, m)) return rc;
  if (int rc = check_eos(p, eos)) return rc;
  KArgs a = p->args();
  a.met.M = m->M; a.met.a = m->a;
  fill_eos(a, eos);
  const Plan &pl = p->plan;
  const bool ks = m->kind == GRMHD_METRIC_KS_LOGSPH;
  const dim3 g(pl.ch_int.size());
  const int2 *ch = dptr<int2>(p, pl.o_chi);
  if (p->desc.nscalar) {
    if (ks) hipLaunchKernelGGL((k_p2c<MK_KS, 1>), g, dim3(256), 0, p->stream, a, ch);
    else hipLaunchKernelGGL((k_p2c<MK_MINK, 1>), g, dim3(256), 0, p->stream, a, ch);
  } else {
    if (ks) hipLaunchKernelGGL((k_p2c<MK_KS, 0>), g, dim3(256), 0, p->stream, a, ch);
    else hipLaunchKernelGGL((k_p2c<MK_MINK, 0>), g, dim3(256), 0, p->stream, a, ch);
  }
  LAUNCHCHK(p);
  return GRMHD_OK;
}

int grmhd_reductions(grmhd_pack *p, const grmhd_metric *m, const grmhd_eos *eos, double cfl,
                     grmhd_reduction_out *out)
{
  if (!p) return GRMHD_E_INVALID;
  if (int rc = check_metric(p, m)) return rc;
  if (int rc = check_eos(p, eos)) return rc;
  KArgs a = p->args();
  a.met.M = m->M; a.met.a = m->a;
  fill_eos(a, eos);
  const Plan &pl = p->plan;
  double *part = (double *)(p->ws + pl.o_part);
  double *res = (double *)(p->ws + pl.o_res);
  {
  Prof t(p, GRMHD_PROF_REDUCE);
  const bool ks = m->kind == GRMHD_METRIC_KS_LOGSPH;
  const dim3 g(pl.ch_int.size());
  const int2 *ch = dptr<int2>(p, pl.o_chi);
  if (p->desc.nscalar) {
    if (ks) hipLaunchKernelGGL((k_reduce<MK_KS, 1>), g, dim3(256), 0, p->stream, a, ch, part);
    else hipLaunchKernelGGL((k_reduce<MK_MINK, 1>), g, dim3(256), 0, p->stream, a, ch, part);
  } else {
    if (ks) hipLaunchKernelGGL((k_reduce<MK_KS, 0>), g, dim3(256), 0, p->stream, a, ch, part);
    else hipLaunchKernelGGL((k_reduce<MK_MINK, 0>), g, dim3(256), 0, p->stream, a, ch, part);
  }
  hipLaunchKernelGGL(k_reduce_fin, dim3(1), dim3(256), 0, p->stream, (const double *)part,
                     (int)pl.ch_int.size(), cfl, pl.dxmin, res);
  }
  LAUNCHCHK(p);
  p->dt_ready = true;
  if (out) {
    double h[RES_SLOTS];
    HIPCHK(p, hipMemcpyAsync(h, res, sizeof h, hipMemcpyDeviceToHost, p->stream));
    HIPCHK(p, hipStreamSynchronize(p->stream));
    out->dt = h[0];
    out->divb_rel = h[1];
    out->divb_max = h[2];
    for (int v = 0; v < 5; ++v) out->totals[v] = h[3 + v];
    out->c2p_fail = (long long)h[8];
    out->floor_hits = (long long)h[9];
    long long ncell = 0, nwave = 0;
    for (int b = 0; b < pl.nb; ++b) {
      const long long nb = (long long)pl.blocks[b].n[0] * pl.blocks[b].n[1] * pl.blocks[b].n[2];
      ncell += nb;
    }
    for (const int2 &c : pl.ch_int) {
      const BlockInfo &b = pl.blocks[c.x];
      const long long nb = (long long)b.n[0] * b.n[1] * b.n[2];
      const long long live = std::min<long long>(256, nb - c.y);
      nwave += (live + 63) / 64;
    }
    unsigned long long nfail;
    std::memcpy(&nfail, &h[RES_NFAIL], sizeof nfail);
    out->c2p_fail_total = (long long)nfail;
    out->guess_fallback = (long long)h[14];
    out->total_scalar = h[15];
    out->c2p_iter_mean = ncell ? h[10] / ncell : 0.0;
    out->c2p_iter_wavemax_mean = nwave ? h[11] / nwave : 0.0;
  }
  return GRMHD_OK;
}

int grmhd_mlp_bind(grmhd_pack *p, const float *params, const float *feat_mean,
                   const float *feat_std)
{
  if (!p || !params || !feat_mean || !feat_std) return perr(p, "null pointer", GRMHD_E_INVALID);
  const Plan &pl = p->plan;
  hipLaunchKernelGGL(k_mlp_pack, dim3((64 * 64 + 255) / 256), dim3(256), 0, p->stream, params,
                     feat_mean, feat_std, (unsigned short *)(p->ws + pl.o_mlpw),
                     (float *)(p->ws + pl.o_mlpf));
  LAUNCHCHK(p);
  p->mlp_bound = true;
  return GRMHD_OK;
}

}  // extern "C"

namespace {
// Z1 H1 Z2 H2 Z3 H3 d1 d2 d3 (64 each), out, d4 (2 each), grads, loss partials,
// BF16 weights + FP32 biases for the MFMA inference
constexpr size_t mlp_scratch_floats(size_t b)
{
  return 9 * 64 * b + 2 * 2 * b + MLP_NPARAM + (b + 255) / 256 + 4;
}
constexpr size_t mlp_scratch_bytes(size_t b)
{
  return align_up(mlp_scratch_floats(b) * sizeof(float)) + align_up(MLPB_N * 2) +
         align_up(MLPF_N * 4);
}

// Device memory of grmhd_mlp_train_step_noalloc: the same scratch as the
// caller-provided one of grmhd_mlp_train_step, sized for the largest batch it
// takes.  Each GPU the library runs on holds its own copy until the process
// ends.  In host code this name is only a stand-in for the symbol: its device
// address (per device) comes from hipGetSymbolAddress.
constexpr size_t NOALLOC_BYTES = mlp_scratch_bytes(GRMHD_MLP_NOALLOC_MAX_BATCH);
}  // namespace

static __device__ __align__(256) unsigned char noalloc_scratch[NOALLOC_BYTES];

extern "C" size_t grmhd_mlp_scratch_bytes(int batch)
{
  if (batch < 1) return 0;
  return mlp_scratch_bytes((size_t)batch);
}

namespace {
struct MlpScratch {
  float *Z1, *H1, *Z2, *H2, *Z3, *H3, *d1, *d2, *d3, *out, *d4, *grad, *part, *loss;
  unsigned short *w;
  float *f;
};
MlpScratch carve(void *s, int batch)
{
  float *q = (float *)s;
  const size_t b = (size_t)batch;
  MlpScratch m;
  m.Z1 = q; q += 64 * b; m.H1 = q; q += 64 * b; m.Z2 = q; q += 64 * b; m.H2 = q; q += 64 * b;
  m.Z3 = q; q += 64 * b; m.H3 = q; q += 64 * b; m.d1 = q; q += 64 * b; m.d2 = q; q += 64 * b;
  m.d3 = q; q += 64 * b; m.out = q; q += 2 * b; m.d4 = q; q += 2 * b;
  m.grad = q; q += MLP_NPARAM; m.part = q; q += (b + 255) / 256; m.loss = q; q += 4;
  char *c = (char *)s + align_up(mlp_scratch_floats(b) * sizeof(float));
  m.w = (unsigned short *)c;
  m.f = (float *)(c + align_up(MLPB_N * 2));
  return m;
}

dim3 g256(size_t n) { return dim3((unsigned)((n + 255) / 256)); }

// forward + loss + backward into m.grad; returns 0 or a HIP error
hipError_t mlp_fwd_bwd(const float *P, const float *X, const float *Y, int B, MlpScratch &m,
                       hipStream_t st)
{
  const float *W1 = P + MLP_OFF_W1, *b1 = P + MLP_OFF_B1, *W2 = P + MLP_OFF_W2,
              *b2 = P + MLP_OFF_B2, *W3 = P + MLP_OFF_W3, *b3 = P + MLP_OFF_B3,
              *W4 = P + MLP_OFF_W4, *b4 = P + MLP_OFF_B4;
  float *g = m.grad;
  hipLaunchKernelGGL(k_dense_fwd, g256((size_t)B * 64), dim3(256), 0, st, X, 5, W1, b1, 64, m.Z1, m.H1, B, 1);
  hipLaunchKernelGGL(k_dense_fwd, g256((size_t)B * 64), dim3(256), 0, st, m.H1, 64, W2, b2, 64, m.Z2, m.H2, B, 1);
  hipLaunchKernelGGL(k_dense_fwd, g256((size_t)B * 64), dim3(256), 0, st, m.H2, 64, W3, b3, 64, m.Z3, m.H3, B, 1);
  hipLaunchKernelGGL(k_dense_fwd, g256((size_t)B * 2), dim3(256), 0, st, m.H3, 64, W4, b4, 2, m.out, m.out, B, 0);
  hipLaunchKernelGGL(k_mse, g256(B), dim3(256), 0, st, m.out, Y, B, m.d4, m.part);
  hipLaunchKernelGGL(k_sum, dim3(1), dim3(256), 0, st, m.part, (B + 255) / 256, m.loss);
  hipLaunchKernelGGL(k_dense_bwd_weight, g256(2 * 65), dim3(256), 0, st, m.d4, 2, m.H3, 64, B,
                     g + MLP_OFF_W4, g + MLP_OFF_B4);
  hipLaunchKernelGGL(k_dense_bwd_data, g256((size_t)B * 64), dim3(256), 0, st, m.d4, 2, W4, 64, m.Z3, m.d3, B);
  hipLaunchKernelGGL(k_dense_bwd_weight, g256(64 * 65), dim3(256), 0, st, m.d3, 64, m.H2, 64, B,
                     g + MLP_OFF_W3, g + MLP_OFF_B3);
  hipLaunchKernelGGL(k_dense_bwd_data, g256((size_t)B * 64), dim3(256), 0, st, m.d3, 64, W3, 64, m.Z2, m.d2, B);
  hipLaunchKernelGGL(k_dense_bwd_weight, g256(64 * 65), dim3(256), 0, st, m.d2, 64, m.H1, 64, B,
                     g + MLP_OFF_W2, g + MLP_OFF_B2);
  hipLaunchKernelGGL(k_dense_bwd_data, g256((size_t)B * 64), dim3(256), 0, st, m.d2, 64, W2, 64, m.Z1, m.d1, B);
  hipLaunchKernelGGL(k_dense_bwd_weight, g256(64 * 6), dim3(256), 0, st, m.d1, 64, X, 5, B,
                     g + MLP_OFF_W1, g + MLP_OFF_B1);
  return hipGetLastError();
}
}  // namespace

extern "C" {

int grmhd_mlp_grad(const float *params, const float *X, const float *Y, int batch, float *grad,
                   float *loss, void *scratch, size_t scratch_bytes, void *hip_stream)
{
  if (!params || !X || !Y || !grad || !loss || !scratch || batch < 1)
    return fail("null pointer or empty batch", GRMHD_E_INVALID);
  if (scratch_bytes < grmhd_mlp_scratch_bytes(batch)) return fail("scratch too small", GRMHD_E_SHAPE);
  hipStream_t st = (hipStream_t)hip_stream;
  MlpScratch m = carve(scratch, batch);
  hipError_t e = mlp_fwd_bwd(params, X, Y, batch, m, st);
  if (!e) e = hipMemcpyAsync(grad, m.grad, sizeof(float) * MLP_NPARAM, hipMemcpyDeviceToDevice, st);
  if (!e) e = hipMemcpyAsync(loss, m.loss, sizeof(float), hipMemcpyDeviceToDevice, st);
  if (e) return fail(std::string("mlp grad: ") + hipGetErrorString(e), GRMHD_E_HIP);
  return GRMHD_OK;
}

}  // extern "C"

namespace {
// forward, loss, backward and one Adam step on a carved scratch
int train_step_on(float *params, float *adam_m, float *adam_v, const float *X, const float *Y,
                  int batch, float lr, int t, float *loss, void *scratch, hipStream_t st)
{
  MlpScratch m = carve(scratch, batch);
  hipError_t e = mlp_fwd_bwd(params, X, Y, batch, m, st);
  if (!e) {
    hipLaunchKernelGGL(k_adam, g256(MLP_NPARAM), dim3(256), 0, st, params, m.grad, adam_m, adam_v,
                       MLP_NPARAM, lr, 0.9f, 0.999f, 1e-8f, t);
    e = hipGetLastError();
  }
  if (!e) e = hipMemcpyAsync(loss, m.loss, sizeof(float), hipMemcpyDeviceToDevice, st);
  if (e) return fail(std::string("mlp train: ") + hipGetErrorString(e), GRMHD_E_HIP);
  return GRMHD_OK;
}

// Device address of noalloc_scratch on the current device, looked up once per
// device (with that device current) and kept.
constexpr int NOALLOC_MAXDEV = 64;
std::mutex noalloc_mu;
void *noalloc_ptr[NOALLOC_MAXDEV] = {};

int noalloc_scratch_ptr(hipStream_t st, void **out)
{
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e) return fail(std::string("hipGetDevice: ") + hipGetErrorString(e), GRMHD_E_HIP);
  if (dev < 0 || dev >= NOALLOC_MAXDEV) return fail("device index out of range", GRMHD_E_INVALID);
  if (st) {
    int sdev = -1;
    e = hipStreamGetDevice(st, &sdev);
    if (e) return fail(std::string("hipStreamGetDevice: ") + hipGetErrorString(e), GRMHD_E_HIP);
    if (sdev != dev)
      return fail("the stream belongs to another device than the current one", GRMHD_E_INVALID);
  }
  std::lock_guard<std::mutex> lk(noalloc_mu);
  if (!noalloc_ptr[dev]) {
    void *p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(noalloc_scratch));
    if (e || !p)
      return fail(std::string("hipGetSymbolAddress(noalloc_scratch): ") + hipGetErrorString(e),
                  GRMHD_E_HIP);
    noalloc_ptr[dev] = p;
  }
  *out = noalloc_ptr[dev];
  return GRMHD_OK;
}
}  // namespace

extern "C" {

int grmhd_mlp_train_step(float *params, float *adam_m, float *adam_v, const float *X,
                         const float *Y, int batch, float lr, int t, float *loss, void *scratch,
                         size_t scratch_bytes, void *hip_stream)
{
  if (!params || !adam_m || !adam_v || !X || !Y || !loss || !scratch || batch < 1 || t < 1)
    return fail("bad argument", GRMHD_E_INVALID);
  if (scratch_bytes < grmhd_mlp_scratch_bytes(batch)) return fail("scratch too small", GRMHD_E_SHAPE);
  return train_step_on(params, adam_m, adam_v, X, Y, batch, lr, t, loss, scratch,
                       (hipStream_t)hip_stream);
}

int grmhd_mlp_train_step_noalloc(float *params, float *adam_m, float *adam_v, const float *X,
                                 const float *Y, int batch, float lr, int t, float *loss,
                                 void *hip_stream)
{
  if (!params || !adam_m || !adam_v || !X || !Y || !loss || batch < 1 || t < 1)
    return fail("bad argument", GRMHD_E_INVALID);
  if (batch > GRMHD_MLP_NOALLOC_MAX_BATCH)
    return fail("batch " + std::to_string(batch) + " exceeds the " +
                    std::to_string(GRMHD_MLP_NOALLOC_MAX_BATCH) +
                    " samples the library's own scratch holds (use grmhd_mlp_train_step)",
                GRMHD_E_SHAPE);
  hipStream_t st = (hipStream_t)hip_stream;
  void *scr = nullptr;
  if (int rc = noalloc_scratch_ptr(st, &scr)) return rc;
  return train_step_on(params, adam_m, adam_v, X, Y, batch, lr, t, loss, scr, st);
}

int grmhd_mlp_infer(const float *params, const float *feat_mean, const float *feat_std,
                    const float *X, float *Y, int n, void *scratch, size_t scratch_bytes,
                    void *hip_stream)
{
  if (!params || !feat_mean || !feat_std || !X || !Y || !scratch || n < 1)
    return fail("bad argument", GRMHD_E_INVALID);
  if (scratch_bytes < grmhd_mlp_scratch_bytes(1)) return fail("scratch too small", GRMHD_E_SHAPE);
  hipStream_t st = (hipStream_t)hip_stream;
  MlpScratch m = carve(scratch, 1);
  hipLaunchKernelGGL(k_mlp_pack, dim3((64 * 64 + 255) / 256), dim3(256), 0, st, params,
                     feat_mean, feat_std, m.w, m.f);
  MlpDev md{m.w, m.f};
  hipLaunchKernelGGL(k_mlp_infer, dim3((n + 63) / 64), dim3(64), 0, st, md, X, Y, n);
  hipError_t e = hipGetLastError();
  if (e) return fail(std::string("mlp infer: ") + hipGetErrorString(e), GRMHD_E_HIP);
  return GRMHD_OK;
}

int grmhd_m1_source(grmhd_pack *p, const grmhd_metric *m, double dt, int nspecies, void *R,
                    const void *kappa, int couple, double tol, int max_iter, void *iters)
{
  if (!p) return GRMHD_E_INVALID;
  if (int rc = check_metric(p, m)) return rc;
  if (!R || !kappa) return perr(p, "null moments or opacities", GRMHD_E_INVALID);
  if (nspecies < 1 || nspecies > 8) return perr(p, "nspecies must be 1..8", GRMHD_E_INVALID);
  if (!(dt >= 0.0) || !std::isfinite(dt)) return perr(p, "dt must be finite and >= 0", GRMHD_E_INVALID);
  if (max_iter < 1 || max_iter > 254) return perr(p, "max_iter must be 1..254", GRMHD_E_INVALID);
  if (!(tol > 0.0)) tol = 1e-13;
  KArgs a = p->args();
  a.met.M = m->M; a.met.a = m->a;
  const Plan &pl = p->plan;
  Prof t(p, GRMHD_PROF_M1);
  hipLaunchKernelGGL(k_m1_source, dim3(pl.ch_int.size()), dim3(256), 0, p->stream, a,
                     dptr<int2>(p, pl.o_chi), nspecies, (double *)R, (const double *)kappa, dt,
                     tol, max_iter, couple ? 1 : 0, (uint8_t *)iters,
                     m->kind == GRMHD_METRIC_KS_LOGSPH ? (int)MK_KS : (int)MK_MINK);
  LAUNCHCHK(p);
  return GRMHD_OK;
}

int grmhd_tag(grmhd_pack *p, int var, double *block_max)
{
  if (!p || !block_max) return GRMHD_E_INVALID;
  if (var < 0 || var >= p->args().npv) return perr(p, "bad tag variable", GRMHD_E_INVALID);
  const Plan &pl = p->plan;
  KArgs a = p->args();
  double *part = (double *)(p->ws + pl.o_part);
  hipLaunchKernelGGL(k_tag, dim3(pl.ch_int.size()), dim3(256), 0, p->stream, a,
                     dptr<int2>(p, pl.o_chi), var, part);
  LAUNCHCHK(p);
  std::vector<double> h(pl.ch_int.size());
  HIPCHK(p, hipMemcpyAsync(h.data(), part, sizeof(double) * h.size(), hipMemcpyDeviceToHost, p->stream));
  HIPCHK(p, hipStreamSynchronize(p->stream));
  for (int b = 0; b < pl.nb; ++b) block_max[b] = 0.0;
  for (size_t c = 0; c < h.size(); ++c)
    block_max[pl.ch_int[c].x] = std::max(block_max[pl.ch_int[c].x], h[c]);
  return GRMHD_OK;
}

int grmhd_regrid_layout(const grmhd_pack_desc *desc, const int *tags, int cap, int *nb_out,
                        int *nx_out, int *lloc_out, int *level_out)
{
  if (!desc || !tags || !nb_out) return fail("null argument", GRMHD_E_INVALID);
  if (int rc = validate(desc)) return rc;
  const int nb = desc->nblocks;
  auto lev = [&](int b) { return desc->level ? desc->level[b] : 0; };
  std::vector<int> onx, oll, olv;
  auto emit = [&](int l, const int *n, const int *ll) {
    for (int d = 0; d < 3; ++d) { onx.push_back(n[d]); oll.push_back(ll[d]); }
    olv.push_back(l);
  };
  // sibling groups of level-1 blocks: 8 blocks of one size m at base + {0, m}^3,
  // base a multiple of 2m
  std::map<std::tuple<int, int, int, int, int, int>, std::vector<int>> groups;
  for (int b = 0; b < nb; ++b) {
    if (lev(b) != 1) continue;
    const int *n = desc->nx + 3 * b, *ll = desc->lloc + 3 * b;
    if (n[0] != n[1] || n[1] != n[2]) continue;
    const int m = n[0];
    groups[std::make_tuple(m, ll[0] - ll[0] % (2 * m), ll[1] - ll[1] % (2 * m),
                           ll[2] - ll[2] % (2 * m), 0, 0)].push_back(b);
  }
  std::vector<int> gleader(nb, -1);     // -2: merged into its group's leader
  for (auto &kv : groups) {
    auto &v = kv.second;
    if (v.size() != 8) continue;
    bool all = true;
    for (int b : v) all = all && tags[b] < 0;
    if (!all) continue;
    const int lead = *std::min_element(v.begin(), v.end());
    for (int b : v) gleader[b] = b == lead ? lead : -2;
  }
  for (int b = 0; b < nb; ++b) {
    const int *n = desc->nx + 3 * b, *ll = desc->lloc + 3 * b;
    if (lev(b) == 0 && tags[b] > 0 && !(n[0] & 1) && !(n[1] & 1) && !(n[2] & 1)) {
      for (int z = 0; z < 2; ++z)
        for (int y = 0; y < 2; ++y)
          for (int x = 0; x < 2; ++x) {
            const int cl[3] = {2 * ll[0] + x * n[0], 2 * ll[1] + y * n[1], 2 * ll[2] + z * n[2]};
            emit(1, n, cl);
          }
    } else if (gleader[b] == b) {
      const int m = n[0];
      const int cl[3] = {(ll[0] - ll[0] % (2 * m)) / 2, (ll[1] - ll[1] % (2 * m)) / 2,
                         (ll[2] - ll[2] % (2 * m)) / 2};
      const int cn[3] = {m, m, m};
      emit(0, cn, cl);
    } else if (lev(b) == 1 && tags[b] < 0 && gleader[b] != -2 && n[0] / 2 >= desc->ng &&
               n[1] / 2 >= desc->ng && n[2] / 2 >= desc->ng) {
      const int cn[3] = {n[0] / 2, n[1] / 2, n[2] / 2};
      const int cl[3] = {ll[0] / 2, ll[1] / 2, ll[2] / 2};
      emit(0, cn, cl);
    } else if (gleader[b] != -2) {
      emit(lev(b), n, ll);
    }
  }
  *nb_out = (int)olv.size();
  if ((int)olv.size() > cap || !nx_out || !lloc_out || !level_out)
    return fail("regrid: output capacity too small", GRMHD_E_SHAPE);
  std::copy(onx.begin(), onx.end(), nx_out);
  std::copy(oll.begin(), oll.end(), lloc_out);
  std::copy(olv.begin(), olv.end(), level_out);
  return GRMHD_OK;
}

size_t grmhd_remap_scratch_bytes(const grmhd_pack *dst, const grmhd_pack *src)
{
  if (!dst || !src) return 0;
  RemapPlan R;
  if (build_remap(dst->plan, src->plan, R)) return 0;
  return R.total;
}

int grmhd_remap(grmhd_pack *dst, const grmhd_pack *src, const grmhd_metric *metric,
                const grmhd_eos *eos, void *scratch, size_t scratch_bytes)
{
  if (!dst || !src || !scratch) return perr(dst, "null argument", GRMHD_E_INVALID);
  if (dst == src || dst->st.P == src->st.P || dst->st.U == src->st.U || dst->st.Bf == src->st.Bf)
    return perr(dst, "remap needs two packs with their own state arrays", GRMHD_E_INVALID);
  if (int rc = check_metric(dst, metric)) return rc;
  if (int rc = check_eos(dst, eos)) return rc;
  if (dst->desc.nscalar || src->desc.nscalar)
    return perr(dst, "remap carries no passive scalar", GRMHD_E_UNSUPPORTED);
  if ((uintptr_t)scratch % ALIGN) return perr(dst, "scratch must be 256-byte aligned", GRMHD_E_INVALID);
  RemapPlan R;
  if (int rc = build_remap(dst->plan, src->plan, R)) return perr(dst, g_err, rc);
  if (scratch_bytes < R.total) return perr(dst, "remap scratch too small", GRMHD_E_SHAPE);
  char *w = (char *)scratch;
  hipStream_t st = dst->stream;
  const Plan &Dp = dst->plan, &Sp = src->plan;
  auto up = [&](size_t off, const void *h, size_t bytes) -> hipError_t {
    return bytes ? hipMemcpyAsync(w + off, h, bytes, hipMemcpyHostToDevice, st) : hipSuccess;
  };
  HIPCHK(dst, up(R.o_cells, R.cells.data(), sizeof(RemapC) * R.cells.size()));
  HIPCHK(dst, up(R.o_faces, R.faces.data(), sizeof(RemapF) * R.faces.size()));
  HIPCHK(dst, up(R.o_par, R.parents.data(), sizeof(RemapP) * R.parents.size()));
  HIPCHK(dst, up(R.o_M, R.M, sizeof(double) * 96));
  RemapArgs ra;
  ra.sP = (const double *)src->st.P; ra.sU = (const double *)src->st.U;
  ra.sBf = (const double *)src->st.Bf;
  ra.dP = (double *)dst->st.P; ra.dU = (double *)dst->st.U; ra.dBf = (double *)dst->st.Bf;
  ra.snct = Sp.nct; ra.dnct = Dp.nct;
  // identical blocks: whole padded blocks, every plane
  for (const auto &cp : R.copies) {
    const BlockInfo &db = Dp.blocks[cp.first], &sb = Sp.blocks[cp.second];
    const size_t cnt = (size_t)db.s[0] * db.s[1] * db.s[2] * sizeof(double);
    for (int q = 0; q < 5; ++q) {
      HIPCHK(dst, hipMemcpyAsync(ra.dP + q * ra.dnct + db.off, ra.sP + q * ra.snct + sb.off, cnt,
                                 hipMemcpyDeviceToDevice, st));
      HIPCHK(dst, hipMemcpyAsync(ra.dU + q * ra.dnct + db.off, ra.sU + q * ra.snct + sb.off, cnt,
                                 hipMemcpyDeviceToDevice, st));
    }
    for (int q = 0; q < 3; ++q)
      HIPCHK(dst, hipMemcpyAsync(ra.dBf + q * ra.dnct + db.off, ra.sBf + q * ra.snct + sb.off, cnt,
                                 hipMemcpyDeviceToDevice, st));
  }
  if (!R.cells.empty())
    hipLaunchKernelGGL(k_remap_cells, dim3((R.cells.size() + 255) / 256), dim3(256), 0, st, ra,
                       (const RemapC *)(w + R.o_cells), (int)R.cells.size());
  if (!R.faces.empty())
    hipLaunchKernelGGL(k_remap_faces, dim3((R.faces.size() + 255) / 256), dim3(256), 0, st, ra,
                       (const RemapF *)(w + R.o_faces), (int)R.faces.size());
  if (!R.parents.empty()) {
    hipLaunchKernelGGL(k_remap_div, dim3((R.parents.size() + 255) / 256), dim3(256), 0, st, ra,
                       (const RemapP *)(w + R.o_par), (int)R.parents.size(),
                       (const double *)(w + R.o_M), R.id[0], R.id[1], R.id[2]);
    // refined cells: U of the new P and field, then the parents' content
    KArgs a = dst->args();
    a.met.M = metric->M; a.met.a = metric->a;
    fill_eos(a, eos);
    if (metric->kind == GRMHD_METRIC_KS_LOGSPH)
      hipLaunchKernelGGL((k_p2c<MK_KS, 0>), dim3(Dp.ch_int.size()), dim3(256), 0, st, a,
                         dptr<int2>(dst, Dp.o_chi));
    else
      hipLaunchKernelGGL((k_p2c<MK_MINK, 0>), dim3(Dp.ch_int.size()), dim3(256), 0, st, a,
                         dptr<int2>(dst, Dp.o_chi));
    // copied and restricted cells take their U again
    if (!R.cells.empty())
      hipLaunchKernelGGL(k_remap_cells, dim3((R.cells.size() + 255) / 256), dim3(256), 0, st, ra,
                         (const RemapC *)(w + R.o_cells), (int)R.cells.size());
    for (const auto &cp : R.copies) {
      const BlockInfo &db = Dp.blocks[cp.first], &sb = Sp.blocks[cp.second];
      const size_t cnt = (size_t)db.s[0] * db.s[1] * db.s[2] * sizeof(double);
      for (int q = 0; q < 5; ++q)
        HIPCHK(dst, hipMemcpyAsync(ra.dU + q * ra.dnct + db.off, ra.sU + q * ra.snct + sb.off, cnt,
                                   hipMemcpyDeviceToDevice, st));
    }
    hipLaunchKernelGGL(k_remap_cons, dim3((R.parents.size() + 255) / 256), dim3(256), 0, st, ra,
                       (const RemapP *)(w + R.o_par), (int)R.parents.size());
  }
  LAUNCHCHK(dst);
  // the host maps must outlive their copies
  HIPCHK(dst, hipStreamSynchronize(st));
  return GRMHD_OK;
}

int grmhd_debug_ptrs(grmhd_pack *p, void **flags, void **iters, void **flux)
{
  if (!p) return GRMHD_E_INVALID;
  if (flags) *flags = p->ws + p->plan.o_flags;
  if (iters) *iters = p->ws + p->plan.o_iters;
  if (flux) *flux = p->ws + p->plan.o_F;
  return GRMHD_OK;
}

int grmhd_step(grmhd_pack *p, const grmhd_metric *m, const grmhd_eos *eos, double dt, int guess,
               double cfl)
{
  static const double rk1[3] = {1.0, 0.0, 1.0}, rk2[3] = {0.5, 0.5, 0.5};
  if (!p) return GRMHD_E_INVALID;
  // the first stage's state lives in U0 / Bf0 (no copy of the base; the fused
  // stage keeps the copying form), and the flags are cleared on every exit
  struct Reset {
    grmhd_pack *p;
    ~Reset() { p->to_base = false; p->swap = false; }
  } reset{p};
  const bool pp = !p->fused;
  int rc;
  p->to_base = pp;
  if ((rc = grmhd_stage(p, m, eos, dt, rk1))) return rc;
  p->swap = pp;
  if ((rc = grmhd_con2prim(p, m, eos, guess))) return rc;
  if ((rc = grmhd_fill_ghosts(p, m))) return rc;
  if ((rc = grmhd_stage(p, m, eos, dt, rk2))) return rc;
  p->swap = false;
  p->to_base = false;
  // the last inversion also produces the reductions (dt of the next step)
  if ((rc = con2prim_impl(p, m, eos, guess, cfl, cfl > 0.0))) return rc;
  if ((rc = grmhd_fill_ghosts(p, m))) return rc;
  return GRMHD_OK;
}

int grmhd_step_graph(grmhd_pack *p, const grmhd_metric *m, const grmhd_eos *eos, int guess,
                     double cfl, int nsteps)
{
  if (!p) return GRMHD_E_INVALID;
  if (int rc = check_metric(p, m)) return rc;
  if (int rc = check_eos(p, eos)) return rc;
  if (!(cfl > 0.0) || nsteps < 0) return perr(p, "need cfl > 0 and nsteps >= 0", GRMHD_E_INVALID);
  grmhd_eos_table tab{};
  if (eos->table) tab = *eos->table;
  const bool same = p->gexec && p->g_guess == guess && p->g_cfl == cfl &&
                    !std::memcmp(&p->g_metric, m, sizeof *m) &&
                    !std::memcmp(&p->g_eos, eos, sizeof *eos) &&
                    !std::memcmp(&p->g_tab, &tab, sizeof tab);
  // the radial floor table stays outside the graph: brought up to date here,
  // before any capture and before the replays
  if (m->kind == GRMHD_METRIC_KS_LOGSPH) {
    KArgs a = p->args();
    fill_eos(a, eos);
    floor_table(p, a, eos);
  }
  if (!same) {
    if (p->gexec) { (void)hipGraphExecDestroy(p->gexec); p->gexec = nullptr; }
    const bool prof = p->prof;
    p->prof = false;                          // no event records inside the graph
    HIPCHK(p, hipStreamBeginCapture(p->stream, hipStreamCaptureModeThreadLocal));
    p->capturing = true;
    const int rc = grmhd_step(p, m, eos, -1.0, guess, cfl);
    p->capturing = false;
    hipGraph_t g = nullptr;
    const hipError_t ec = hipStreamEndCapture(p->stream, &g);
    p->prof = prof;
    if (rc) { if (g) (void)hipGraphDestroy(g); return rc; }
    if (ec != hipSuccess) return perr(p, std::string("capture: ") + hipGetErrorString(ec), GRMHD_E_HIP);
    const hipError_t ei = hipGraphInstantiate(&p->gexec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (ei != hipSuccess) return perr(p, std::string("instantiate: ") + hipGetErrorString(ei), GRMHD_E_HIP);
    p->g_guess = guess; p->g_cfl = cfl; p->g_metric = *m; p->g_eos = *eos; p->g_tab = tab;
  }
  for (int s = 0; s < nsteps; ++s) HIPCHK(p, hipGraphLaunch(p->gexec, p->stream));
  return GRMHD_OK;
}

int grmhd_set_tiling(grmhd_pack *p, const int shape[3])
{
  if (!p || !shape) return GRMHD_E_INVALID;
  for (int d = 0; d < 3; ++d)
    if (shape[d] < 0 || shape[d] >= NSHAPE) return perr(p, "bad tile shape", GRMHD_E_INVALID);
  for (int d = 0; d < 3; ++d) p->shape[d] = shape[d];
  if (p->gexec) { (void)hipGraphExecDestroy(p->gexec); p->gexec = nullptr; }
  return GRMHD_OK;
}

int grmhd_set_persistent(grmhd_pack *p, int workgroups)
{
  if (!p || workgroups < 0) return GRMHD_E_INVALID;
  p->persist = workgroups;
  if (p->gexec) { (void)hipGraphExecDestroy(p->gexec); p->gexec = nullptr; }
  return GRMHD_OK;
}

int grmhd_set_fused(grmhd_pack *p, int enable)
{
  if (!p) return GRMHD_E_INVALID;
  if (enable && (p->plan.maxlev > 0 || p->desc.nscalar))
    return perr(p, "the fused stage needs a single-level pack without the scalar",
                GRMHD_E_UNSUPPORTED);
  p->fused = enable != 0;
  if (p->gexec) { (void)hipGraphExecDestroy(p->gexec); p->gexec = nullptr; }
  return GRMHD_OK;
}

int grmhd_set_concurrency(grmhd_pack *p, int enable)
{
  if (!p) return GRMHD_E_INVALID;
  p->concurrent = enable != 0;
  if (p->gexec) { (void)hipGraphExecDestroy(p->gexec); p->gexec = nullptr; }
  return GRMHD_OK;
}

int grmhd_get_tiling(const grmhd_pack *p, int shape[3])
{
  if (!p || !shape) return GRMHD_E_INVALID;
  for (int d = 0; d < 3; ++d) shape[d] = p->shape[d];
  return GRMHD_OK;
}

int grmhd_autotune(grmhd_pack *p, const grmhd_metric *m, const grmhd_eos *eos, int reps,
                   int chosen[3], double *ms_table)
{
  if (!p || !chosen) return GRMHD_E_INVALID;
  if (int rc = check_metric(p, m)) return rc;
  if (int rc = check_eos(p, eos)) return rc;
  if (reps < 1) reps = 1;
  KArgs a = p->args();
  a.met.M = m->M; a.met.a = m->a;
  fill_eos(a, eos);
  const int rcn = p->desc.recon, rs = p->desc.riemann, fv = p->desc.weno_fv;
  const int prec = p->desc.precision;
  const bool all = rcn == RC_WENO && fv == 0 && (!p->desc.nscalar || rs == RS_LLF);
  if (p->fused) {
    // the fused x3 tiles end in the Runge-Kutta update: timed here, it writes
    // into unused flux scratch (the x2 hydro slots) instead of U, U0
    a.U = a.F + 8 * a.nct;
    a.U0 = a.U;
    p->rk = RkArgs{1.0, nullptr, 1.0, 0.0, 1.0, 0};
  }
  hipEvent_t e0, e1;
  HIPCHK(p, hipEventCreate(&e0));
  HIPCHK(p, hipEventCreate(&e1));
  const bool prof = p->prof;
  p->prof = false;
  int status = GRMHD_OK;
  for (int d = 0; d < 3 && !status; ++d) {
    double best = 1e300;
    int bsh = 0;
    for (int sh = 0; sh < NSHAPE; ++sh) {
      double ms = -1.0;
      if (sh == 0 || all) {
        p->tune_dir = d;
        p->tune_sh = sh;
        // one untimed launch, then reps timed launches
        for (int r = 0; r <= reps; ++r) {
          if (r == 1) (void)hipEventRecord(e0, p->stream);
          if (m->kind == GRMHD_METRIC_KS_LOGSPH) launch_flux_all<MK_KS>(p, a, rcn, fv, rs, prec);
          else launch_flux_all<MK_MINK>(p, a, rcn, fv, rs, prec);
        }
        (void)hipEventRecord(e1, p->stream);
        hipError_t err = hipEventSynchronize(e1);
        float t = 0.0f;
        if (!err) err = hipEventElapsedTime(&t, e0, e1);
        if (err) { status = perr(p, std::string("autotune: ") + hipGetErrorString(err), GRMHD_E_HIP); break; }
        ms = t / reps;
        if (ms < best) { best = ms; bsh = sh; }
      }
      if (ms_table) ms_table[d * NSHAPE + sh] = ms;
    }
    chosen[d] = bsh;
  }
  p->tune_dir = -1;
  p->tune_sh = -1;
  p->prof = prof;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (status) return status;
  return grmhd_set_tiling(p, chosen);
}

int grmhd_profile(grmhd_pack *p, int enable)
{
  if (!p) return GRMHD_E_INVALID;
  HIPCHK(p, hipStreamSynchronize(p->stream));
  for (auto &r : p->ev_rec) {
    p->ev_free.push_back(std::get<1>(r));
    p->ev_free.push_back(std::get<2>(r));
  }
  p->ev_rec.clear();
  p->prof = enable != 0;
  return GRMHD_OK;
}

int grmhd_profile_read(grmhd_pack *p, double *ms, long long *count)
{
  if (!p || !ms || !count) return GRMHD_E_INVALID;
  HIPCHK(p, hipStreamSynchronize(p->stream));
  for (int f = 0; f < GRMHD_PROF_NFAM; ++f) { ms[f] = 0.0; count[f] = 0; }
  for (auto &r : p->ev_rec) {
    float t = 0.0f;
    HIPCHK(p, hipEventElapsedTime(&t, std::get<1>(r), std::get<2>(r)));
    ms[std::get<0>(r)] += t;
    count[std::get<0>(r)] += 1;
    p->ev_free.push_back(std::get<1>(r));
    p->ev_free.push_back(std::get<2>(r));
  }
  p->ev_rec.clear();
  return GRMHD_OK;
}

const char *grmhd_last_error(const grmhd_pack *p)
{
  if (p && !p->err.empty()) return p->err.c_str();
  return g_err.c_str();
}

}  // extern "C"
