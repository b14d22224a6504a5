// Source-level FP64 operation counts of the stage's device math (dev.h
// compiled unmodified with a counting scalar).  add/sub, mul, div and sqrt
// count one flop each, fma two; comparisons and min/max are tallied apart.
#include <hip/hip_runtime.h>
#include "../csrc/dev.h"
#undef double

#include <cstdio>

OpCount g_ops;
using namespace grmhd;

static OpCount snap() { OpCount o = g_ops; g_ops = OpCount(); return o; }
static long long flops(const OpCount &o) { return o.add + o.mul + o.div + o.sqrt + 2 * o.fma; }
static void emit(const char *name, const OpCount &o, bool last = false)
{
  std::printf("  \"%s\": {\"flops\": %lld, \"add\": %lld, \"mul\": %lld, \"div\": %lld, "
              "\"fma\": %lld, \"sqrt\": %lld, \"cmp\": %lld}%s\n",
              name, flops(o), o.add, o.mul, o.div, o.fma, o.sqrt, o.cmp, last ? "" : ",");
}

int main()
{
  const MetricP m{cd(1.0), cd(0.9375)};
  const cd gam(13.0 / 9.0);
  // a torus-interior point and two nearby states
  snap();
  const Geo G = geo_ks(cd(12.0), cd(0.93), cd(0.37), m);
  const OpCount o_geo = snap();
  Prim L{cd(0.8), cd(0.01), cd(0.002), cd(0.02), cd(0.01), cd(0.001), cd(0.0005), cd(0.0)};
  Prim R{cd(0.75), cd(0.012), cd(0.001), cd(0.021), cd(0.011), cd(0.001), cd(0.0004), cd(0.0)};
  cd out[8];
  snap();
  riemann<0, RS_LLF>(G, gam, L, R, out);
  const OpCount o_llf = snap();
  riemann<0, RS_HLL>(G, gam, L, R, out);
  const OpCount o_hll = snap();
  cd l, r;
  // smooth non-extremal stencil: every branch of the limiter takes its full path
  recon5<RC_WENO, 0>(cd(1.0), cd(1.1), cd(1.25), cd(1.45), cd(1.7), l, r);
  const OpCount o_weno = snap();
  recon5<RC_PLM_MC, 0>(cd(1.0), cd(1.1), cd(1.25), cd(1.45), cd(1.7), l, r);
  const OpCount o_mc = snap();
  recon5<RC_PLM_MINMOD, 0>(cd(1.0), cd(1.1), cd(1.25), cd(1.45), cd(1.7), l, r);
  const OpCount o_mm = snap();
  // MP5 on the same smooth stencil: both faces keep the unlimited value (the
  // common path; the limiter's extra work is counted nowhere)
  recon5<RC_MP5, 0>(cd(1.0), cd(1.1), cd(1.25), cd(1.45), cd(1.7), l, r);
  const OpCount o_mp5 = snap();
  recon5<RC_CONST, 0>(cd(1.0), cd(1.1), cd(1.25), cd(1.45), cd(1.7), l, r);
  const OpCount o_const = snap();
  const Aux A = aux_of(G, gam, L);
  const OpCount o_aux = snap();
  const Sym4 T = tmunu(G, A);
  cd S1, S2, St;
  ks_sources(cd(12.0), cd(0.93), cd(0.37), m, G, T, S1, S2, St);
  const OpCount o_src = snap();
  C2P c{cd(0.05), cd(0.01), cd(0.001), cd(0.0002), gam, cd(0.01 / 1.01)};
  cd df;
  master(c, cd(0.9), df);
  const OpCount o_master = snap();
  const Geo Gm = geo_mink();
  (void)Gm;
  riemann<0, RS_HLL>(geo_mink(), cd(4.0 / 3.0), L, R, out);
  const OpCount o_hll_mink = snap();
  std::printf("{\n");
  emit("geo_ks", o_geo);
  emit("riemann_llf", o_llf);
  emit("riemann_hll", o_hll);
  emit("riemann_hll_minkowski", o_hll_mink);
  emit("recon_weno5z_aoah", o_weno);
  emit("recon_plm_mc", o_mc);
  emit("recon_plm_minmod", o_mm);
  emit("recon_mp5", o_mp5);
  emit("recon_const", o_const);
  emit("aux_of", o_aux);
  emit("sources_ks", o_src);
  emit("master_iteration", o_master, true);
  std::printf("}\n");
  return 0;
}
