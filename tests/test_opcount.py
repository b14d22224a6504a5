"""The algorithmic flop counts behind the benchmark's roofline: the counter
(the device math header compiled for the host with a counting scalar) still
builds against the current kernels' math and reproduces the committed table,
and the per-face figures are the sums they claim to be."""
import importlib.util
import json
import os

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HERE = os.path.join(ROOT, "paper_2410_09146_amd", "opcount")


def _counter():
    spec = importlib.util.spec_from_file_location("opcount_count", os.path.join(HERE, "count.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_table_is_reproduced():
    fresh = _counter().count(write=False)
    committed = json.load(open(os.path.join(HERE, "opcount.json")))
    assert fresh == committed


def test_per_face_figures_add_up():
    t = json.load(open(os.path.join(HERE, "opcount.json")))
    f = {k: v["flops"] for k, v in t.items() if isinstance(v, dict)}
    assert t["per_face_flux_ks_weno_llf"] == 7 * f["recon_weno5z_aoah"] + f["geo_ks"] + f["riemann_llf"]
    for rc in ("weno5z_aoah", "mp5", "plm_mc", "plm_minmod", "const"):
        for rs in ("llf", "hll"):
            assert t[f"per_face_flux_ks_{rc}_{rs}"] == 7 * f[f"recon_{rc}"] + f["geo_ks"] + f[f"riemann_{rs}"]
    assert f["recon_const"] == 0
    # WENO5-Z-AOAH is the costliest reconstruction
    assert max(f[f"recon_{rc}"] for rc in ("mp5", "plm_mc", "plm_minmod")) < f["recon_weno5z_aoah"]
