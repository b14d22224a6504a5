"""Compile and run the operation counter; write opcount.json beside it.

The per-face flop figure of the flux kernels (the dominant kernels) is
  7 reconstructions of a cell + one face metric + one Riemann solve,
the per-cell figure of the update kernel is the flux divergence, the
edge-averaged EMF curl and the Runge-Kutta combination (written out below,
they are plain sums and products) plus the Kerr-Schild source terms.
"""
import json
import os
import subprocess
import tempfile

HERE = os.path.dirname(os.path.abspath(__file__))
OUT = os.path.join(HERE, "opcount.json")

# k_update arithmetic per interior cell outside dev.h:
#   divergence: 5 vars x (3 differences, 3 scalings, 2 sums)          = 40
#   CT: 3 faces x (4 EMFs x (3 adds + 1 scale) + 2 diffs + 2 scalings + 1 sum) = 63
#   RK combination: 8 vars x (3 products + 2 sums)                      = 40
UPDATE_LOCAL = 40 + 63 + 40


def count(write=True):
    exe = os.path.join(tempfile.mkdtemp(), "opcount")
    subprocess.run(["g++", "-std=c++17", "-O0", "-I", os.path.join(HERE, "shim"),
                    os.path.join(HERE, "opcount.cpp"), "-o", exe], check=True)
    res = json.loads(subprocess.run([exe], check=True, capture_output=True, text=True).stdout)
    f = {k: v["flops"] for k, v in res.items()}
    res["per_face_flux_ks_weno_llf"] = 7 * f["recon_weno5z_aoah"] + f["geo_ks"] + f["riemann_llf"]
    # every reconstruction x Riemann solver on the Kerr-Schild face
    for rc in ("weno5z_aoah", "mp5", "plm_mc", "plm_minmod", "const"):
        for rs in ("llf", "hll"):
            res[f"per_face_flux_ks_{rc}_{rs}"] = 7 * f[f"recon_{rc}"] + f["geo_ks"] + f[f"riemann_{rs}"]
    res["per_face_flux_mink_plm_hll"] = 7 * f["recon_plm_mc"] + f["riemann_hll_minkowski"]
    res["per_cell_update_ks"] = UPDATE_LOCAL + f["geo_ks"] + f["aux_of"] + f["sources_ks"]
    res["per_cell_update_local"] = UPDATE_LOCAL
    if write:
        with open(OUT, "w") as fh:
            json.dump(res, fh, indent=1, sort_keys=True)
    return res


if __name__ == "__main__":
    r = count()
    print(json.dumps({k: r[k] for k in r if k.startswith("per_")}, indent=1))
