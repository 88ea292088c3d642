"""Workload parameters for the PSFD solve (plain numbers, no solver arithmetic).

A configuration is a plain ``dict`` whose keys mirror the fields of the C
plan descriptor ``psfd_desc`` in ``include/psfd.h``.  Lengths are in nm,
angles in radians.

Physical setting (paper, Results section, opening paragraph): EUV
wavelength 13.5 nm, a Mo/Si Bragg reflector of 40 bilayers with a 7 nm
period under the absorber.  The paper does not print the optical constants
of Mo and Si; the values below are an assumption recorded here and used
identically by every consumer (they only set the numbers the multilayer
reflection takes, not the structure of the method).
"""

import math

LAMBDA_NM = 13.5
# Assumed complex refractive indices at 13.5 nm (not printed in the paper).
N_MO = complex(0.921, 0.0064)
N_SI = complex(0.999, 0.0018)
ML_BILAYERS = 40
T_SI = 4.2  # nm, Si on top of each bilayer (Gamma = 0.4)
T_MO = 2.8  # nm
# Absorber permittivity used by every synthetic workload: (0.94 + 0.04 i)^2.
ABSORBER_N = complex(0.94, 0.04)


def eps_absorber_default():
    return ABSORBER_N * ABSORBER_N


def multilayer_stack(n_bilayers=ML_BILAYERS):
    """Layer permittivities and thicknesses, top to bottom, plus the substrate."""
    eps_si = N_SI * N_SI
    eps_mo = N_MO * N_MO
    ml_eps, ml_thick = [], []
    for _ in range(n_bilayers):
        ml_eps += [eps_si, eps_mo]
        ml_thick += [T_SI, T_MO]
    return ml_eps, ml_thick, eps_si


def nz_total(cfg):
    return cfg["nz_abs"] + cfg["nz_gap_bot"] + cfg["nz_gap_top"] + 2 * cfg["nz_pml"]


def base_config(nx, ny, nz_abs, t_abs, dx=2.0, dy=None, theta_deg=6.0, phi_deg=0.0,
                pol=0, precond=1, nz_pml=6, nz_gap=2, multilayer=True):
    """One solve's parameters.  ``pol``: 0 = TE, 1 = TM."""
    ml_eps, ml_thick, eps_sub = multilayer_stack() if multilayer else ([], [], 1.0 + 0j)
    return {
        "nx": int(nx), "ny": int(ny), "nz_abs": int(nz_abs),
        "nz_gap_bot": int(nz_gap), "nz_gap_top": int(nz_gap), "nz_pml": int(nz_pml),
        "dx": float(dx), "dy": float(dx if dy is None else dy), "dz": float(t_abs) / nz_abs,
        "lam": LAMBDA_NM,
        "theta": math.radians(theta_deg), "phi": math.radians(phi_deg), "pol": int(pol),
        "eps_bg": 1.0,
        "ml_eps": list(ml_eps), "ml_thick": list(ml_thick), "eps_sub": complex(eps_sub),
        "pml_sigma0": 6.0, "pml_order": 3,
        "precond": int(precond),
        "pc_mmin": 0.0, "pc_kref": 0.0, "pc_gamma": 1.0, "pc_reg": 0.0,
        "smooth_sigma": 1.0,
        "ml_kz_min": 0.0,
    }


def config_c1(pol=0):
    """32 x 32 lateral, 2 nm pitch; 16 absorber cells over 30 nm; 6 deg, TE."""
    return base_config(32, 32, 16, 30.0, pol=pol)


def config_c2(pol=0):
    """256 x 256 lateral, 2 nm pitch; 32 absorber cells over 60 nm; 6 deg."""
    return base_config(256, 256, 32, 60.0, pol=pol)


def config_c3_sizes():
    """Lateral sizes, incidence angles (deg) and polarisations of the batched workload."""
    return [64, 128, 192, 256], [0.0, 2.5, 5.0, 7.5, 10.0], [0, 1]


def config_c4(pol=0):
    """1024 x 1024 lateral, 2 nm pitch; 48 absorber cells over 70 nm; 6 deg."""
    return base_config(1024, 1024, 48, 70.0, pol=pol)


def config_c5():
    """128 x 128 lateral, 2 nm pitch; 32 absorber cells over 60 nm; 6 deg, TE."""
    return base_config(128, 128, 32, 60.0, pol=0)


# Standard full-domain comparison (paper, Results, "Background-decomposition"
# paragraph): the bare multilayer discretised on the grid.  Axial sizes per
# grid step: stack rows plus a 12 nm PML on each side and equal gaps, padded
# to a length the axial transforms take.
FULL_DOMAIN_NZ = {1.0: 324, 0.5: 648, 0.25: 1296}
# Incidence angles the paper's 150 nm periodic cell represents below 20 deg:
# sin(theta_m) = m lambda / 150 nm.
FULL_DOMAIN_THETAS_DEG = [math.degrees(math.asin(m * LAMBDA_NM / 150.0)) for m in range(4)]


def full_domain_config(dz, theta_deg=0.0, pol=0, nx=1, n_bilayers=ML_BILAYERS, nz=None,
                       pml_nm=12.0):
    """Configuration of a full-domain solve of the bare stack (no multilayer
    operator; the stack goes into the absorber rows, see ``full_domain_stack``).

    ``nz`` defaults to FULL_DOMAIN_NZ[dz]; lateral size nx x nx with pitch dz."""
    _, thick, _ = multilayer_stack(n_bilayers)
    nz_abs = int(math.ceil(round(sum(thick) / dz, 9)))
    nz = FULL_DOMAIN_NZ[dz] if nz is None else int(nz)
    npml = int(round(pml_nm / dz))
    gaps = nz - nz_abs - 2 * npml
    if gaps < 2:
        raise ValueError("axial size too small for the stack and the PML")
    cfg = base_config(nx, nx, nz_abs, nz_abs * dz, dx=dz, theta_deg=theta_deg, pol=pol,
                      nz_pml=npml, nz_gap=gaps // 2, multilayer=False)
    cfg["nz_gap_top"] = gaps - gaps // 2
    return cfg


def full_domain_stack(n_bilayers=ML_BILAYERS):
    """(layer permittivities, thicknesses) of the bare stack, top to bottom."""
    eps, thick, _ = multilayer_stack(n_bilayers)
    return eps, thick


# Factorised Fourier neural operator (paper, section 2.1): sizes and seeded
# random weights (no trained weights exist here).  The flat weight layout is
# documented with psfd_ffno_forward in include/psfd.h.
def ffno_desc(nx, ny, nz, d_v=32, d_h=64, n_layers=4, kx_max=12, ky_max=12, kz_max=8):
    return {"nx": int(nx), "ny": int(ny), "nz": int(nz), "d_v": int(d_v), "d_h": int(d_h),
            "n_layers": int(n_layers), "kx_max": int(kx_max), "ky_max": int(ky_max),
            "kz_max": int(kz_max)}


def ffno_weight_blocks(desc):
    """(name, element count, init scale) of every weight block, in storage order."""
    dv, dh = desc["d_v"], desc["d_h"]
    my, mx, mz = 2 * desc["ky_max"] + 1, desc["kx_max"] + 1, desc["kz_max"] + 1
    blocks = [("P", dv * 4, 0.5), ("p", dv, 0.1)]
    for _ in range(desc["n_layers"]):
        blocks += [("Kxy", dv * dv * my * mx * 2, 1.0 / dv), ("Kz", dv * dv * mz * 2, 1.0 / dv),
                   ("W1", dh * dv, 1.0 / math.sqrt(dv)), ("b1", dh, 0.1),
                   ("W2", dv * dh, 1.0 / math.sqrt(dh)), ("b2", dv, 0.1)]
    blocks += [("Q", 6 * dv, 1.0 / math.sqrt(dv)), ("q", 6, 0.0)]
    return blocks


def ffno_weights(desc, seed):
    """Seeded Gaussian weights, each block scaled by its init scale (float32 values)."""
    import numpy as np
    rng = np.random.default_rng(seed)
    parts = [rng.standard_normal(n) * s for _, n, s in ffno_weight_blocks(desc)]
    return np.concatenate(parts).astype(np.float32)
