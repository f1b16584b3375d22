"""Seeded synthetic inputs shaped like the paper's workloads.

This module only builds inputs (geometry descriptions, gas fields, source and
output settings, request streams).  It holds none of the method's arithmetic
(no line constants, cross-sections or transport): both the oracle and the
HIP path receive the same dicts and arrays from here and derive everything
else themselves.

Workloads (the paper's datasets are not available; these stand in for them):
  sphere   static homogeneous sphere, line-centre radial tau0 = 1e5, T = 1e4 K,
           500 packets from the centre at x = 0 (the Neufeld-type validation
           test of Section 4)
  shell    expanding shell on a 128^3 grid with dust and one peel observer
           (the shell models of Sections 4 and 5.1)
  web      cosmic-web box, log-normal n_HI Gaussian random field on N^3
           (one rank's share of the weak-scaling runs of Section 6.3)
  serving  stream of meshless shell-model solves (the parameter grid of
           Section 5.1)
  forest   Lyman-alpha absorption sightlines through the web box at z = 2
           (the forest and tomography example of Section 5.5)
"""
from __future__ import annotations

import numpy as np

KPC = 3.0856775814913673e21   # cm
KMS = 1.0e5                   # cm/s


# --------------------------------------------------------------------------
# sphere: static homogeneous sphere
# --------------------------------------------------------------------------
def sphere(tau0: float = 1e5, T: float = 1e4, n_packets: int = 500, seed: int = 1,
           kind: str = "sphere", phase: str = "iso"):
    geom = dict(kind=kind, r_inner=0.0, r_outer=1.0, tau0=tau0, T=T)
    src = dict(kind="point", pos=(0.0, 0.0, 0.0), spectrum="delta", dv0=0.0, seed=seed)
    opts = dict(phase=phase, spectrum=dict(nb=200, lo=-40.0, hi=40.0, T_ref=1e4))
    return dict(name="sphere", geom=geom, src=src, opts=opts, n_packets=n_packets)


# --------------------------------------------------------------------------
# shell: expanding shell on a uniform Cartesian grid
# --------------------------------------------------------------------------
def shell_fields(n: int = 128, r_in: float = 0.8, r_out: float = 1.0, N_HI: float = 1e19,
                 v_exp_kms: float = 200.0, T: float = 1e4):
    """Fields on [-1, 1]^3 (box units of 1 kpc); a cell is shell gas when its
    centre radius lies in [r_in, r_out].  Returns float32 arrays [z][y][x]."""
    c = (np.arange(n, dtype=np.float64) + 0.5) * (2.0 / n) - 1.0
    zz, yy, xx = np.meshgrid(c, c, c, indexing="ij")
    r = np.sqrt(xx * xx + yy * yy + zz * zz)
    inside = (r >= r_in) & (r <= r_out)
    n_shell = N_HI / ((r_out - r_in) * KPC)
    dens = np.where(inside, n_shell, 0.0).astype(np.float32)
    temp = np.full((n, n, n), T, dtype=np.float32)
    rs = np.where(r > 0, r, 1.0)
    v = v_exp_kms * KMS
    vx = np.where(inside, v * xx / rs, 0.0).astype(np.float32)
    vy = np.where(inside, v * yy / rs, 0.0).astype(np.float32)
    vz = np.where(inside, v * zz / rs, 0.0).astype(np.float32)
    return dens, temp, vx, vy, vz


def shell(n_grid: int = 128, n_packets: int = 1_000_000, seed: int = 2, cube_nb: int = 256,
          tau_d: float = 0.5, N_HI: float = 1e19, albedo: float = 0.3):
    dens, temp, vx, vy, vz = shell_fields(n_grid, N_HI=N_HI)
    geom = dict(kind="grid", lo=(-KPC, -KPC, -KPC), hi=(KPC, KPC, KPC),
                n_HI_field=dens, T_field=temp, vx=vx, vy=vy, vz=vz,
                sigma_d=tau_d / N_HI, albedo=albedo, g_hg=0.73)
    src = dict(kind="point", pos=(0.0, 0.0, 0.0), spectrum="gauss", dv0=0.0,
               sigma_v=20.0 * KMS, seed=seed)
    vlo, vhi = -1500.0 * KMS, 1500.0 * KMS
    opts = dict(phase="dipole", observers=["+z"],
                cube=dict(nx=n_grid, ny=n_grid, nb=cube_nb, img_lo=(-KPC, -KPC),
                          img_hi=(KPC, KPC), v_lo=vlo, v_hi=vhi),
                spectrum=dict(nb=256, lo=vlo, hi=vhi), tau_cut=40.0)
    return dict(name="shell", geom=geom, src=src, opts=opts, n_packets=n_packets)


# --------------------------------------------------------------------------
# web: cosmic-web box with Gaussian-random-field fields
# --------------------------------------------------------------------------
def grf(n: int, slope: float, rng: np.random.Generator, dtype=np.float32):
    """Periodic Gaussian random field on n^3 with P(k) ~ k^slope (k in units of
    the fundamental mode, P(0) = 0), normalised to zero mean and unit sample
    standard deviation."""
    import scipy.fft as sfft
    white = rng.standard_normal((n, n, n), dtype=np.float32)
    fk = sfft.rfftn(white, workers=-1)
    del white
    kx = np.fft.fftfreq(n, d=1.0 / n).astype(np.float32)
    kz = np.fft.rfftfreq(n, d=1.0 / n).astype(np.float32)
    for i in range(n):   # slab by slab keeps the temporary small
        k2 = kx[i] ** 2 + kx[:, None] ** 2 + kz[None, :] ** 2
        with np.errstate(divide="ignore"):
            amp = np.where(k2 > 0, k2 ** (slope / 4.0), 0.0).astype(np.float32)
        fk[i] *= amp
    field = sfft.irfftn(fk, s=(n, n, n), workers=-1).astype(dtype, copy=False)
    del fk
    field -= field.mean(dtype=np.float64)
    field /= field.std(dtype=np.float64)
    return field


def web_fields(n: int = 1024, sigma_ln: float = 2.0, n_mean: float = 1e-5, slope: float = -2.5,
               sigma_v_kms: float = 100.0, T0: float = 1e4, entropy: int = 2507_11603):
    seqs = np.random.SeedSequence(entropy).spawn(4)
    delta = grf(n, slope, np.random.default_rng(seqs[0]))
    delta *= np.float32(sigma_ln)
    dens = np.exp(delta, dtype=np.float32)
    del delta
    dens *= np.float32(n_mean / dens.mean(dtype=np.float64))
    temp = (np.float32(T0) * np.sqrt(dens / np.float32(n_mean))).astype(np.float32)
    vel = []
    for s in seqs[1:]:
        v = grf(n, slope, np.random.default_rng(s))
        v *= np.float32(sigma_v_kms * KMS)
        vel.append(v)
    return dens, temp, vel[0], vel[1], vel[2]


def grf_torch(n: int, slope: float, seed: int, device="cuda"):
    """Same recipe as `grf` on a HIP device with torch (float32), for the large
    grids; returns a device tensor [z][y][x]."""
    import torch
    g = torch.Generator(device=device)
    g.manual_seed(seed)
    white = torch.randn((n, n, n), generator=g, device=device, dtype=torch.float32)
    fk = torch.fft.rfftn(white)
    del white
    kx = torch.fft.fftfreq(n, d=1.0 / n, device=device, dtype=torch.float32)
    kz = torch.fft.rfftfreq(n, d=1.0 / n, device=device, dtype=torch.float32)
    for i in range(n):   # slab by slab keeps the temporary small
        k2 = kx[i] ** 2 + kx[:, None] ** 2 + kz[None, :] ** 2
        amp = torch.where(k2 > 0, k2.clamp_min(1e-30) ** (slope / 4.0), torch.zeros_like(k2))
        fk[i] *= amp
    field = torch.fft.irfftn(fk, s=(n, n, n))
    del fk
    field -= field.mean(dtype=torch.float64).float()
    field /= field.std().float()
    return field


def web_fields_torch(n: int = 1024, sigma_ln: float = 2.0, n_mean: float = 1e-5, slope: float = -2.5,
                     sigma_v_kms: float = 100.0, T0: float = 1e4, entropy: int = 2507_11603, device="cuda"):
    """Device-tensor version of `web_fields` (different random stream, same
    statistics); used for the 512^3 and 1024^3 boxes."""
    import torch
    seeds = [int(s.generate_state(1)[0]) for s in np.random.SeedSequence(entropy).spawn(4)]
    dens = grf_torch(n, slope, seeds[0], device)
    dens.mul_(sigma_ln).exp_()
    dens.mul_(n_mean / dens.mean(dtype=torch.float64).item())
    temp = torch.sqrt(dens / n_mean).mul_(T0)
    vel = [grf_torch(n, slope, s, device).mul_(sigma_v_kms * KMS) for s in seeds[1:]]
    return dens, temp, vel[0], vel[1], vel[2]


def forest_fields(n: int = 512, n_mean: float = 2e-11, entropy: int = 2507_11603):
    """n_HI, T and v_z of the web box: the same random fields as
    `web_fields(n)` (density and z velocity streams), with the neutral density
    rescaled to a forest-like mean (the Gunn-Peterson depth of the mean is
    then about 0.4 at z = 2)."""
    seqs = np.random.SeedSequence(entropy).spawn(4)
    delta = grf(n, -2.5, np.random.default_rng(seqs[0]))
    delta *= np.float32(2.0)
    dens = np.exp(delta, dtype=np.float32)
    del delta
    dens *= np.float32(n_mean / dens.mean(dtype=np.float64))
    temp = (np.float32(1e4) * np.sqrt(dens / np.float32(n_mean))).astype(np.float32)
    vz = grf(n, -2.5, np.random.default_rng(seqs[3]))
    vz *= np.float32(100.0 * KMS)
    return dens, temp, vz


def forest_fields_torch(n: int = 512, n_mean: float = 2e-11, entropy: int = 2507_11603, device="cuda"):
    """Device-tensor version of `forest_fields` (the torch streams of
    `web_fields_torch`: different numbers, same statistics)."""
    import torch
    seeds = [int(s.generate_state(1)[0]) for s in np.random.SeedSequence(entropy).spawn(4)]
    dens = grf_torch(n, -2.5, seeds[0], device)
    dens.mul_(2.0).exp_()
    dens.mul_(n_mean / dens.mean(dtype=torch.float64).item())
    temp = torch.sqrt(dens / n_mean).mul_(1e4)
    vz = grf_torch(n, -2.5, seeds[3], device).mul_(100.0 * KMS)
    return dens, temp, vz


_FOREST_CACHE = {}


def forest(n_grid: int = 512, box_pmpc: float = 17.22, hubble_kms_mpc: float = 203.6,
           n_sub: int = 4, nb: int = 2048, device=None):
    """Absorption spectra along z through the web box at z = 2 (box 17.22
    proper Mpc, H(z = 2) = 203.6 km/s/Mpc for a flat Omega_m = 0.309
    cosmology): one tomography plane of n_grid rays (all x at y = n_grid/2),
    n_sub steps per cell (H ds / n_sub = 1.7 km/s at 512^3, well below the
    12.8 km/s thermal speed at 1e4 K), nb bins over -500 .. 4000 km/s (the
    Hubble span of the box is 3505 km/s).  Host fields are cached per size;
    device="cuda" builds device tensors instead (not cached)."""
    if device is not None:
        fields = forest_fields_torch(n_grid, device=device)
    else:
        if n_grid not in _FOREST_CACHE:
            _FOREST_CACHE[n_grid] = forest_fields(n_grid)
        fields = _FOREST_CACHE[n_grid]
    L = box_pmpc * 1e3 * KPC
    H = hubble_kms_mpc * KMS / (1e3 * KPC)
    opts = dict(axis=2, ds=L / n_grid, hubble=H, n_sub=n_sub, rays=(0, n_grid, n_grid // 2, 1),
                nb=nb, u_lo=-500.0 * KMS, u_hi=4000.0 * KMS)
    return {"fields": fields, "opts": opts}


def web(n_grid: int = 1024, n_packets: int = 100_000_000, seed: int = 3, box_pmpc: float = 17.22,
        fields=None, cube_npix: int = 512, cube_nb: int = 200, x_crit: float = 3.0, hubble_kms_mpc: float = 0.0,
        stop_kms: float = 1233.0):
    L = box_pmpc * 1e3 * KPC
    if fields is None:
        fields = web_fields(n_grid)
    dens, temp, vx, vy, vz = fields
    geom = dict(kind="grid", lo=(0.0, 0.0, 0.0), hi=(L, L, L), n_HI_field=dens, T_field=temp,
                vx=vx, vy=vy, vz=vz, boundary_handoff=1, sigma_d=0.0, albedo=0.0, g_hg=0.73)
    if hubble_kms_mpc > 0.0:
        # expansion about the box centre; packets stop once 5 A (1233 km/s) to the red
        geom.update(hubble=hubble_kms_mpc * KMS / (1e3 * KPC), hubble_ref=(L / 2, L / 2, L / 2), hubble_step=0.1,
                    stop_dv=stop_kms * KMS)
    src = dict(kind="cell_n2", spectrum="thermal", dv0=0.0, seed=seed)
    vlo, vhi = -1500.0 * KMS, 1500.0 * KMS
    opts = dict(phase="dipole", core_skip="fixed", x_crit=x_crit, observers=["+x", "+y", "+z"],
                cube=dict(nx=cube_npix, ny=cube_npix, nb=cube_nb, img_lo=(0.0, 0.0),
                          img_hi=(L, L), v_lo=vlo, v_hi=vhi),
                spectrum=dict(nb=200, lo=vlo, hi=vhi), tau_cut=40.0)
    return dict(name="web", geom=geom, src=src, opts=opts, n_packets=n_packets)


# --------------------------------------------------------------------------
# validation media of Section 4: dusty slab, sphere with a linear outflow
# --------------------------------------------------------------------------
def dusty_slab(tau0: float = 1e6, T: float = 20.0, tau_d: float = 0.1, n_packets: int = 1000, seed: int = 1,
               albedo: float = 0.0):
    """Infinite slab |z| < Z: line-centre optical depth tau0 and dust optical
    depth tau_d from the mid-plane to a surface, line-centre source at the
    centre, isotropic phase; albedo 0 makes the dust a pure absorber."""
    geom = dict(kind="slab", r_inner=0.0, r_outer=KPC, tau0=tau0, T=T, tau_d=tau_d, albedo=albedo, g_hg=0.73)
    src = dict(kind="point", pos=(0.0, 0.0, 0.0), spectrum="delta", dv0=0.0, seed=seed)
    opts = dict(phase="iso", spectrum=dict(nb=200, lo=-40.0, hi=40.0, T_ref=T))
    return dict(name="dusty_slab", geom=geom, src=src, opts=opts, n_packets=n_packets)


def outflow_sphere(N_HI: float = 2e18, T: float = 2e4, v_max_kms: float = 200.0, n_packets: int = 1000,
                   seed: int = 1, nb: int = 200, v_range_kms: float = 1000.0):
    """Homogeneous sphere of column N_HI (centre to edge) at T with the
    linear velocity profile v = v_max r / R (outflow for v_max > 0), line-centre
    source at the centre, dipole phase; spectrum of dv over +-v_range."""
    R = KPC
    geom = dict(kind="sphere", r_inner=0.0, r_outer=R, n_HI=N_HI / R, T=T, v_profile="linear",
                v_max=v_max_kms * KMS, step_f=0.01)
    src = dict(kind="point", pos=(0.0, 0.0, 0.0), spectrum="delta", dv0=0.0, seed=seed)
    opts = dict(phase="dipole", spectrum=dict(nb=nb, lo=-v_range_kms * KMS, hi=v_range_kms * KMS))
    return dict(name="outflow_sphere", geom=geom, src=src, opts=opts, n_packets=n_packets)


def mg2_sphere(log_N: float = 14.5, T: float = 1e4, v_max_kms: float = 500.0, n_packets: int = 10000,
               seed: int = 1, continuum_kms=(-1500.0, 1000.0), step_f: float = 0.05, line: str = "mg2",
               spectrum: str = "flat", dv0_kms: float = 0.0, nb: int = 250):
    """Section 4's doublet test: a homogeneous sphere of Mg II column 10^log_N
    (centre to edge) at T with the linear outflow v = v_max r/R, a central
    source of a flat continuum over `continuum_kms` (relative to the k line;
    `spectrum="delta"` emits at dv0 instead), dipole phase in the k line
    (isotropic in h); escape spectrum over the continuum's range."""
    R = KPC
    lo, hi = continuum_kms
    geom = dict(kind="sphere", r_inner=0.0, r_outer=R, n_HI=10.0 ** log_N / R, T=T, line=line,
                v_profile="linear" if v_max_kms else "none", v_max=v_max_kms * KMS, step_f=step_f)
    if spectrum == "flat":
        src = dict(kind="point", pos=(0.0, 0.0, 0.0), spectrum="flat", dv0=0.5 * (lo + hi) * KMS,
                   sigma_v=0.5 * (hi - lo) * KMS, seed=seed)
    else:
        src = dict(kind="point", pos=(0.0, 0.0, 0.0), spectrum="delta", dv0=dv0_kms * KMS, seed=seed)
    opts = dict(phase="dipole", spectrum=dict(nb=nb, lo=lo * KMS, hi=hi * KMS))
    return dict(name="mg2_sphere", geom=geom, src=src, opts=opts, n_packets=n_packets)


def hubble_box(n_grid: int = 32, box_mpc: float = 30.0, n_HI: float = 4.8e-11, T: float = 1e4,
               hubble_kms_mpc: float = 100.0, stop_kms: float = 1233.0, n_packets: int = 1000, seed: int = 1,
               observers=("+z",), cube_npix: int = 1, cube_v_kms: float = 0.01):
    """Uniform static gas (no peculiar velocity) on a grid in a Hubble flow
    centred on the box, a line-centre source at the centre, the redshift stop
    at stop_kms; the +z peel cube is one pixel over the box face and one
    narrow bin around dv = 0 (it then holds the emission rays)."""
    L = box_mpc * 1e3 * KPC
    shape = (n_grid,) * 3
    dens = np.full(shape, n_HI, np.float32)
    temp = np.full(shape, T, np.float32)
    zero = np.zeros(shape, np.float32)
    H = hubble_kms_mpc * KMS / (1e3 * KPC)
    geom = dict(kind="grid", lo=(0.0, 0.0, 0.0), hi=(L, L, L), n_HI_field=dens, T_field=temp, vx=zero, vy=zero,
                vz=zero, boundary_handoff=1, sigma_d=0.0, albedo=0.0, g_hg=0.73, hubble=H,
                hubble_ref=(L / 2, L / 2, L / 2), hubble_step=0.1, stop_dv=stop_kms * KMS)
    src = dict(kind="point", pos=(L / 2, L / 2, L / 2), spectrum="delta", dv0=0.0, seed=seed)
    opts = dict(phase="dipole", observers=list(observers),
                cube=dict(nx=cube_npix, ny=cube_npix, nb=1, img_lo=(0.0, 0.0), img_hi=(L, L),
                          v_lo=-0.5 * cube_v_kms * KMS, v_hi=0.5 * cube_v_kms * KMS),
                spectrum=dict(nb=200, lo=-2000.0 * KMS, hi=2000.0 * KMS))
    return dict(name="hubble_box", geom=geom, src=src, opts=opts, n_packets=n_packets)


# --------------------------------------------------------------------------
# serving: stream of meshless shell-model requests
# --------------------------------------------------------------------------
def shell_request(N_HI: float, v_exp_kms: float, tau_d: float, n_packets: int,
                  request_id: int, T: float = 1e4, seed: int = 5):
    """One shell-model solve: homogeneous shell r in [0.8, 1.0] kpc with constant
    radial expansion, central Gaussian source (sigma 20 km/s), dipole phase,
    albedo 0.3, adaptive core skipping, 400-bin spectrum over +-2500 km/s."""
    r_in, r_out = 0.8 * KPC, 1.0 * KPC
    geom = dict(kind="shell", r_inner=r_in, r_outer=r_out, n_HI=N_HI / (r_out - r_in), T=T,
                v_profile="const_radial", v_max=v_exp_kms * KMS, step_f=0.01,
                tau_d=tau_d, albedo=0.3, g_hg=0.73)
    src = dict(kind="point", pos=(0.0, 0.0, 0.0), spectrum="gauss", dv0=0.0,
               sigma_v=20.0 * KMS, seed=seed, request_id=request_id)
    opts = dict(phase="dipole", core_skip="adaptive",
                spectrum=dict(nb=400, lo=-2500.0 * KMS, hi=2500.0 * KMS))
    return dict(name="shell_request", geom=geom, src=src, opts=opts, n_packets=n_packets)


def request_stream(n_requests: int = 4500, rate_hz: float = 200.0, entropy: int = 2507_4,
                   logN=(17.0, 21.0), vexp=(0.0, 500.0), taud=(0.0, 2.0), logn_pk=(3.0, 5.0)):
    """Open-loop Poisson arrivals; per request log N_HI ~ U[17, 21],
    v_exp ~ U[0, 500] km/s, tau_d ~ U[0, 2], packets = round(10^U[3, 5])."""
    rng = np.random.default_rng(np.random.SeedSequence(entropy))
    gaps = rng.exponential(1.0 / rate_hz, n_requests)
    t = np.cumsum(gaps) - gaps[0]
    out = []
    for i in range(n_requests):
        out.append(dict(t_arrival=float(t[i]), request_id=i,
                        N_HI=float(10 ** rng.uniform(*logN)),
                        v_exp_kms=float(rng.uniform(*vexp)),
                        tau_d=float(rng.uniform(*taud)),
                        n_packets=int(round(10 ** rng.uniform(*logn_pk)))))
    return out
