"""Gaussian random field on a periodic box (oracle, FP64).

Follows section "Mock generation" and eq:deltaL, eq:eta of the paper:

* the noise is drawn directly in k-space (the footnote of "Mock generation"
  notes this is equivalent and saves one FFT), as unit-variance complex
  normals W(k) obeying W(-k) = conj(W(k)) so the real-space field is real;
* delta_hat(k) = s(n^2) W(k) with s = sqrt(P/V_box) (see oracle.power);
* eta_pq_hat(k) = f k_p k_q / k^2 delta_hat(k) (eq:eta), and the
  line-of-sight component for a fixed line of sight z is
  eta_par_hat = f mu_z^2 delta_hat (section "The expected auto-correlation
  function of the mocks" writes eta_par_hat = f mu_k^2 delta_hat);
* real space: delta(m) = sum_k delta_hat(k) exp(+2 pi i n.m / N), the
  unnormalised inverse DFT; grid point m sits at x = m dx.

Mode bookkeeping (paper silent; reading chosen here):
* index i in [0, N) per axis, signed frequency n = i for i < N/2, else i - N
  (so the Nyquist index N/2 has n = -N/2);
* linear index lin(i) = (ix N + iy) N + iz; partner i' = (-i) mod N;
* the owner of a pair is the mode with the lower linear index; its normals
  come from oracle.philox.normal_pair(seed, 0, lin(owner));
* W(owner) = (z1 + i z2)/sqrt(2), W(partner) = conj(W(owner)); a
  self-conjugate mode (every index 0 or N/2) takes W = z1;
* fixed_amp (Angulo & Pontzen 2016 test hook): W <- W/|W|;
* only_n2 (test hook): keep only modes with n^2 == only_n2;
* k = 0 carries no power (s(0) = 0);
* cross components (p != q) vanish on the Nyquist plane of p or q, where
  k_p k_q would break the Hermitian symmetry.

The packed output of the hot path is the complex field delta + i eta_par,
obtained from one inverse transform of delta_hat + i eta_par_hat.
"""
import numpy as np

from . import philox

COMPONENTS = ("delta", "xx", "yy", "zz", "xy", "xz", "yz", "vx", "vy", "vz")


def signed_freq(i, n):
    i = np.asarray(i, dtype=np.int64)
    return np.where(i < n // 2, i, i - n)


def mode_grid(n, ix_slice=None):
    """Integer index grids (ix, iy, iz) for all modes, or for a slab of ix."""
    ix = np.arange(n, dtype=np.int64) if ix_slice is None else \
        np.arange(n, dtype=np.int64)[ix_slice]
    iy = np.arange(n, dtype=np.int64)
    iz = np.arange(n, dtype=np.int64)
    return np.meshgrid(ix, iy, iz, indexing="ij")


def noise_at(n, seed, gx, gy, gz, fixed_amp=False):
    """Hermitian-paired unit complex noise W of the modes with index arrays
    (gx, gy, gz) in [0, n): the lower linear index of a mode and its partner
    -n mod N owns the Philox draw; the partner takes the conjugate;
    self-conjugate modes take the real normal."""
    gx, gy, gz = (np.asarray(a, dtype=np.int64) for a in (gx, gy, gz))
    lin = (gx * n + gy) * n + gz
    px, py, pz = (-gx) % n, (-gy) % n, (-gz) % n
    plin = (px * n + py) * n + pz
    owner = np.minimum(lin, plin)
    z1, z2 = philox.normal_pair(seed, 0, owner.astype(np.uint64))
    w = (z1 + 1j * z2) / np.sqrt(2.0)
    w = np.where(lin > plin, np.conj(w), w)
    w = np.where(lin == plin, z1 + 0j, w)
    if fixed_amp:
        w = w / np.abs(w)
    return w


def white_noise(n, seed, ix_slice=None, fixed_amp=False):
    """Hermitian-paired unit complex noise W for all modes (or an ix slab)."""
    gx, gy, gz = mode_grid(n, ix_slice)
    return noise_at(n, seed, gx, gy, gz, fixed_amp)


def multiplier_at(n, comp, f, gx, gy, gz, box_len=None):
    """Multiplier turning delta_hat into the requested component at the
    modes (gx, gy, gz); None for delta.  Real for eta_pq; for the velocity
    v_j (eq:velocity, at z = 0 with aH = 100 km/s per Mpc/h) it is
    i f 100 k_j / k^2 (km/s), k_j = 2 pi n_j / box_len, zero on the Nyquist
    plane of j (odd in k: such a mode is its own partner)."""
    if comp == "delta":
        return None
    nv = [signed_freq(gx, n), signed_freq(gy, n), signed_freq(gz, n)]
    n2 = nv[0] ** 2 + nv[1] ** 2 + nv[2] ** 2
    axis = {"x": 0, "y": 1, "z": 2}
    if comp[0] == "v":
        j = nv[axis[comp[1]]]
        kj_over_k2 = np.where((n2 > 0) & (j != -(n // 2)), j / np.where(n2 > 0, n2, 1), 0.0) * box_len / (2 * np.pi)
        return 1j * f * 100.0 * kj_over_k2
    p, q = axis[comp[0]], axis[comp[1]]
    num = (nv[p] * nv[q]).astype(np.float64)
    if p != q:
        nyq = (nv[p] == -(n // 2)) | (nv[q] == -(n // 2))
        num = np.where(nyq, 0.0, num)
    return f * np.where(n2 > 0, num / np.where(n2 > 0, n2, 1), 0.0)


def component_multiplier(n, comp, f=1.0, ix_slice=None, box_len=None):
    """Multiplier turning delta_hat into the requested component."""
    if comp == "delta":
        return None
    gx, gy, gz = mode_grid(n, ix_slice)
    return multiplier_at(n, comp, f, gx, gy, gz, box_len)


def amplitudes(n, table, ix_slice=None, only_n2=-1):
    gx, gy, gz = mode_grid(n, ix_slice)
    n2 = signed_freq(gx, n) ** 2 + signed_freq(gy, n) ** 2 + signed_freq(gz, n) ** 2
    s = table[n2]
    if only_n2 >= 0:
        s = np.where(n2 == only_n2, s, 0.0)
    return s


def spectrum(n, seed, table, comps=("delta", "zz"), f=1.0, fixed_amp=False,
             only_n2=-1, ix_slice=None, box_len=None):
    """Packed k-space field X = C_a + i C_b for the component pair comps
    (box_len, the box side in Mpc/h, is needed by the velocities)."""
    w = white_noise(n, seed, ix_slice, fixed_amp)
    s = amplitudes(n, table, ix_slice, only_n2)
    base = s * w
    out = []
    for c in comps:
        m = component_multiplier(n, c, f, ix_slice, box_len)
        out.append(base if m is None else m * base)
    if len(out) == 1:
        return out[0]
    return out[0] + 1j * out[1]


def inverse_dft3(x):
    """Unnormalised inverse DFT with exp(+2 pi i n.m/N)."""
    n = x.shape[0]
    return np.fft.ifftn(x) * float(n) ** 3


def make_box(n, seed, table, comps=("delta", "zz"), f=1.0, fixed_amp=False,
             only_n2=-1, box_len=None):
    """Complex field C_a + i C_b on the grid (for comps=("delta","zz"),
    real part = delta, imaginary part = eta_par along z)."""
    x = spectrum(n, seed, table, comps, f, fixed_amp, only_n2, box_len=box_len)
    return inverse_dft3(x)


def brute_force_field(n, xhat):
    """Direct triple sum of the inverse DFT (test pin, tiny n only)."""
    m = np.arange(n)
    nn = signed_freq(m, n)
    ph = np.exp(2j * np.pi * np.outer(nn, m) / n)   # [freq, grid]
    out = np.zeros((n, n, n), dtype=np.complex128)
    for a in range(n):
        for b in range(n):
            for c in range(n):
                out += xhat[a, b, c] * (ph[a][:, None, None] * ph[b][None, :, None]
                                        * ph[c][None, None, :])
    return out


def shell_modes(n, seed, table, only_n2, comps=("delta", "zz"), f=1.0, box_len=None):
    """The modes of one shell |n|^2 = only_n2 of the packed spectrum (the
    spectrum() field with every other mode zero): integer frequencies
    [M, 3] and complex coefficients [M], from the same noise, amplitude and
    component rules as spectrum()."""
    r = int(np.floor(np.sqrt(only_n2))) + 1
    v = np.arange(-r, r + 1)
    nx, ny, nz = np.meshgrid(v, v, v, indexing="ij")
    sel = (nx ** 2 + ny ** 2 + nz ** 2 == only_n2) & (np.abs(nx) <= n // 2) & (np.abs(ny) <= n // 2) & \
        (np.abs(nz) <= n // 2) & (nx != n // 2) & (ny != n // 2) & (nz != n // 2)
    freqs = np.stack([nx[sel], ny[sel], nz[sel]], axis=1).astype(np.int64)
    gx, gy, gz = (freqs[:, i] % n for i in range(3))
    base = table[only_n2] * noise_at(n, seed, gx, gy, gz)
    vals = []
    for comp in comps:
        mult = multiplier_at(n, comp, f, gx, gy, gz, box_len)
        vals.append(base if mult is None else mult * base)
    coef = vals[0] if len(vals) == 1 else vals[0] + 1j * vals[1]
    return freqs, coef


def shell_field_at(n, freqs, coef, ix, iy, iz, chunk=1 << 15):
    """Direct sum of the inverse DFT over the given modes at grid points
    (ix, iy, iz) (integer arrays of equal shape): sum_m coef_m
    exp(2 pi i (a ix + b iy + c iz) / n), the phase reduced mod n in integers
    first (so it is exact), then taken from a table of exp(2 pi i k / n)."""
    ix, iy, iz = (np.asarray(a, dtype=np.int64) for a in (ix, iy, iz))
    pts = np.stack([ix.ravel(), iy.ravel(), iz.ravel()], axis=1)
    cis = np.exp(2j * np.pi * np.arange(n) / n)
    f = np.asarray(freqs, dtype=np.int64).T
    coef = np.asarray(coef, dtype=np.complex128)
    out = np.empty(len(pts), dtype=np.complex128)
    for s in range(0, len(pts), chunk):
        out[s:s + chunk] = cis[(pts[s:s + chunk] @ f) % n] @ coef
    return out.reshape(ix.shape)
