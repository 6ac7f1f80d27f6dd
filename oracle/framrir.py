"""FRAM-RIR (Luo & Gu, arXiv 2304.08052), plain FP64 CPU oracle.

TEST INFRASTRUCTURE ONLY (see the package docstring).

What is computed, in the paper's order and notation
----------------------------------------------------
Per room (Sec. II, Sec. III-A):
  R   = volume / total surface area of the empty shoebox room      (Sec. III-A)
  r   = sqrt(1 - (1 - exp(-0.16 R / T60))^2)                       (Eq. 2)
  T   = ceil(T60 * fs) output samples per channel   (length L of Sec. III-D,
        taken at the output rate fs; reading R-14)
  centre = mean of the microphone positions: the sphere centre of Sec. III-B
        (reading R-2)
Per source:
  d0  = |src - centre|,  cT = c0 * T60,  q = cT / d0
  RR_max = (log10 cT - log10 d0 - 3) / log10 r, clamped below at 1  (Eq. 5, R-8)
  I   = number of sampled virtual sources, drawn from the header counter
        (reading R-6)
Per virtual source i = 1..I (Sec. III-B, III-C), from four Philox words:
  theta ~ U[0, 2 pi],  phi ~ U[-pi/2, pi/2]                        (Sec. III-B)
  xhat  ~ P(x) = 3 x^2 / (beta^3 - alpha^3) on (alpha, beta]       (Eq. 3),
          by the inverse CDF xhat = cbrt(alpha^3 + u (beta^3 - alpha^3))
  DR    = 1 + (xhat - alpha)/(beta - alpha) * (cT/d0 - 1)          (Eq. 4, R-7)
  D     = d0 * DR
  p     ~ U(a, b)
  g     = clamp(1 + (D/cT)^2 (RR_max - 1) + p DR^tau, 1, RR_max)   (Eq. 6)
  pos   = centre + D (cos phi cos theta, cos phi sin theta, sin phi)
The direct path is image 0 with pos = src and g = 0 (Sec. III-D).
Per microphone m and image i (Eq. 1, with the delay kept fractional, R-10):
  D_im = |pos_i - mic_m|,  t = D_im fs / c0,  A = r^g_i / D_im
  h_m[n] += A * P(n - t)  for the 81 taps n = round(t) - 40 .. round(t) + 40
  that fall in [0, T), where P(x) = sinc(x) * (1 + cos(2 pi x / 81)) / 2 is the
  81-tap Hann-windowed sinc (reading R-11) and round(t) = floor(t + 1/2).

The numbered readings R-n are the interpretations adopted where the paper is
silent or ambiguous; each is stated next to the code that depends on it.

FP64 discipline.  The draws are evaluated one IEEE operation at a time in the
order written (numpy ufuncs never fuse a multiply and an add), with correctly
rounded sqrt and a correctly rounded cube root, so the reflection counts g are a
function of the inputs alone.  exp and log10 appear only in the per-room and
per-source scalars and are taken from the C library through ``math``.
"""
import math
from dataclasses import dataclass

import numpy as np

from .cbrt import cbrt_rn
from .philox import philox4x32

TWO_PI = 6.283185307179586      # the double nearest 2*pi
PI = 3.141592653589793          # the double nearest pi
TAPS = 81                       # pulse length (reading R-11)
HALF = TAPS // 2                # 40
TWO_NEG32 = 2.0 ** -32


@dataclass(frozen=True)
class Params:
    """Free constants of the method.  The paper names alpha, beta (Eq. 3),
    a, b (Eq. 6) and tau (Eq. 6) but gives no values (reading R-5); the image
    count range is reading R-6."""
    alpha: float = 0.25
    beta: float = 1.0
    a: float = -2.0
    b: float = 2.0
    tau: float = 0.25
    img_lo: int = 1024
    img_hi: int = 4096


# ---------------------------------------------------------------------------
# Per-room and per-source scalars (Eq. 2, Eq. 5, Sec. III-A, Sec. III-D)
# ---------------------------------------------------------------------------

def rir_length(rt60, fs):
    """Samples per channel: ceil(T60 * fs) (Sec. III-D, at the output rate)."""
    return int(math.ceil(rt60 * fs))


def room_ratio(size):
    """R = V / S of an empty shoebox room (Sec. III-A, quantity of Eq. 2)."""
    lx, ly, lz = (float(v) for v in size)
    volume = (lx * ly) * lz
    area = 2.0 * ((lx * ly + lx * lz) + ly * lz)
    return volume / area


def eyring_r(size, rt60):
    """Reflection coefficient of Eq. 2, as printed (constant 0.16)."""
    big_r = room_ratio(size)
    x = (0.16 * big_r) / rt60
    eps = 1.0 - math.exp(-x)
    return math.sqrt(1.0 - eps * eps)


def array_centre(mics):
    """Sphere centre of Sec. III-B: the mean microphone position (R-2),
    summed in microphone order."""
    mics = np.asarray(mics, dtype=np.float64).reshape(-1, 3)
    cx = cy = cz = 0.0
    for m in mics:
        cx += float(m[0])
        cy += float(m[1])
        cz += float(m[2])
    n = float(len(mics))
    return np.array([cx / n, cy / n, cz / n])


def source_scalars(src, centre, c, rt60, r):
    """d0, cT, q = cT/d0 and RR_max (Eq. 5) for one source."""
    dx = float(src[0]) - float(centre[0])
    dy = float(src[1]) - float(centre[1])
    dz = float(src[2]) - float(centre[2])
    d0 = math.sqrt((dx * dx + dy * dy) + dz * dz)
    ct = c * rt60
    q = ct / d0
    rr = ((math.log10(ct) - math.log10(d0)) - 3.0) / math.log10(r)
    # Reading R-8: when c0 T60 / d0 >= 1000 r, spherical spreading alone
    # already reaches -60 dB and Eq. 5 gives RR_max <= 1 (negative beyond
    # 1000); clamp so Eq. 6's clamp is well defined (g == 1 then).
    rr = max(rr, 1.0)
    return d0, ct, q, rr


# ---------------------------------------------------------------------------
# Counter-based draws (Sec. III-B, III-C)
# ---------------------------------------------------------------------------

def _key(seed):
    seed = int(seed)
    return seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF


def num_images(seed, s, prm):
    """I for source s of a room with this seed (reading R-6): the first word
    of the header counter (0, s, 1, 0), scaled onto [img_lo, img_hi] by a
    64-bit multiply-shift."""
    k0, k1 = _key(seed)
    w = int(philox4x32(0, s, 1, 0, k0, k1)[0])
    span = prm.img_hi - prm.img_lo + 1
    return prm.img_lo + ((w * span) >> 32)


def image_words(seed, s, n_img):
    """Philox-4x32-10 words of images 0..n_img-1 of source s: counter
    (i, s, 0, 0), key (seed low word, seed high word) (reading R-21)."""
    k0, k1 = _key(seed)
    i = np.arange(n_img, dtype=np.uint64)
    return np.stack(philox4x32(i, s, 0, 0, k0, k1), axis=1)    # (n_img, 4)


def words_to_unit(words):
    """u = (w + 1/2) 2^-32: exact in FP64 and strictly inside (0, 1)."""
    return (words.astype(np.float64) + 0.5) * TWO_NEG32


def dr_pow_tau(dr, tau):
    """DR^tau of Eq. 6 for the supported shrinkage factors, each a chain of
    correctly rounded square roots."""
    if tau == 0.25:
        return np.sqrt(np.sqrt(dr))
    if tau == 0.5:
        return np.sqrt(dr)
    if tau == 1.0:
        return dr.copy()
    raise ValueError("tau must be 0.25, 0.5 or 1.0")


def distance_ratio(xhat, q, prm):
    """Eq. 4: rescale xhat in [alpha, beta] linearly onto DR in [1, q],
    q = c0 T60 / d0.  Written (xhat - alpha)/(beta - alpha), which equals the
    printed alpha/(beta - alpha) * (xhat/alpha - 1) and stays defined at
    alpha = 0 (reading R-7)."""
    tt = (np.asarray(xhat, dtype=np.float64) - prm.alpha) / (prm.beta - prm.alpha)
    return 1.0 + tt * (q - 1.0)


def reflection_count(dist, dr, p, ct, rrmax, prm):
    """Eq. 6: g = clamp(1 + (D/cT)^2 (RR_max - 1) + p DR^tau, 1, RR_max)."""
    s2 = np.asarray(dist, dtype=np.float64) / ct
    g = 1.0 + (s2 * s2) * (rrmax - 1.0)            # distance term
    g = g + p * dr_pow_tau(np.asarray(dr, dtype=np.float64), prm.tau)   # perturbation
    return np.minimum(np.maximum(g, 1.0), rrmax)   # clamp


def draw_images(seed, s, n_img, centre, d0, q, ct, rrmax, prm):
    """The I sampled virtual sources of one source (Sec. III-B, III-C).

    Returns a dict of arrays of length n_img: words (n,4), theta, phi, xhat,
    p, dr, dist, g, dir (n,3), pos (n,3)."""
    words = image_words(seed, s, n_img)
    u = words_to_unit(words)
    theta = u[:, 0] * TWO_PI                       # azimuth ~ U[0, 2pi]
    phi = (u[:, 1] - 0.5) * PI                     # elevation ~ U[-pi/2, pi/2]
    a3 = (prm.alpha * prm.alpha) * prm.alpha
    b3 = (prm.beta * prm.beta) * prm.beta
    arg = a3 + u[:, 2] * (b3 - a3)                 # inverse CDF of Eq. 3
    xhat = np.array([cbrt_rn(v) for v in arg], dtype=np.float64)
    p = prm.a + u[:, 3] * (prm.b - prm.a)          # p ~ U(a, b), Eq. 6
    dr = distance_ratio(xhat, q, prm)
    dist = d0 * dr                                 # D_i = D_0 * DR_i
    g = reflection_count(dist, dr, p, ct, rrmax, prm)
    cphi = np.cos(phi)
    direction = np.stack([cphi * np.cos(theta), cphi * np.sin(theta), np.sin(phi)], axis=1)
    pos = centre[None, :] + dist[:, None] * direction
    return dict(words=words, theta=theta, phi=phi, xhat=xhat, p=p, dr=dr,
                dist=dist, g=g, dir=direction, pos=pos)


# ---------------------------------------------------------------------------
# Batch description
# ---------------------------------------------------------------------------

@dataclass
class Room:
    size: tuple
    rt60: float
    fs: float
    c: float
    seed: int
    src: np.ndarray          # (S, 3)
    mic: np.ndarray          # (M, 3)
    r_override: float = float("nan")


def rooms_from_batch(batch):
    """Split the flat arrays of a synthetic batch (see the workloads module)
    into Room records."""
    rooms = []
    so = mo = 0
    for b in range(len(batch["rt60"])):
        ns = int(batch["n_src"][b])
        nm = int(batch["n_mic"][b])
        rooms.append(Room(size=tuple(float(v) for v in batch["size"][b]),
                          rt60=float(batch["rt60"][b]), fs=float(batch["fs"][b]),
                          c=float(batch["c"][b]), seed=int(batch["seed"][b]),
                          src=np.asarray(batch["src"][so:so + ns], dtype=np.float64),
                          mic=np.asarray(batch["mic"][mo:mo + nm], dtype=np.float64),
                          r_override=float(batch["r_override"][b])))
        so += ns
        mo += nm
    return rooms


def room_plan(room, prm):
    """All per-room and per-source scalars plus the image tables.

    Returns dict(T, r, centre, sources=[dict(d0, ct, q, rrmax, I, draws,
    pos (I+1,3), g (I+1,))])."""
    t_len = rir_length(room.rt60, room.fs)
    r = eyring_r(room.size, room.rt60) if math.isnan(room.r_override) else float(room.r_override)
    centre = array_centre(room.mic)
    sources = []
    for s, src in enumerate(room.src):
        d0, ct, q, rr = source_scalars(src, centre, room.c, room.rt60, r)
        n_img = num_images(room.seed, s, prm)
        dr = draw_images(room.seed, s, n_img, centre, d0, q, ct, rr, prm)
        pos = np.vstack([np.asarray(src, dtype=np.float64)[None, :], dr["pos"]])
        g = np.concatenate([[0.0], dr["g"]])          # direct path: g_0 = 0
        sources.append(dict(d0=d0, ct=ct, q=q, rrmax=rr, I=n_img, draws=dr, pos=pos, g=g))
    return dict(T=t_len, r=r, centre=centre, sources=sources)


# ---------------------------------------------------------------------------
# Rendering (Eq. 1 / Eq. 8 with a band-limited fractional-delay pulse)
# ---------------------------------------------------------------------------

def pulse(x):
    """P(x): 81-tap Hann-windowed sinc, zero for |x| >= 40.5 (reading R-11)."""
    x = np.asarray(x, dtype=np.float64)
    val = np.sinc(x) * 0.5 * (1.0 + np.cos(TWO_PI * x / TAPS))
    return np.where(np.abs(x) < TAPS / 2.0, val, 0.0)


def pulse_deriv(x):
    """P'(x) = sinc'(x) w(x) + sinc(x) w'(x), w(x) = (1 + cos(2 pi x/81))/2,
    sinc'(x) = (cos(pi x) - sinc(x)) / x (0 at x = 0; for |x| < 1e-5 the
    two-term Taylor series -pi^2 x/3 + pi^4 x^3/30 avoids cancellation)."""
    x = np.asarray(x, dtype=np.float64)
    sinc = np.sinc(x)
    small = np.abs(x) < 1e-5
    xs = np.where(small, 1.0, x)
    dsinc = np.where(small, -(PI * PI) * x / 3.0 + (PI ** 4) * x ** 3 / 30.0,
                     (np.cos(PI * x) - sinc) / xs)
    w = 0.5 * (1.0 + np.cos(TWO_PI * x / TAPS))
    dw = -(PI / TAPS) * np.sin(TWO_PI * x / TAPS)
    val = dsinc * w + sinc * dw
    return np.where(np.abs(x) < TAPS / 2.0, val, 0.0)


def pair_geometry(pos, g, mic, r, fs, c):
    """Per (image, microphone) distance, delay in samples and amplitude (Eq. 1)."""
    diff = pos - np.asarray(mic, dtype=np.float64)[None, :]
    dist = np.sqrt(np.sum(diff * diff, axis=1))
    t = dist * fs / c
    amp = np.power(r, g) / dist
    return diff, dist, t, amp


def footprint(t):
    """Sample indices (float) and offsets x = n - t of the 81 taps per image."""
    k = np.floor(t + 0.5)
    n = k[:, None] + np.arange(-HALF, HALF + 1, dtype=np.float64)[None, :]
    return n, n - t[:, None]


def render_channel(pos, g, mic, r, fs, c, t_len):
    """h_m[n], n in [0, T), for one microphone and one image table (Eq. 1, 8)."""
    _, _, t, amp = pair_geometry(pos, g, mic, r, fs, c)
    n, x = footprint(t)
    w = amp[:, None] * pulse(x)
    ok = (n >= 0) & (n < t_len)
    return np.bincount(n[ok].astype(np.int64), weights=w[ok], minlength=t_len)[:t_len]


def render_room(plan, room, mic=None, src=None, r=None):
    """[S, M, T] RIRs of one room.  ``mic``, ``src`` and ``r`` default to the
    room's own; passing others re-renders with the image table held fixed
    (only the direct path follows ``src``)."""
    mic = room.mic if mic is None else np.asarray(mic, dtype=np.float64)
    src = room.src if src is None else np.asarray(src, dtype=np.float64)
    r = plan["r"] if r is None else float(r)
    out = np.zeros((len(plan["sources"]), len(mic), plan["T"]))
    for s, so in enumerate(plan["sources"]):
        pos = so["pos"].copy()
        pos[0] = src[s]
        for m in range(len(mic)):
            out[s, m] = render_channel(pos, so["g"], mic[m], r, room.fs, room.c, plan["T"])
    return out


def simulate(batch, prm=Params()):
    """Oracle for a whole batch: list of [S_b, M_b, T_b] arrays and the plans."""
    rooms = rooms_from_batch(batch)
    plans = [room_plan(rm, prm) for rm in rooms]
    return [render_room(p, rm) for p, rm in zip(plans, rooms)], plans, rooms


# ---------------------------------------------------------------------------
# Adjoint with the draws held fixed (reading R-20)
# ---------------------------------------------------------------------------

def adjoint_room(plan, room, grad_h, mic=None, src=None, r=None):
    """dL/dmic (M,3), dL/dsrc (S,3), dL/dr (scalar) for dL/dh = grad_h [S,M,T].

    With u = (pos - mic)/D, dt/dmic = -(fs/c) u and dA/dmic = (A/D) u, so
      dL/dmic_m = sum_i u (A/D S0 + A fs/c S1),
      S0 = sum_n G[n] P(n - t),  S1 = sum_n G[n] P'(n - t);
    only the direct path depends on the source, with the opposite sign;
      dL/dr = sum (g/r) A S0   (A = r^g / D)."""
    mic = room.mic if mic is None else np.asarray(mic, dtype=np.float64)
    src = room.src if src is None else np.asarray(src, dtype=np.float64)
    r = plan["r"] if r is None else float(r)
    fs, c, t_len = room.fs, room.c, plan["T"]
    g_mic = np.zeros((len(mic), 3))
    g_src = np.zeros((len(src), 3))
    g_r = 0.0
    for s, so in enumerate(plan["sources"]):
        pos = so["pos"].copy()
        pos[0] = src[s]
        g = so["g"]
        for m in range(len(mic)):
            diff, dist, t, amp = pair_geometry(pos, g, mic[m], r, fs, c)
            u = diff / dist[:, None]
            n, x = footprint(t)
            ok = (n >= 0) & (n < t_len)
            gn = np.where(ok, grad_h[s, m][np.clip(n, 0, t_len - 1).astype(np.int64)], 0.0)
            s0 = np.sum(gn * pulse(x), axis=1)
            s1 = np.sum(gn * pulse_deriv(x), axis=1)
            coef = amp / dist * s0 + amp * (fs / c) * s1
            contrib = u * coef[:, None]
            g_mic[m] += contrib.sum(axis=0)
            g_src[s] -= contrib[0]
            g_r += float(np.sum((g / r) * amp * s0))
    return g_mic, g_src, g_r


def l2_loss(out, target):
    """L = sum (h - target)^2 and its gradient dL/dh = 2 (h - target)."""
    d = out - target
    return float(np.sum(d * d)), 2.0 * d


def fd_grads(plan, room, target, step=1e-6, mic=None, src=None, r=None):
    """Central finite differences of l2_loss(render(...), target) with respect
    to every microphone and source coordinate and to r, table held fixed."""
    mic = (room.mic if mic is None else np.asarray(mic, dtype=np.float64)).copy()
    src = (room.src if src is None else np.asarray(src, dtype=np.float64)).copy()
    r = plan["r"] if r is None else float(r)

    def loss(mm, ss, rr):
        return l2_loss(render_room(plan, room, mic=mm, src=ss, r=rr), target)[0]

    g_mic = np.zeros_like(mic)
    for m in range(mic.shape[0]):
        for k in range(3):
            mp, mn = mic.copy(), mic.copy()
            mp[m, k] += step
            mn[m, k] -= step
            g_mic[m, k] = (loss(mp, src, r) - loss(mn, src, r)) / (2 * step)
    g_src = np.zeros_like(src)
    for s in range(src.shape[0]):
        for k in range(3):
            sp, sn = src.copy(), src.copy()
            sp[s, k] += step
            sn[s, k] -= step
            g_src[s, k] = (loss(mic, sp, r) - loss(mic, sn, r)) / (2 * step)
    g_r = (loss(mic, src, r + step) - loss(mic, src, r - step)) / (2 * step)
    return g_mic, g_src, g_r


def adjoint_room_draws(plan, room, grad_h, prm):
    """dL/dmic, dL/dsrc, dL/dr of the whole map, the images re-drawn at the
    inputs: the Philox variates (theta, phi, xhat, p) depend on the seed only,
    while with t_i = (xhat_i - alpha)/(beta - alpha) (Eq. 4)
      D_i = d0 + t_i (cT - d0),  DR_i = D_i / d0,  pos_i = centre + D_i dir_i,
      g_i = clamp(gamma_i, 1, RR),  gamma_i = 1 + (D_i/cT)^2 (RR - 1) + p_i DR_i^tau,
      RR = max(1, (log10 cT - log10 d0 - 3) / log10 r)  (Eq. 5, 6),
      d0 = |src - centre|,  centre = mean of the microphones.
    Per image the pairs give dL/dpos_i (minus the microphone term) and dL/dg_i
    = ln(r) A S0; then
      dL/dd0 = sum_i (dir_i . dL/dpos_i)(1 - t_i) + dL/dg_i dg_i/dd0,
      dg/dd0 = 2 (D/cT^2)(RR - 1)(1 - t) + (D/cT)^2 dRR/dd0 - tau p DR^(tau-1) t cT / d0^2
               inside the clamp, dRR/dd0 at the top clamp, 0 at the bottom,
      dRR/dd0 = -1 / (d0 ln r),  dRR/dr = -RR / (r ln r)  (0 where RR is clamped to 1),
      dL/dsrc += dL/dd0 (src - centre) / d0,
      dL/dmic += (sum_i dL/dpos_i - dL/dd0 (src - centre) / d0) / M  (every microphone),
      dL/dr += sum_i dL/dg_i dg_i/dr  (dg/dr = (D/cT)^2 dRR/dr inside, dRR/dr at the top).
    Gradient at the room's own positions (where the images were drawn)."""
    g_mic, g_src, g_r = adjoint_room(plan, room, grad_h)
    r, centre, fs, c, t_len = plan["r"], plan["centre"], room.fs, room.c, plan["T"]
    ln_r = math.log(r)
    n_mic = len(room.mic)
    g_centre = np.zeros(3)
    for s, so in enumerate(plan["sources"]):
        d = so["draws"]
        d0, ct, rr = so["d0"], so["ct"], so["rrmax"]
        pos, g = so["pos"][1:], so["g"][1:]
        dpos = np.zeros_like(pos)
        dg = np.zeros(len(g))
        for m in range(n_mic):
            diff, dist, t, amp = pair_geometry(pos, g, room.mic[m], r, fs, c)
            u = diff / dist[:, None]
            n, x = footprint(t)
            ok = (n >= 0) & (n < t_len)
            gn = np.where(ok, grad_h[s, m][np.clip(n, 0, t_len - 1).astype(np.int64)], 0.0)
            s0 = np.sum(gn * pulse(x), axis=1)
            s1 = np.sum(gn * pulse_deriv(x), axis=1)
            coef = amp / dist * s0 + amp * (fs / c) * s1
            dpos -= u * coef[:, None]
            dg += ln_r * amp * s0
        tt = (d["xhat"] - prm.alpha) / (prm.beta - prm.alpha)
        D, DR, p = d["dist"], d["dr"], d["p"]
        rr_raw = ((math.log10(ct) - math.log10(d0)) - 3.0) / math.log10(r)
        drr_dd0 = -1.0 / (d0 * ln_r) if rr_raw > 1.0 else 0.0
        drr_dr = -rr_raw / (r * ln_r) if rr_raw > 1.0 else 0.0
        gamma = 1.0 + (D / ct) ** 2 * (rr - 1.0) + p * DR ** prm.tau
        dgam_dd0 = (2.0 * D / ct ** 2 * (rr - 1.0) * (1.0 - tt) + (D / ct) ** 2 * drr_dd0
                    - prm.tau * p * DR ** (prm.tau - 1.0) * tt * ct / d0 ** 2)
        dgam_dr = (D / ct) ** 2 * drr_dr
        top, bottom = gamma >= rr, gamma <= 1.0
        dg_dd0 = np.where(top, drr_dd0, np.where(bottom, 0.0, dgam_dd0))
        dg_dr = np.where(top, drr_dr, np.where(bottom, 0.0, dgam_dr))
        dl_dd0 = float(np.sum(np.sum(d["dir"] * dpos, axis=1) * (1.0 - tt) + dg * dg_dd0))
        g_r += float(np.sum(dg * dg_dr))
        u0 = (np.asarray(room.src[s], dtype=np.float64) - centre) / d0
        g_src[s] += dl_dd0 * u0
        g_centre += dpos.sum(axis=0) - dl_dd0 * u0
    g_mic += g_centre[None, :] / n_mic
    return g_mic, g_src, g_r


def fd_grads_draws(room, prm, grad_h, step=1e-6):
    """Central finite differences of L = sum(grad_h * h) with the images
    re-drawn at every perturbed input (same seed), r given as an override."""
    base = room_plan(room, prm)

    def loss(mic, src, r):
        rm = Room(room.size, room.rt60, room.fs, room.c, room.seed, src, mic, r)
        return float(np.sum(grad_h * render_room(room_plan(rm, prm), rm)))

    mic, src, r = room.mic.copy(), room.src.copy(), base["r"]
    g_mic, g_src = np.zeros_like(mic), np.zeros_like(src)
    for arr, out in ((mic, g_mic), (src, g_src)):
        for i in range(arr.shape[0]):
            for k in range(3):
                plus, minus = arr.copy(), arr.copy()
                plus[i, k] += step
                minus[i, k] -= step
                lp = loss(plus, src, r) if arr is mic else loss(mic, plus, r)
                lm = loss(minus, src, r) if arr is mic else loss(mic, minus, r)
                out[i, k] = (lp - lm) / (2 * step)
    g_r = (loss(mic, src, r + step) - loss(mic, src, r - step)) / (2 * step)
    return g_mic, g_src, g_r


# ---------------------------------------------------------------------------
# Early-reverberation mask (Eq. 9), at the output rate
# ---------------------------------------------------------------------------

def early_window(t_direct, fs):
    """[lo, hi] sample range kept by Eq. 9 around the direct-path delay:
    n - ceil(t0) in [-ceil(6 fs/1000), ceil(50 fs/1000)]."""
    k0 = math.ceil(t_direct)
    return k0 - math.ceil(6.0 * fs / 1000.0), k0 + math.ceil(50.0 * fs / 1000.0)


def early_room(room, h):
    """Early-reverberation filter of Eq. 9 for one room's RIRs h [S, M, T].

    Reading R-23: the window is taken at the output rate (the paper states it
    on its high-rate grid, r_h fs), and D_0 is the direct-path distance from
    the source to each microphone, so t0 = D_0 fs / c0 per (source, mic).
    h_e[n] = h[n] for lo <= n <= hi and 0 elsewhere; only the window can be
    non-zero, so it is returned compactly: early [S, M, W] holds h_e[lo..hi]
    (zero where n falls outside [0, T)) and start [S, M] holds lo."""
    n_src, n_mic, t_len = h.shape
    pre, post = math.ceil(6.0 * room.fs / 1000.0), math.ceil(50.0 * room.fs / 1000.0)
    width = pre + post + 1
    early = np.zeros((n_src, n_mic, width))
    start = np.zeros((n_src, n_mic), dtype=np.int64)
    for s in range(n_src):
        for m in range(n_mic):
            _, _, t, _ = pair_geometry(np.asarray(room.src[s], dtype=np.float64)[None, :], np.zeros(1),
                                       room.mic[m], 0.5, room.fs, room.c)
            lo, hi = early_window(float(t[0]), room.fs)
            start[s, m] = lo
            for n in range(max(lo, 0), min(hi, t_len - 1) + 1):
                early[s, m, n - lo] = h[s, m, n]
    return early, start
