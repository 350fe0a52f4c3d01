// Host planner: filter coefficients of Algorithm 2, lines 2-4 (FP64 output,
// extended-precision internals).
//
//  * Theorem 1 (eq. ZoloFunc, eq. coef): c_j = l^2 sc^2(j K'/(2r); l'),
//    K' = K(l') = pi / (2 AGM(1, l)).  sc is evaluated through Jacobi's
//    imaginary transformation: for a modulus k near 1 the descending Landen
//    recursion of the complementary modulus at argument i u stays on the
//    imaginary axis and gives sc(u; k) = sinh(psi_0), dn(u; k) =
//    sech(psi_1 - psi_0).  For u > K'/2 the quarter-period shift
//    sc(K' - v) = 1 / (l sc(v)) gives c_j = 1 / sc^2(v).  A modest modulus
//    (l >= 1/sqrt 2) uses the direct descending Landen scheme.
//  * M from equioscillation: M P(l) = 1 - delta, M P(x_1) = 1 + delta with
//    x_1 = l / dn(K'/(2r); l').
//  * eq. rZ: M_hat = M / (1 + delta), l2 = (1 - delta) / (1 + delta).
//  * Proposition 1 (partial fractions a_j), Proposition 2 (sigma_hat_j,
//    w_hat_j, constant term), Corollary 1 (outer shifts +- i sqrt(c_j)).
//  * Moebius map (eq. mo, eq. req), closed form: with t = (1 - l1)/2,
//    W = b_- - a_+, g_a = a_+ - a_-, g_b = b_+ - b_-,
//      alpha = a_- + t g_a (b_- - a_-) / (W + t g_a)
//      beta  = b_+ - t g_b (b_+ - a_+) / (W + t g_b)
//      gamma = -g_b (1 - t)(W + t g_a) / ((W + t g_b)(W + g_a))
//    which sends a_- -> -l1, a_+ -> l1, b_- -> 1, b_+ -> -1 (alpha in the
//    left gap, beta in the right gap), l1 = eps / (sqrt(1+eps)+1)^2 with eps
//    the cross-ratio of the four gap ends.  An infinite end replaces its
//    condition by T(+-inf) = gamma.
#include <cmath>
#include <complex>
#include <cstring>

#include "zolo_internal.h"

namespace zolo {
namespace {

typedef long double ld;

ld agm_ld(ld a, ld b) {
  for (int i = 0; i < 64 && fabsl(a - b) > 1e-19L * a; ++i) {
    ld an = 0.5L * (a + b);
    b = sqrtl(a * b);
    a = an;
  }
  return 0.5L * (a + b);
}

// K(k) with complementary modulus kc.
ld ellipk_kc(ld kc) { return 3.14159265358979323846264338327950288L / (2.0L * agm_ld(1.0L, kc)); }

struct Landen {
  ld a[70];
  ld c[70];
  int n;
};

// AGM from (1, b0) with c_1 = (1 - b0)/2 given; c_{n+1} = c_n^2 / (4 a_{n+1}).
// Stops once c_n exp(2^n a_n growth) is below rounding.
void landen(ld b0, ld c1, ld growth, Landen* L) {
  L->a[0] = 1.0L;
  L->c[0] = 0.0L;
  L->a[1] = 0.5L * (1.0L + b0);
  L->c[1] = c1;
  int n = 1;
  while (n < 66) {
    ld cn = L->c[n];
    if (cn == 0.0L) break;
    ld e = (ld)ldexpl(1.0L, n) * L->a[n] * growth;
    if (e > 11000.0L) e = 11000.0L;
    if (logl(cn) + e <= logl(1e-21L * L->a[n])) break;
    ld an = L->a[n];
    ld bn = sqrtl(an * an - cn * cn);
    L->a[n + 1] = 0.5L * (an + bn);
    L->c[n + 1] = cn * cn / (4.0L * L->a[n + 1]);
    ++n;
  }
  L->n = n;
}

// Modulus k near 1 (complement kc small), 0 <= u <= K/2: returns sc(u) and dn(u).
void sc_dn_imag(ld u, ld kc, ld* sc, ld* dn) {
  ld k = sqrtl((1.0L - kc) * (1.0L + kc));
  Landen L;
  landen(k, 0.5L * kc * kc / (1.0L + k), u, &L);
  ld psi = ldexpl(1.0L, L.n) * L.a[L.n] * u;
  ld prev = psi;
  for (int j = L.n; j >= 1; --j) {
    prev = psi;
    psi = 0.5L * (psi + asinhl(L.c[j] * sinhl(psi) / L.a[j]));
  }
  *sc = sinhl(psi);
  *dn = 1.0L / coshl(prev - psi);
}

// Modest modulus (kc >= 1/sqrt 2): direct descending Landen.
void sc_dn_direct(ld u, ld kc, ld* sc, ld* dn) {
  ld k = sqrtl((1.0L - kc) * (1.0L + kc));
  Landen L;
  landen(kc, 0.5L * (1.0L - kc), 0.0L, &L);
  ld phi = ldexpl(1.0L, L.n) * L.a[L.n] * u;
  for (int j = L.n; j >= 1; --j) {
    ld s = L.c[j] * sinl(phi) / L.a[j];
    if (s > 1.0L) s = 1.0L;
    if (s < -1.0L) s = -1.0L;
    phi = 0.5L * (phi + asinl(s));
  }
  ld sn = sinl(phi), cn = cosl(phi);
  *sc = sn / cn;
  *dn = sqrtl(kc * kc + k * k * cn * cn);
}

// Zolotarev data of Z_2r(x; l) (Theorem 1).
struct ZoloData {
  int r;
  ld l;
  ld c[2 * ZOLO_MAX_R];  // c[j-1] = c_j, j = 1..2r-1
  ld M, delta;
  ld a[ZOLO_MAX_R];      // Proposition 1
};

ld zolo_P(const ZoloData& z, ld x) {
  ld x2 = x * x, num = 1.0L, den = 1.0L;
  for (int j = 1; j <= z.r - 1; ++j) num *= x2 + z.c[2 * j - 1];
  for (int j = 1; j <= z.r; ++j) den *= x2 + z.c[2 * j - 2];
  return x * num / den;
}

void zolo_make(int r, ld l, ZoloData* z) {
  z->r = r;
  z->l = l;
  ld Kp = ellipk_kc(l);  // K' = K(l'), complement of l' is l
  bool imag = l < 0.70710678118654752440L;
  for (int j = 1; j <= 2 * r - 1; ++j) {
    ld u = (ld)j * Kp / (ld)(2 * r);
    ld sc, dn;
    if (!imag) {
      sc_dn_direct(u, l, &sc, &dn);
      z->c[j - 1] = l * l * sc * sc;
    } else if (2 * j <= 2 * r) {
      sc_dn_imag(u, l, &sc, &dn);
      z->c[j - 1] = l * l * sc * sc;
    } else {
      sc_dn_imag(Kp - u, l, &sc, &dn);  // sc(K' - v) = 1/(l sc(v))
      z->c[j - 1] = 1.0L / (sc * sc);
    }
  }
  ld sc1, dn1;
  ld u1 = Kp / (ld)(2 * r);
  if (imag)
    sc_dn_imag(u1, l, &sc1, &dn1);
  else
    sc_dn_direct(u1, l, &sc1, &dn1);
  ld x0 = l, x1 = l / dn1;
  ld p0 = zolo_P(*z, x0), p1 = zolo_P(*z, x1);
  z->M = 2.0L / (p0 + p1);
  z->delta = 1.0L - z->M * p0;
  // Proposition 1
  ld b[ZOLO_MAX_R];
  ld suma = 0.0L;
  for (int j = 1; j <= r - 1; ++j) {
    ld c2jm1 = z->c[2 * j - 2];
    ld prod = 1.0L;
    for (int k = 1; k <= r - 1; ++k)
      if (k != j) prod *= (z->c[2 * k - 1] - c2jm1) / (z->c[2 * k - 2] - c2jm1);
    b[j - 1] = (z->c[2 * j - 1] - c2jm1) * prod;
    z->a[j - 1] = b[j - 1] / (z->c[2 * r - 2] - c2jm1);
    suma += z->a[j - 1];
  }
  z->a[r - 1] = 1.0L - suma;
}

}  // namespace

int plan_filter(double am, double ap, double bm, double bp, int r1, int r2, double eps, zolo_filter_coeffs* out,
                char* err, size_t errlen) {
  std::memset(out, 0, sizeof(*out));
  bool inf_a = std::isinf(am), inf_b = std::isinf(bp);
  if (std::isnan(am) || std::isnan(ap) || std::isnan(bm) || std::isnan(bp) || (inf_a && inf_b) ||
      !(am < ap && ap < bm && bm < bp)) {
    snprintf(err, errlen, "eigengaps must satisfy a_- < a_+ < b_- < b_+ with at most one infinite end");
    return ZOLO_EINVAL;
  }
  if (r1 < 1 || r1 > ZOLO_MAX_R || r2 < 0 || r2 > ZOLO_MAX_R) {
    snprintf(err, errlen, "r1 must be in [1,%d] and r2 in [0,%d]", ZOLO_MAX_R, ZOLO_MAX_R);
    return ZOLO_EINVAL;
  }
  ld W = (ld)bm - (ld)ap;
  ld ga = inf_a ? 0.0L : (ld)ap - (ld)am;
  ld gb = inf_b ? 0.0L : (ld)bp - (ld)bm;
  ld e;
  if (inf_a)
    e = gb / W;
  else if (inf_b)
    e = ga / W;
  else
    e = ga * gb / (W * (W + ga + gb));
  ld s1 = sqrtl(1.0L + e) + 1.0L;
  ld l1 = e / (s1 * s1);
  if (!(l1 > 0.0L && l1 < 1.0L)) {
    snprintf(err, errlen, "degenerate eigengaps (l1 = %g)", (double)l1);
    return ZOLO_EINVAL;
  }
  ld alpha, beta, gamma;
  if (inf_a) {
    gamma = -l1;
    beta = (ld)bm + 2.0L * l1 * W / (1.0L - l1);
    alpha = (ld)ap - W * (1.0L + l1) / (1.0L - l1);
  } else if (inf_b) {
    gamma = -1.0L;
    alpha = (ld)ap - 2.0L * l1 * W / (1.0L - l1);
    beta = (ld)bm + W * (1.0L + l1) / (1.0L - l1);
  } else {
    ld t = 0.5L * (1.0L - l1);
    alpha = (ld)am + t * ga * ((ld)bm - (ld)am) / (W + t * ga);
    beta = (ld)bp - t * gb * ((ld)bp - (ld)ap) / (W + t * gb);
    gamma = -gb * (1.0L - t) * (W + t * ga) / ((W + t * gb) * (W + ga));
  }
  ZoloData in;
  zolo_make(r1, l1, &in);
  ld l2 = (1.0L - in.delta) / (1.0L + in.delta);
  ZoloData outz;
  if (r2 == 0) {
    int r;
    for (r = 1; r <= ZOLO_MAX_R; ++r) {
      zolo_make(r, l2, &outz);
      if (0.5L * outz.delta <= (ld)eps) break;
    }
    if (r > ZOLO_MAX_R) r = ZOLO_MAX_R;
    r2 = r;
  }
  zolo_make(r2, l2, &outz);
  out->r1 = r1;
  out->r2 = r2;
  out->a_minus = am;
  out->a_plus = ap;
  out->b_minus = bm;
  out->b_plus = bp;
  out->l1 = (double)l1;
  out->l2 = (double)l2;
  out->alpha = (double)alpha;
  out->beta = (double)beta;
  out->gamma = (double)gamma;
  out->delta1 = (double)in.delta;
  out->M_hat = (double)(in.M / (1.0L + in.delta));
  ld c0 = 0.0L;
  for (int j = 0; j < r1; ++j) {
    ld c = in.c[2 * j];
    ld sq = sqrtl(c);
    std::complex<ld> den(gamma, sq);
    std::complex<ld> sig = std::complex<ld>(gamma * alpha, sq * beta) / den;
    std::complex<ld> w = in.a[j] * (sig - std::complex<ld>(beta, 0.0L)) / (2.0L * den);
    out->sigma_hat_re[j] = (double)sig.real();
    out->sigma_hat_im[j] = (double)sig.imag();
    out->w_hat_re[j] = (double)w.real();
    out->w_hat_im[j] = (double)w.imag();
    out->a_hat[j] = (double)in.a[j];
    out->c_hat[j] = (double)c;
    c0 += in.a[j] * gamma / (gamma * gamma + c);
  }
  out->c0 = (double)c0;
  out->M = (double)outz.M;
  for (int j = 0; j < r2; ++j) {
    out->a[j] = (double)outz.a[j];
    out->c[j] = (double)outz.c[2 * j];
  }
  out->delta_S = (double)outz.delta;
  out->delta0 = 0.5 * (double)outz.delta;
  return ZOLO_OK;
}

// Comparison filters (Sec. 2.2, Figs. 2-3): quadratures of the contour integral
// (1/(2 pi i)) oint dz / (z - x) over the circle through a and b, centre c,
// radius rho, z(theta) = c + rho e^{i theta}.  A rule {theta_k, omega_k} in
// conjugate pairs gives, for real x, R(x) = sum over upper nodes of
// 2 Re(alpha_k / (z_k - x)) with alpha_k = omega_k rho e^{i theta_k} / (2 pi),
// which is the pole form g(x) = M_hat [c0 + sum 2 Re(w_hat_k / (x - sigma_hat_k))]
// with sigma_hat_k = z_k, w_hat_k = -alpha_k, c0 = 0, M_hat = 1.
//   kind 2, trapezoidal rule: p = 2 npole nodes theta_k = pi (2k + 1) / p,
//     weights 2 pi / p;
//   kind 3, Gauss-Legendre rule: npole nodes on the upper half-circle,
//     theta in (0, pi), and their mirror images.
// Legendre nodes by Newton's method on the three-term recurrence from the
// asymptotic guesses cos(pi (i + 3/4) / (q + 1/2)).
int plan_contour(int kind, double a, double b, int npole, zolo_filter_coeffs* out, char* err, size_t errlen) {
  std::memset(out, 0, sizeof(*out));
  if (!(a < b) || !std::isfinite(a) || !std::isfinite(b)) {
    snprintf(err, errlen, "contour filter: need finite a < b");
    return ZOLO_EINVAL;
  }
  if (npole < 1 || npole > ZOLO_MAX_R || (kind != 2 && kind != 3)) {
    snprintf(err, errlen, "contour filter: kind 2 or 3 and 1 <= poles <= %d", ZOLO_MAX_R);
    return ZOLO_EINVAL;
  }
  const ld pi = 3.14159265358979323846264338327950288L;
  const ld c = 0.5L * ((ld)a + (ld)b), rho = 0.5L * ((ld)b - (ld)a);
  ld theta[ZOLO_MAX_R], omega[ZOLO_MAX_R];
  const int q = npole;
  if (kind == 2) {
    const int p = 2 * q;
    for (int k = 0; k < q; ++k) {
      theta[k] = pi * (2.0L * k + 1.0L) / p;
      omega[k] = 2.0L * pi / p;
    }
  } else {
    for (int i = 0; i < q; ++i) {
      ld x = cosl(pi * (i + 0.75L) / (q + 0.5L));
      ld dp = 1.0L;
      for (int it = 0; it < 100; ++it) {
        ld p0 = 1.0L, p1 = x;  // P_0, P_1
        for (int m = 2; m <= q; ++m) {
          ld p2 = ((2.0L * m - 1.0L) * x * p1 - (m - 1.0L) * p0) / m;
          p0 = p1;
          p1 = p2;
        }
        if (q == 1) p1 = x, p0 = 1.0L;
        dp = q * (x * p1 - p0) / (x * x - 1.0L);  // P_q'
        ld dx = p1 / dp;
        x -= dx;
        if (fabsl(dx) < 1e-19L) break;
      }
      const ld w = 2.0L / ((1.0L - x * x) * dp * dp);
      theta[i] = 0.5L * pi * (x + 1.0L);  // [-1, 1] onto (0, pi)
      omega[i] = 0.5L * pi * w;
    }
  }
  out->kind = kind;
  out->r1 = q;
  out->r2 = 1;
  out->M_hat = 1.0;
  out->c0 = 0.0;
  out->a_minus = out->a_plus = out->b_minus = out->b_plus = NAN;
  for (int k = 0; k < q; ++k) {
    const std::complex<ld> e(cosl(theta[k]), sinl(theta[k]));
    const std::complex<ld> z = c + rho * e;
    const std::complex<ld> alpha = omega[k] * rho * e / (2.0L * pi);
    out->sigma_hat_re[k] = (double)z.real();
    out->sigma_hat_im[k] = (double)z.imag();
    out->w_hat_re[k] = -(double)alpha.real();
    out->w_hat_im[k] = -(double)alpha.imag();
  }
  return ZOLO_OK;
}

}  // namespace zolo
