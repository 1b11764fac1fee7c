"""Zolotarev coefficients in plain FP64 (oracle; test infrastructure only).

Paper: Li, Liu & Du, arXiv 1806.06204, Section 2.2.

* eq. (6): Z_{2r+1}(x; l) = M x prod_j (x^2 + c_{2j}) / (x^2 + c_{2j-1}).
* eq. (7): c_i = l^2 sn^2(i K'/(2r+1); l') / cn^2(i K'/(2r+1); l'),
  l' = sqrt(1 - l^2), K' = K(l') the complete elliptic integral of modulus l'.
* eq. (8): the scaled function Zhat = Z / Z(1) = Mhat x prod(...),
  Mhat = prod_j (1 + c_{2j-1}) / (1 + c_{2j}).
* eqs. (9)-(10) (Theorem 2.1): Zhat(x) = Mhat x (1 + sum_j a_j/(x^2 + c_{2j-1})).
  The paper prints a_j as a product of the two products; the partial-fraction
  identity (9) only holds for their quotient
      a_j = - prod_k (c_{2j-1} - c_{2k}) / prod_{k != j} (c_{2j-1} - c_{2k-1}),
  which is the residue of prod(t + c_{2k})/(t + c_{2k-1}) at t = -c_{2j-1}.
* Algorithm 1 step 4(c): l <- Zhat(l; l).  The printed update has (l + c_{2j})
  in the numerator; Zhat evaluated at x = l has (l^2 + c_{2j}), which is what
  reproduces Table 1, so that is the reading taken here.
* Table 1: the iteration count k is the smallest k with
  Zhat composed k times mapping [1/kappa, 1] into [1 - 1e-15, 1], evaluated
  through the scalar recursion l_{k+1} = Zhat(l_k; l_k) from l_0 = 1/kappa.

Evaluation of eq. (7).  Computing sn/cn with parameter m = l'^2 loses all
accuracy when l is tiny, because l' rounds to 1.  Instead the ratio sn/cn is
written with Jacobi theta functions whose nome is small on both halves of the
range, so every term is a plain exponential:

* l <= 1/sqrt(2): with the imaginary transformation sc(u; l') = -i sn(iu; l)
  and sn = (theta3/theta2) theta1/theta4 (theta3^2/theta2^2 = 1/l), nome
  q = exp(-pi K'/K) with K = K(l), and y = pi u / (2K):
      c_i = 4 l (S/C)^2,
      S = sum_{n>=0} (-1)^n q^{(n+1/2)^2} sinh((2n+1) y),
      C = 1 + 2 sum_{n>=1} (-1)^n q^{n^2} cosh(2 n y).
* l > 1/sqrt(2): sc(u; l') = (theta3/theta4)(0) theta1/theta2 with nome
  q' = exp(-pi K/K'), theta3/theta4 = 1/sqrt(l), and v = pi u / (2 K') =
  i pi / (2(2r+1)):
      c_i = l (S'/C')^2,
      S' = sum (-1)^n q'^{(n+1/2)^2} sin((2n+1) v),
      C' = sum q'^{(n+1/2)^2} cos((2n+1) v).

K and K' come from the arithmetic-geometric mean, K(k) = pi / (2 AGM(1, k')).
Both nomes are at most exp(-pi), so a handful of terms reach full precision.
Only c_1..c_r are evaluated this way; the rest follow from the reflection
c_i c_{2r+1-i} = l^2, which holds because sn(K'-u)=cd(u) and cn(K'-u)=l sd(u)
for modulus l'.

Evaluation of the l-update near 1.  Once Zhat(l; l) is within ~1e-3 of 1 the
product form loses digits of 1 - Zhat (Table 1 asks for 1 - l_k <= 1e-15,
about 9 ulps).  One step of Zolo-PD acts on the modulus as the degree-(2r+1)
modular transformation: the nome of the complementary modulus of the new l is
q'^(2r+1).  So l'_new = theta2(q1)^2 / theta3(q1)^2 with q1 = q'^(2r+1), and
1 - l_new = l'_new^2 / (1 + l_new) carries no cancellation.  Both forms are
evaluations of the same number Zhat(l; l).
"""

import math

import numpy as np

L_MIN = 1e-20          # smallest l accepted (c_1 ~ l^2 nears underflow below)
CONVERGED = 1.0 - 1e-15  # Table 1 threshold: Zhat^k([1/kappa,1]) in [1-1e-15, 1]
N_THETA = 10           # theta-series terms; the nome is <= exp(-pi)


def agm(a, b):
    """Arithmetic-geometric mean of two non-negative numbers."""
    a = float(a)
    b = float(b)
    for _ in range(64):
        if abs(a - b) <= 1e-16 * a:
            break
        a, b = 0.5 * (a + b), math.sqrt(a * b)
    return 0.5 * (a + b)


def complementary(l):
    """l' = sqrt(1 - l^2) without cancellation near l = 1."""
    return math.sqrt((1.0 - l) * (1.0 + l))


def ellipk_pair(l):
    """(K, K') = (K(l), K(l')) with K(k) = integral_0^{pi/2} (1-k^2 sin^2)^{-1/2}.

    K' is the quarter period that appears in eq. (7)."""
    lp = complementary(l)
    kp = math.pi / (2.0 * agm(1.0, l))            # K(l') = pi / (2 AGM(1, l))
    k = math.inf if lp == 0.0 else math.pi / (2.0 * agm(1.0, lp))
    return k, kp


def _check(l, r):
    if not (r >= 1 and int(r) == r):
        raise ValueError("r must be a positive integer")
    if not (0.0 < l <= 1.0) or math.isnan(l):
        raise ValueError("l must lie in (0, 1]")


def zolo_c(l, r):
    """c_1..c_{2r} of eq. (7), returned as a length-2r array (index i-1)."""
    _check(l, r)
    r = int(r)
    l = max(float(l), L_MIN)
    c = np.empty(2 * r)
    big_k, kp = ellipk_pair(l)
    for i in range(1, r + 1):
        u = i * kp / (2 * r + 1)
        if l <= 1.0 / math.sqrt(2.0):
            lnq = -math.pi * kp / big_k
            y = math.pi * u / (2.0 * big_k)
            s = 0.0
            for n in range(N_THETA):
                e = lnq * (n + 0.5) ** 2
                s += (-1) ** n * 0.5 * (math.exp(e + (2 * n + 1) * y)
                                        - math.exp(e - (2 * n + 1) * y))
            cc = 1.0
            for n in range(1, N_THETA):
                e = lnq * n * n
                cc += (-1) ** n * (math.exp(e + 2 * n * y) + math.exp(e - 2 * n * y))
            c[i - 1] = 4.0 * l * (s / cc) ** 2
        else:
            # q' = exp(-pi K / K').  The common factor q'^(1/4) cancels in
            # S'/C', leaving weights q'^(n(n+1)); at l = 1 (K infinite) only
            # n = 0 survives and c_i = tan^2(v), the l -> 1 limit.
            v = i * math.pi / (2.0 * (2 * r + 1))
            s = math.sin(v)
            cc = math.cos(v)
            if not math.isinf(big_k):
                lnq = -math.pi * big_k / kp
                for n in range(1, N_THETA):
                    w = math.exp(lnq * n * (n + 1))
                    s += (-1) ** n * w * math.sin((2 * n + 1) * v)
                    cc += w * math.cos((2 * n + 1) * v)
            c[i - 1] = l * (s / cc) ** 2
    for i in range(r + 1, 2 * r + 1):          # reflection c_i c_{2r+1-i} = l^2
        c[i - 1] = l * l / c[2 * r - i]
    return c


def zolo_a(c):
    """a_1..a_r of eq. (10), as the quotient (see module docstring)."""
    r = len(c) // 2
    a = np.empty(r)
    for j in range(1, r + 1):
        codd = c[2 * j - 2]                      # c_{2j-1}
        val = -(codd - c[2 * j - 1])            # k = j factor of the numerator
        for k in range(1, r + 1):
            if k != j:
                val *= (codd - c[2 * k - 1]) / (codd - c[2 * k - 2])
        a[j - 1] = val
    return a


def zolo_mhat(c):
    """Mhat = prod_j (1 + c_{2j-1}) / (1 + c_{2j}) of eq. (8)."""
    r = len(c) // 2
    m = 1.0
    for j in range(1, r + 1):
        m *= (1.0 + c[2 * j - 2]) / (1.0 + c[2 * j - 1])
    return m


def zhat(x, c, mhat=None):
    """Zhat(x) in product form, eq. (8); x may be an array."""
    r = len(c) // 2
    if mhat is None:
        mhat = zolo_mhat(c)
    x = np.asarray(x, dtype=np.float64)
    x2 = x * x
    f = mhat * x
    for j in range(1, r + 1):
        f = f * (x2 + c[2 * j - 1]) / (x2 + c[2 * j - 2])
    return f


def zhat_partial_fractions(x, c, a, mhat):
    """Zhat(x) in partial-fraction form, eq. (9)."""
    x = np.asarray(x, dtype=np.float64)
    x2 = x * x
    s = np.ones_like(x2)
    for j in range(len(a)):
        s = s + a[j] / (x2 + c[2 * j])
    return mhat * x * s


def one_minus_l_next(l, r):
    """1 - Zhat(l; l) via the nome q1 = q'^(2r+1) (see module docstring)."""
    _check(l, r)
    l = max(float(l), L_MIN)
    big_k, kp = ellipk_pair(l)
    if math.isinf(big_k):
        return 0.0
    lnq1 = -(2 * int(r) + 1) * math.pi * big_k / kp
    th2 = 2.0 * math.exp(lnq1 / 4.0) * sum(math.exp(lnq1 * n * (n + 1)) for n in range(30))
    th3 = 1.0 + 2.0 * sum(math.exp(lnq1 * n * n) for n in range(1, 30))
    lp1 = (th2 / th3) ** 2
    l1 = complementary(lp1)
    return lp1 * lp1 / (1.0 + l1)


def coefficients(l, r):
    """All per-iteration scalars for (l, r): dict with c, a, mhat, l_next.

    l_next = Zhat(l; l), the l-update of Algorithm 1 step 4(c) (read with
    l^2 + c_{2j}, see the module docstring)."""
    c = zolo_c(l, r)
    a = zolo_a(c)
    mhat = zolo_mhat(c)
    l_eff = max(float(l), L_MIN)
    l_next = float(zhat(l_eff, c, mhat))
    if 1.0 - l_next < 1e-3:
        l_next = 1.0 - one_minus_l_next(l_eff, r)
    return {"c": c, "a": a, "mhat": mhat, "l_next": min(l_next, 1.0)}


def iterations_to_converge(kappa, r, max_iter=50):
    """Table 1 entry: smallest k with l_k >= 1 - 1e-15, l_0 = 1/kappa."""
    l = 1.0 / kappa
    k = 0
    while l < CONVERGED:
        l = coefficients(l, r)["l_next"]
        k += 1
        if k >= max_iter:
            break
    return k


def choose_r(l, max_r=8, max_iters=2):
    """Smallest r in [1, max_r] whose scalar recursion converges in at most
    max_iters steps from l (Section 2.2: choose r so that at most two
    iterations are needed).  Returns max_r if none does."""
    for r in range(1, max_r + 1):
        if iterations_to_converge(1.0 / l, r, max_iter=max_iters + 1) <= max_iters:
            return r
    return max_r


def z_condition_bound(l, c):
    """max_j kappa(X^T X + c_{2j-1} I) for singular values of X in [l, 1]:
    (1 + c_1) / (l^2 + c_1), attained for the smallest shift c_1."""
    return (1.0 + c[0]) / (l * l + c[0])
