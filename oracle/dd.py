"""Domain decomposition for entropic unbalanced OT on 2-D grids (oracle, FP64).

TEST INFRASTRUCTURE ONLY (see the package header).

Follows Sec. 3 (Definitions basic/composite partitions and cell subproblem,
Algorithm 3 sequential and Algorithm 4 parallel DomDecIter, Algorithm 2 outer
loop) and Sec. 4.1/4.4 (cell Sinkhorn with the Newton Y-update, nu_{-J} from the
aggregated Y-marginal, truncation of basic-cell marginals, bounding boxes,
padded B partition, PD stopping rule, GetWeights variants of Sec. 3.4).

Every cell problem is solved densely: an explicit |X_J| x |box_J| cost matrix
and library log-sum-exp.  Readings of points the paper leaves open (all of
them also fixed in the design notes):

  R1 grid: x = h (i1, i2); cost c = |x - y|^2, so c = h^2 |i - j|^2.
  R2 partitions: basic cells are s1 x s2 blocks; partition A groups 2 x 2
     basic cells from the origin, B is offset by one basic cell; the B cells
     at the border contain only the basic cells that exist (padding of X only).
     An axis with a single basic cell is not paired.
  R3 state: the basic-cell Y-marginals nu_i stored on bounding boxes, plus the
     X-marginal P_X pi, plus per basic cell a tracked score Hbar_i and the
     last cell potential alpha (stitched).
  R4 cell Y-domain: Sec. 4.1 keeps the cell problem on the (sparse) support
     of nu_J = sum of the basic marginals of J, whatever its extent; it is
     stored as a box, the bbox of the union of the basic boxes of J dilated by
     the margin M per axis and clipped to the grid, and (support = True, the
     paper's rule) the points of the box where nu_J = 0 are left out of the
     cell problem, so supports grow only through the alternation of the
     partitions.  support = False solves on the whole box (the margin then
     lets supports grow by M per step).  An all-empty union uses the X
     rectangle of J, with the whole box as domain.
  R5 warm start (the paper only says "for a given initialization beta^0"):
     when every basic cell of J holds a stored X-potential (the stitched
     alpha of the last solve covering it, of a refinement or of a potential
     start), the solve starts from alpha^0 = that alpha on X_J with a
     Y-half; otherwise beta^0 = -lam log(P_Y pi / nu) on the box (0 where
     P_Y pi = 0), i.e. the Y optimality condition eq.
     (optimality-conditions-KL) evaluated for the current plan, followed by
     an X-half.  (beta^0 carries lam/eps times the relative error of P_Y pi,
     10^6 on the finest grids; alpha^0 carries no such factor.)  beta^0 also
     enters the first translation step (R6).
  R6 inner loop: X-half, then repeat {Y-half (Newton), X-half, PD check};
     with `translate`, every Y-half is preceded by the exact maximisation of
     the cell dual along (alpha + s, beta - s), which has the closed form
     e^{s/lam} = (R + sqrt(R^2 + 4AB)) / (2B), A = sum e^{-alpha/lam} mu_J,
     B = sum e^{-beta/lam} nu, R = |nu_{-J}| (a dual ascent step that removes
     the slowly contracting constant mode; not part of the paper);
     the cell solve ends after a Y-half, the final pair is the alpha used in
     that Y-half and the new beta.  Stop when PD_J / lam <= Err |mu_J|
     (per-cell rule), or after exactly `fixed_iters` Y-halves (parity mode),
     or at `max_iter`.
  R7 truncation: after the re-split and again after mixing, entries below
     `trunc` are set to 0 and the box shrinks to the bbox of the nonzeros.
  R8 tracked score: Ebar = sum_i Hbar_i + lam KL(P_Y pi | nu); Hbar_i is the
     exact cell-restricted score of a diagonal-scaling plan and is mixed with
     the same weights as the plans, so Ebar >= E with equality after greedy
     steps (convexity of each term).
  R9 GetWeights: greedy theta = 1; safe theta = 1/n with n the number of cells
     updated in the step; swift takes greedy iff
     Ebar_greedy <= Ebar_cur + lenience |Ebar_cur|, else safe; staggered runs
     the partition as four batches of non-adjacent cells (parity of the cell
     position), one swift step each, in batch order.
  R10 multiscale refinement (warm start of a finer layer): see `refine`.
  R12 GetWeights `line` on the tracked score: see `line_weight`.
  R14 GetWeights `opt` on the tracked score: see `opt_weights`.
  R13 balancing step: see `balance_cell`.
  R11 global Sinkhorn warm start: the coarse layers are solved by the global
     Sinkhorn iteration (uot.sinkhorn), each warm-started from the previous
     layer's beta (`interpolate_potential`); the plan of the last global
     layer's potentials is split by basic cells (`init_from_duals`) and
     refined to the first DD layer by `refine` (R10).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from . import uot


# --------------------------------------------------------------------------
# problem, options, partitions
# --------------------------------------------------------------------------
@dataclass
class Problem:
    mu: np.ndarray            # (n1, n2) point masses, > 0
    nu: np.ndarray            # (n1, n2) point masses, > 0
    eps: float
    lam: float
    h: float
    s1: int                   # basic cell sides
    s2: int
    ypos: np.ndarray | None = None   # (n1, n2, 2) moved Y points y'; None = the grid

    @property
    def n1(self):
        return self.mu.shape[0]

    @property
    def n2(self):
        return self.mu.shape[1]

    @property
    def nb1(self):
        return self.n1 // self.s1

    @property
    def nb2(self):
        return self.n2 // self.s2


@dataclass
class Options:
    err: float = 2e-5          # Err of Sec. 4.4
    max_iter: int = 1000
    fixed_iters: int = 0       # > 0: exactly this many Y-halves per cell
    trunc: float = 1e-15       # Sec. 4.4
    lenience: float = 0.0      # 0.005 in Sec. 4.4; 0 = strict
    margin: int = 2
    getweights: str = "swift"  # greedy | safe | swift | staggered | line | opt
    support: bool = True       # cell problem on the support of nu_J (R4)
    translate: bool = False    # dual line search along (alpha + s, beta - s)
    balance: bool = False      # balancing step of Sec. 4.1 (reading R13)


def make_problem(mu, nu, eps, lam, h, s1, s2=None, ypos=None) -> Problem:
    """ypos: optional (n1, n2, 2) coordinates y' of the Y points (a displaced
    support, cost |x - y'|^2); the index structure (boxes, cells) stays that
    of the grid."""
    s2 = s1 if s2 is None else s2
    mu = np.asarray(mu, dtype=np.float64)
    nu = np.asarray(nu, dtype=np.float64)
    if mu.shape != nu.shape or mu.ndim != 2:
        raise ValueError("mu and nu must be 2-D arrays of one shape")
    if not (np.all(mu > 0) and np.all(nu > 0)):
        raise ValueError("full support required (Assumption 2)")
    n1, n2 = mu.shape
    if n1 % s1 or n2 % s2:
        raise ValueError("grid not divisible by the basic cell size")
    if ypos is not None:
        ypos = np.asarray(ypos, dtype=np.float64)
        if ypos.shape != (n1, n2, 2):
            raise ValueError("ypos must have shape (n1, n2, 2)")
    return Problem(mu, nu, float(eps), float(lam), float(h), int(s1), int(s2), ypos)


def basic_rect(p: Problem, b: int):
    """X rectangle (o1, o2, l1, l2) of basic cell b = b1*nb2 + b2."""
    b1, b2 = divmod(b, p.nb2)
    return (b1 * p.s1, b2 * p.s2, p.s1, p.s2)


def _axis_groups(nb: int, offset: bool):
    """Groups of basic indices along one axis: pairs from 0 (A) or pairs
    offset by one with singletons at both ends (B).  A single basic cell is
    never paired."""
    if nb == 1:
        return [[0]]
    if not offset:
        return [[2 * a, 2 * a + 1] for a in range(nb // 2)]
    groups = []
    for c in range(nb // 2 + 1):
        g = [b for b in (2 * c - 1, 2 * c) if 0 <= b < nb]
        groups.append(g)
    return groups


def composite_cells(p: Problem, part: str):
    """Composite cells of partition 'A' or 'B' in row-major order.  Each is a
    dict with the ordered basic ids and the X rectangle (o1, o2, l1, l2)."""
    off = part == "B"
    g1 = _axis_groups(p.nb1, off)
    g2 = _axis_groups(p.nb2, off)
    cells = []
    for r in g1:
        for c in g2:
            basic = [b1 * p.nb2 + b2 for b1 in r for b2 in c]
            rect = (r[0] * p.s1, c[0] * p.s2, len(r) * p.s1, len(c) * p.s2)
            cells.append(dict(basic=basic, rect=rect))
    return cells


def rect_index(rect, n2):
    """Flat grid indices of a rectangle, row-major."""
    o1, o2, l1, l2 = rect
    i1, i2 = np.meshgrid(np.arange(o1, o1 + l1), np.arange(o2, o2 + l2), indexing="ij")
    return (i1 * n2 + i2).ravel()


def rect_coords(rect, h):
    o1, o2, l1, l2 = rect
    i1, i2 = np.meshgrid(np.arange(o1, o1 + l1), np.arange(o2, o2 + l2), indexing="ij")
    return h * np.stack([i1.ravel(), i2.ravel()], axis=1).astype(np.float64)


def y_coords(p: Problem, yrect):
    """Coordinates of the Y points of a rectangle: the grid, or the moved
    points y' when the problem has them."""
    if p.ypos is None:
        return rect_coords(yrect, p.h)
    o1, o2, l1, l2 = yrect
    return p.ypos[o1:o1 + l1, o2:o2 + l2].reshape(-1, 2)


def rect_cost(p: Problem, xrect, yrect):
    """Dense cost matrix c(x, y) = |x - y|^2 between two rectangles."""
    return uot.sq_cost(rect_coords(xrect, p.h), y_coords(p, yrect))


def full_cost(p: Problem):
    """Dense cost between all X and all Y points (small grids only)."""
    full = (0, 0, p.n1, p.n2)
    return rect_cost(p, full, full)


# --------------------------------------------------------------------------
# state
# --------------------------------------------------------------------------
@dataclass
class State:
    boxes: list               # per basic cell: (o1, o2, arr (L1, L2))
    px: np.ndarray            # (n1, n2) X-marginal of the plan
    hbar: np.ndarray          # (nbasic,) tracked cell-restricted scores
    abar: np.ndarray          # (n1, n2) last cell potential alpha
    plan: np.ndarray | None = None   # dense plan (tiny problems only)
    warm: np.ndarray | None = None   # (nbasic,) abar holds a potential on X_i (R5)
    k: int = 0                # half-iterations done
    force_greedy: bool = False
    history: list = field(default_factory=list)


def cell_piece(pi_box, mu_x, nu_box, nu_total, c_box, eps, lam) -> float:
    """Score of a cell-restricted plan supported on X_i x box (definition):
    <c,pi> + eps KL(pi | mu_i x nu) + lam KL(P_X pi | mu_i), where the KL over
    X_i x Y counts the "+1" term mu_i(x) nu(y) also outside the box."""
    prod = np.outer(mu_x, nu_box)
    outside = mu_x.sum() * (nu_total - nu_box.sum())
    return (float((c_box * pi_box).sum()) + eps * (uot.kl(pi_box, prod) + outside)
            + lam * uot.kl(pi_box.sum(1), mu_x))


def _embed_full(p: Problem, rect, arr):
    full = np.zeros((p.n1, p.n2))
    o1, o2, l1, l2 = rect
    full[o1:o1 + l1, o2:o2 + l2] = arr
    return full


def init_product(p: Problem, dense_plan: bool = False) -> State:
    """pi^0 = mu x nu (the toy initialisation of Sec. 4.2): nu_i = |mu_i| nu on
    the whole grid, P_X pi = |nu| mu."""
    nbasic = p.nb1 * p.nb2
    nu_tot = p.nu.sum()
    full = (0, 0, p.n1, p.n2)
    boxes, hbar = [], np.zeros(nbasic)
    for b in range(nbasic):
        rect = basic_rect(p, b)
        mu_x = p.mu.ravel()[rect_index(rect, p.n2)]
        boxes.append((0, 0, mu_x.sum() * p.nu.copy()))
        pi_box = np.outer(mu_x, p.nu.ravel())
        hbar[b] = cell_piece(pi_box, mu_x, p.nu.ravel(), nu_tot,
                             rect_cost(p, rect, full), p.eps, p.lam)
    st = State(boxes, nu_tot * p.mu.copy(), hbar, np.zeros_like(p.mu))
    if dense_plan:
        st.plan = np.outer(p.mu.ravel(), p.nu.ravel())
    return st


def init_block(p: Problem, dense_plan: bool = False) -> State:
    """Block-diagonal start: pi^0 restricted to X_i x Y is mu_i x (nu on X_i)
    divided by |mu_i|, so nu_i = nu restricted to the block X_i (box = block),
    P_Y pi = nu, and P_X pi = mu |nu(X_i)| / |mu_i| on X_i."""
    nbasic = p.nb1 * p.nb2
    nu_tot = p.nu.sum()
    boxes, hbar = [], np.zeros(nbasic)
    px = np.zeros_like(p.mu)
    plan = np.zeros((p.n1 * p.n2, p.n1 * p.n2)) if dense_plan else None
    for b in range(nbasic):
        rect = basic_rect(p, b)
        o1, o2, l1, l2 = rect
        idx = rect_index(rect, p.n2)
        mu_x = p.mu.ravel()[idx]
        nu_b = p.nu.ravel()[idx]
        boxes.append((o1, o2, p.nu[o1:o1 + l1, o2:o2 + l2].copy()))
        pi_box = np.outer(mu_x, nu_b) / mu_x.sum()
        px.ravel()[idx] = pi_box.sum(1)
        hbar[b] = cell_piece(pi_box, mu_x, nu_b, nu_tot, rect_cost(p, rect, rect),
                             p.eps, p.lam)
        if plan is not None:
            plan[np.ix_(idx, idx)] = pi_box
    return State(boxes, px, hbar, np.zeros_like(p.mu), plan)


def aggregate(p: Problem, boxes) -> np.ndarray:
    """P_Y pi = sum_i nu_i (Sec. 4.1, computing nu_{-J})."""
    P = np.zeros((p.n1, p.n2))
    for o1, o2, arr in boxes:
        P[o1:o1 + arr.shape[0], o2:o2 + arr.shape[1]] += arr
    return P


def tracked_score(p: Problem, st: State, P=None) -> float:
    """Ebar = sum_i Hbar_i + lam KL(P_Y pi | nu)   (reading R8)."""
    if P is None:
        P = aggregate(p, st.boxes)
    return float(st.hbar.sum()) + p.lam * uot.kl(P, p.nu)


def exact_score(p: Problem, st: State) -> float:
    """E(pi) of the dense plan (Definition unbalanced-entropic-transport)."""
    c = full_cost(p)
    return uot.primal(st.plan, p.mu, p.nu, c, p.eps, p.lam)


# --------------------------------------------------------------------------
# one cell
# --------------------------------------------------------------------------
def cell_box(p: Problem, cell, boxes, opt: Options):
    """Y-box of composite cell J (reading R4): (o1, o2, L1, L2)."""
    rect = cell["rect"]
    los, his = [], []
    for b in cell["basic"]:
        o1, o2, arr = boxes[b]
        if arr.size:
            los.append((o1, o2))
            his.append((o1 + arr.shape[0], o2 + arr.shape[1]))
    if los:
        lo = [min(v[0] for v in los), min(v[1] for v in los)]
        hi = [max(v[0] for v in his), max(v[1] for v in his)]
    else:
        lo = [rect[0], rect[1]]
        hi = [rect[0] + rect[2], rect[1] + rect[3]]
    out = []
    for ax, n in ((0, p.n1), (1, p.n2)):
        out.append((max(lo[ax] - opt.margin, 0), min(hi[ax] + opt.margin, n)))
    return (out[0][0], out[1][0], out[0][1] - out[0][0], out[1][1] - out[1][0])


def translation_shift(alpha, beta, mu_x, nu_y, r_y, lam):
    """Maximiser s of the cell dual D_J(alpha + s, beta - s | nu_{-J}).  Along
    this direction the plan is fixed and D changes by
    -lam (e^{-s/lam} - 1) A - lam (e^{s/lam} - 1) B + s R, whose stationary
    point solves B w^2 - R w - A = 0 for w = e^{s/lam}."""
    A = float((np.exp(-alpha / lam) * mu_x).sum())
    B = float((np.exp(-beta / lam) * nu_y).sum())
    R = float((r_y * nu_y).sum())
    w = (R + np.sqrt(R * R + 4.0 * A * B)) / (2.0 * B)
    return lam * np.log(w)


def solve_cell(mu_x, nu_y, r_y, beta0, C, eps, lam, tol, opt: Options, alpha0=None):
    """Cell Sinkhorn of Sec. 4.1 (reading R6).

    alpha from eq. (sinkhorn-X-iteration); beta from eq. (proxdiv-problem)
    with r = d nu_{-J} / d nu; PD from eq. (PD-gap-KL).  alpha0 (reading R5):
    start from this alpha instead of the X-half of beta0.
    Returns dict(alpha, beta, px, iters, converged, pd)."""
    with np.errstate(divide="ignore"):
        lr = np.log(r_y)
    beta = beta0.copy()
    alpha = uot.x_update(beta, nu_y, C, eps, lam) if alpha0 is None else alpha0.copy()
    it, pd, conv = 0, np.inf, False
    while True:
        it += 1
        if opt.translate:
            sh = translation_shift(alpha, beta, mu_x, nu_y, r_y, lam)
            alpha = alpha + sh
            beta = beta - sh
        z = uot.y_log_integral(alpha, mu_x, C, eps)
        beta, _ = uot.y_update_root(z, lr, eps, lam)
        alpha_next = uot.x_update(beta, nu_y, C, eps, lam)
        px = uot.plan(alpha, beta, mu_x, nu_y, C, eps).sum(1)
        pd = uot.pd_gap_kl(alpha, px, mu_x, lam) / lam
        conv = pd <= tol
        if opt.fixed_iters > 0:
            if it >= opt.fixed_iters:
                break
        elif conv or it >= opt.max_iter:
            break
        alpha = alpha_next
    return dict(alpha=alpha, beta=beta, px=px, iters=it, converged=bool(conv), pd=pd)


def cell_inputs(p: Problem, cell, box, boxes, P):
    """nu_J, nu_{-J} = P_Y pi - nu_J (Sec. 4.1, clamped at 0), r = nu_{-J}/nu and
    the warm start beta^0 of reading R5, all on the cell Y-box.  Returns
    (r, beta^0, nu_J), flattened."""
    o1, o2, L1, L2 = box
    nuJ = np.zeros((L1, L2))
    for b in cell["basic"]:
        bo1, bo2, arr = boxes[b]
        if arr.size:
            nuJ[bo1 - o1:bo1 - o1 + arr.shape[0], bo2 - o2:bo2 - o2 + arr.shape[1]] += arr
    Pb = P[o1:o1 + L1, o2:o2 + L2]
    nub = p.nu[o1:o1 + L1, o2:o2 + L2]
    r = np.maximum(Pb - nuJ, 0.0) / nub
    with np.errstate(divide="ignore"):
        beta0 = np.where(Pb > 0, -p.lam * np.log(Pb / nub), 0.0)
    return r.ravel(), beta0.ravel(), nuJ.ravel()


def balance_cell(p: Problem, cell, sol, pi, mu_x, nu_y, C, rows_of):
    """Balancing step (Sec. 4.1 "Balancing", reading R13).  One more X-half
    of the final beta gives mubar = e^{-alpha'/lam} mu; basic cell i should
    carry m_i = mubar(X_i) |nu_J| / mubar(X_J).  Mass moves horizontally
    (same y) inside the cell: every donor (|nu_i| > m_i) keeps the fraction
    m_i / |nu_i| of its plan, the removed profile R(y) = sum of the donors'
    (1 - m_i/|nu_i|) nu_i(y) goes to the receivers in proportion to their
    deficits, and a receiver spreads what it gets at y over its rows like
    its own plan column, i.e. with the cell kernel e^{(alpha(x) - c)/eps}
    mu(x) restricted to X_j and normalised.  nu_J stays unchanged."""
    a2 = uot.x_update(sol["beta"], nu_y, C, p.eps, p.lam)
    mubar = np.exp(-a2 / p.lam) * mu_x
    basics = cell["basic"]
    M = {b: pi[rows_of[b]].sum() for b in basics}
    tot = sum(M.values())
    mtot = mubar.sum()
    if not (tot > 0.0 and mtot > 0.0):
        return pi
    m = {b: mubar[rows_of[b]].sum() * tot / mtot for b in basics}
    e = {b: M[b] - m[b] for b in basics}
    E = sum(v for v in e.values() if v > 0.0)
    if not (E > 0.0):
        return pi
    pi = pi.copy()
    R = np.zeros(pi.shape[1])
    for b in basics:
        if e[b] > 0.0:
            R += (e[b] / M[b]) * pi[rows_of[b]].sum(0)
            pi[rows_of[b]] *= m[b] / M[b]
    for b in basics:
        if e[b] < 0.0:
            rows = rows_of[b]
            lk = (sol["alpha"][rows][:, None] - C[rows]) / p.eps + np.log(mu_x[rows])[:, None]
            lk -= lk.max(0)[None, :]
            k = np.exp(lk)
            pi[rows] += (-e[b] / E) * R[None, :] * k / k.sum(0)[None, :]
    return pi


def process_cell(p: Problem, cell, boxes, P, opt: Options, abar=None, warm=None):
    """Solve one composite cell and re-split its plan into basic cells.

    abar, warm: the stitched X-potential and its per-basic-cell validity
    (warm start of reading R5; None: the beta^0 start).  Returns a dict with
    the box, its domain mask `dom` (R4), the cell potentials and plan on the
    domain, the candidate basic marginals on the box (untruncated), their
    pieces H_i (definition cell_piece), P_X of the cell plan, iteration
    count."""
    box = cell_box(p, cell, boxes, opt)
    rect = cell["rect"]
    xi = rect_index(rect, p.n2)
    yi = rect_index(box, p.n2)
    C = rect_cost(p, rect, box)
    r, beta0, nuJ = cell_inputs(p, cell, box, boxes, P)
    # the cell's Y-domain (R4): the support of nu_J inside the box
    dom = nuJ > 0 if (opt.support and np.any(nuJ > 0)) else np.ones(nuJ.size, dtype=bool)
    yi, C, r, beta0 = yi[dom], C[:, dom], r[dom], beta0[dom]
    mu_x = p.mu.ravel()[xi]
    nu_y = p.nu.ravel()[yi]
    tol = opt.err * mu_x.sum()
    alpha0 = None
    if abar is not None and warm is not None and all(warm[b] for b in cell["basic"]):
        alpha0 = np.ravel(abar)[xi]
    sol = solve_cell(mu_x, nu_y, r, beta0, C, p.eps, p.lam, tol, opt, alpha0)
    pi = uot.plan(sol["alpha"], sol["beta"], mu_x, nu_y, C, p.eps)
    nu_tot = p.nu.sum()
    cand, pieces = {}, {}
    rows_of = {b: np.isin(xi, rect_index(basic_rect(p, b), p.n2)) for b in cell["basic"]}
    if opt.balance and len(cell["basic"]) > 1:
        pi = balance_cell(p, cell, sol, pi, mu_x, nu_y, C, rows_of)
    for b in cell["basic"]:
        rows = rows_of[b]
        pib = pi[rows]
        nut = np.zeros(box[2] * box[3])
        nut[dom] = pib.sum(0)
        pieces[b] = cell_piece(pib, mu_x[rows], nu_y, nu_tot, C[rows], p.eps, p.lam)
        cand[b] = nut.reshape(box[2], box[3])
    return dict(box=box, rect=rect, xi=xi, yi=yi, dom=dom, alpha=sol["alpha"], beta=sol["beta"],
                px=pi.sum(1), pi=pi, cand=cand, pieces=pieces, iters=sol["iters"],
                converged=sol["converged"], pd=sol["pd"])


def truncate_to_box(o1, o2, arr, trunc):
    """Entries below `trunc` -> 0, then shrink to the bbox of the nonzeros
    (reading R7).  An all-zero array becomes an empty box at (o1, o2)."""
    arr = np.where(arr < trunc, 0.0, arr)
    nz = np.argwhere(arr > 0)
    if nz.size == 0:
        return (o1, o2, np.zeros((0, 0)))
    a1, a2 = nz.min(0)
    b1, b2 = nz.max(0) + 1
    return (o1 + int(a1), o2 + int(a2), arr[a1:b1, a2:b2].copy())


def _on_box(entry, box):
    o1, o2, L1, L2 = box
    out = np.zeros((L1, L2))
    bo1, bo2, arr = entry
    if arr.size:
        out[bo1 - o1:bo1 - o1 + arr.shape[0], bo2 - o2:bo2 - o2 + arr.shape[1]] = arr
    return out


# --------------------------------------------------------------------------
# Algorithm 4 (parallel) and Algorithm 3 (sequential)
# --------------------------------------------------------------------------
def staggered_batches(p: Problem, part: str):
    """The composite cells of a partition in 2^d = 4 batches by the parity of
    their position in the partition's cell grid, so that no batch holds two
    adjacent composite cells (Sec. 3.4 `staggered`, Sec. 4.4)."""
    off = part == "B"
    n2g = len(_axis_groups(p.nb2, off))
    batches = [[], [], [], []]
    for idx, c in enumerate(composite_cells(p, part)):
        ga, gb = divmod(idx, n2g)
        batches[(ga % 2) * 2 + (gb % 2)].append(c)
    return batches


def line_weight(p: Problem, P, Pg, dH: float, n_upd: int) -> float:
    """GetWeights `line` (Proposition converging-getweights) on the tracked
    score (reading R12): one weight z for every updated cell, minimising
        f(z) = sum Hbar + z dH + lam KL((1 - z) P + z Pg | nu)
    over [1/n, 1] (the mixed pieces are linear in z, the KL term convex).
    The minimiser is an endpoint or the root of
        f'(z) = dH + lam sum (Pg - P) log(P_z / nu),
    found by bracketed root finding."""
    from scipy.optimize import brentq
    lo = 1.0 / max(n_upd, 1)
    D = (Pg - P).ravel()
    m = D != 0.0
    D, P0, nu = D[m], P.ravel()[m], p.nu.ravel()[m]

    def fprime(z):
        with np.errstate(divide="ignore", invalid="ignore"):
            t = D * (np.log(P0 + z * D) - np.log(nu))
        return dH + p.lam * float(np.sum(t))

    if lo >= 1.0 or fprime(lo) >= 0.0:
        return lo
    if fprime(1.0) <= 0.0:
        return 1.0
    return float(brentq(fprime, lo, 1.0, xtol=1e-16, rtol=1e-15, maxiter=500))


def opt_weights(p: Problem, P, deltas, dH, n_upd: int, z0: float) -> np.ndarray:
    """GetWeights `opt` (eq. opt-weights-problem) on the tracked score
    (reading R14): one weight theta_J per updated cell minimising
        f(theta) = sum_J theta_J dH_J + lam KL(P + sum_J theta_J Delta_J | nu)
    over [1/n, 1]^J (the safe weight as the lower bound, as for `line`),
    Delta_J = the change of the cell's basic marginals, dH_J = the change of
    its pieces.  f is convex (linear pieces, convex KL of an affine map), so
    the minimiser is found by a bounded quasi-Newton method (L-BFGS-B) with
    the exact gradient g_J = dH_J + lam sum_y Delta_J log(P_theta / nu),
    started at the line weight z0."""
    from scipy.optimize import minimize
    lo = 1.0 / max(n_upd, 1)
    D = np.stack([np.ravel(x) for x in deltas])          # (cells, grid)
    P0 = np.ravel(P)
    nu = p.nu.ravel()
    dH = np.asarray(dH, dtype=np.float64)

    def fg(th):
        Pt = P0 + th @ D
        with np.errstate(divide="ignore", invalid="ignore"):
            lg = np.where(Pt > 0, np.log(Pt) - np.log(nu), 0.0)
        f = float(th @ dH) + p.lam * float(np.sum(np.where(Pt > 0, Pt * lg, 0.0) - Pt + nu))
        return f, dH + p.lam * (D @ lg)
    x0 = np.full(len(deltas), min(max(z0, lo), 1.0))
    res = minimize(fg, x0, jac=True, method="L-BFGS-B", bounds=[(lo, 1.0)] * len(deltas),
                   options=dict(ftol=1e-16, gtol=1e-14, maxiter=20000, maxcor=30))
    return np.clip(res.x, lo, 1.0)


def _mark_warm(p: Problem, st: State, cell):
    """abar on the basic cells of `cell` now holds a cell potential (R5)."""
    if st.warm is None:
        st.warm = np.zeros(p.nb1 * p.nb2, dtype=bool)
    for b in cell["basic"]:
        st.warm[b] = True


def _dd_step(p: Problem, st: State, cells, part: str, rule: str, opt: Options,
             force: bool) -> dict:
    """One parallel DomDecIter (Algorithm 4) over `cells`, with GetWeights
    `rule` (reading R9; force = greedy).  Mutates `st`."""
    P = aggregate(p, st.boxes)
    upd = [(c, process_cell(p, c, st.boxes, P, opt, st.abar, st.warm)) for c in cells]
    n_upd = len(upd)

    # candidate state for the greedy choice
    cand_boxes = list(st.boxes)
    htil = st.hbar.copy()
    for c, r in upd:
        o1, o2 = r["box"][0], r["box"][1]
        for b in c["basic"]:
            cand_boxes[b] = truncate_to_box(o1, o2, r["cand"][b], opt.trunc)
            htil[b] = r["pieces"][b]
    Pg = aggregate(p, cand_boxes)
    e_cur = float(st.hbar.sum()) + p.lam * uot.kl(P, p.nu)
    e_grd = float(htil.sum()) + p.lam * uot.kl(Pg, p.nu)

    if rule == "greedy" or force:
        theta = 1.0
    elif rule == "safe":
        theta = 1.0 / max(n_upd, 1)
    elif rule == "swift":
        theta = 1.0 if e_grd <= e_cur + opt.lenience * abs(e_cur) else 1.0 / max(n_upd, 1)
    elif rule in ("line", "opt"):
        theta = line_weight(p, P, Pg, float(htil.sum() - st.hbar.sum()), n_upd)
    else:
        raise ValueError(rule)
    thetas = [theta] * n_upd
    if rule == "opt" and not force:
        deltas, dHs = [], []
        for c, r in upd:
            dl = np.zeros((p.n1, p.n2))
            for b in c["basic"]:
                for sign, (o1, o2, arr) in ((1.0, cand_boxes[b]), (-1.0, st.boxes[b])):
                    if arr.size:
                        dl[o1:o1 + arr.shape[0], o2:o2 + arr.shape[1]] += sign * arr
            deltas.append(dl)
            dHs.append(sum(htil[b] - st.hbar[b] for b in c["basic"]))
        thetas = list(opt_weights(p, P, deltas, dHs, n_upd, theta))
        theta = float(np.mean(thetas))

    # Algorithm 4: pi' = sum_J (1 - theta_J) pi_J + theta_J pi~_J
    for (c, r), theta_c in zip(upd, thetas):
        theta = theta_c
        box = r["box"]
        for b in c["basic"]:
            v = (1.0 - theta) * _on_box(st.boxes[b], box) + theta * _on_box(cand_boxes[b], box)
            st.boxes[b] = truncate_to_box(box[0], box[1], v, opt.trunc)
            st.hbar[b] = (1.0 - theta) * st.hbar[b] + theta * htil[b]
        pxf = st.px.ravel()
        pxf[r["xi"]] = (1.0 - theta) * pxf[r["xi"]] + theta * r["px"]
        st.abar.ravel()[r["xi"]] = r["alpha"]
        _mark_warm(p, st, c)
        if st.plan is not None:
            rows = r["xi"]
            new = np.zeros((rows.size, p.n1 * p.n2))
            new[:, r["yi"]] = r["pi"]
            st.plan[rows] = (1.0 - theta) * st.plan[rows] + theta * new
    theta = float(np.mean(thetas)) if thetas else 1.0
    stats = dict(part=part, theta=theta, thetas=np.asarray(thetas), e_cur=e_cur, e_greedy=e_grd,
                 n_cells=len(cells), n_updated=n_upd,
                 iters=[r["iters"] for _, r in upd],
                 n_unconverged=sum(1 for _, r in upd if not r["converged"]),
                 point_iters=sum(r["iters"] * r["xi"].size for _, r in upd))
    st.history.append(stats)
    return stats


def half_iteration(p: Problem, st: State, part: str, opt: Options):
    """One half-iteration over partition `part`: a parallel DomDecIter
    (Algorithm 4) over all its cells with GetWeights per reading R9, or, for
    `staggered`, four of them in turn over the staggered batches, each with
    swift.  Mutates `st`; returns the step's statistics (a list of the four
    batch steps for `staggered`).  After an eps change or a refinement the
    whole half-iteration is greedy."""
    force = st.force_greedy
    if opt.getweights == "staggered":
        out = [_dd_step(p, st, cells, part, "swift", opt, force)
               for cells in staggered_batches(p, part)]
    else:
        out = _dd_step(p, st, composite_cells(p, part), part, opt.getweights, opt, force)
    st.force_greedy = False
    st.k += 1
    return out


def half_iteration_sequential(p: Problem, st: State, part: str, opt: Options) -> dict:
    """Sequential DomDecIter (Algorithm 3): cells in order, each solved against
    the plan updated by all previous cells."""
    cells = composite_cells(p, part)
    iters = []
    for c in cells:
        P = aggregate(p, st.boxes)
        r = process_cell(p, c, st.boxes, P, opt, st.abar, st.warm)
        iters.append(r["iters"])
        o1, o2 = r["box"][0], r["box"][1]
        for b in c["basic"]:
            st.boxes[b] = truncate_to_box(o1, o2, r["cand"][b], opt.trunc)
            st.hbar[b] = r["pieces"][b]
        st.px.ravel()[r["xi"]] = r["px"]
        st.abar.ravel()[r["xi"]] = r["alpha"]
        _mark_warm(p, st, c)
        if st.plan is not None:
            new = np.zeros((r["xi"].size, p.n1 * p.n2))
            new[:, r["yi"]] = r["pi"]
            st.plan[r["xi"]] = new
    st.k += 1
    stats = dict(part=part, theta=1.0, iters=iters)
    st.history.append(stats)
    return stats


def run(p: Problem, st: State, n_half: int, opt: Options, sequential=False, single=False):
    """Algorithm 2: k odd -> partition A, k even -> B (k counted from 1).
    `single` uses partition A only (Remark on one partition)."""
    out = []
    for _ in range(n_half):
        part = "A" if (single or st.k % 2 == 0) else "B"
        f = half_iteration_sequential if sequential else half_iteration
        out.append(f(p, st, part, opt))
    return out


def set_eps(p: Problem, st: State, eps: float):
    """Next epsilon stage (Sec. 4.4 epsilon-scaling).  The tracked pieces were
    computed for the old eps, so the next half-iteration is taken greedily,
    which makes every Hbar_i exact again."""
    p.eps = float(eps)
    st.force_greedy = True


# --------------------------------------------------------------------------
# multiscale (Sec. 4.4 "Multi-scale and eps-scaling")
# --------------------------------------------------------------------------
def coarsen(a):
    """Masses of the next coarser layer: sums over 2 x 2 blocks of points."""
    n1, n2 = a.shape
    return a.reshape(n1 // 2, 2, n2 // 2, 2).sum(axis=(1, 3))


def refine(pc: Problem, stc: State, pf: Problem, trunc: float) -> State:
    """Warm start of the finer layer from a coarse DD state.

    Reading R10: the coarse plan is carried to the fine grid by splitting each
    entry pi_c(X, Y) in proportion to the fine masses inside the 2 x 2 blocks
    X and Y; the state keeps only basic-cell Y-marginals, so a fine basic
    cell i inside the coarse basic cell I takes the share |mu_f(X_i)| /
    |mu_c(X_I)| of the refined marginal of I.  Boxes double, then entries
    below `trunc` are dropped and the box shrinks (R7).  The tracked pieces
    are scaled alike (estimates: the next step is forced greedy).  The stitched
    X-potential (cost units) is interpolated linearly to the fine grid (as in
    R11), which keeps its error at the curvature of the potential times h^2
    where a copy per 2 x 2 block would leave its gradient times h; it stays a
    warm start (R5) where the coarse basic cell's was."""
    ones = np.ones((2, 2))
    nbasic = pf.nb1 * pf.nb2
    boxes, hbar = [], np.zeros(nbasic)
    for b in range(nbasic):
        rect = basic_rect(pf, b)
        x1, x2 = rect[0], rect[1]
        I1, I2 = (x1 // 2) // pc.s1, (x2 // 2) // pc.s2
        I = I1 * pc.nb2 + I2
        crect = basic_rect(pc, I)
        f = pf.mu[x1:x1 + rect[2], x2:x2 + rect[3]].sum() / \
            pc.mu[crect[0]:crect[0] + crect[2], crect[1]:crect[1] + crect[3]].sum()
        hbar[b] = f * stc.hbar[I]
        o1, o2, arr = stc.boxes[I]
        if arr.size == 0:
            boxes.append((2 * o1, 2 * o2, np.zeros((0, 0))))
            continue
        l1, l2 = arr.shape
        fine = np.kron(arr / pc.nu[o1:o1 + l1, o2:o2 + l2], ones) * \
            pf.nu[2 * o1:2 * (o1 + l1), 2 * o2:2 * (o2 + l2)] * f
        boxes.append(truncate_to_box(2 * o1, 2 * o2, fine, trunc))
    px = np.kron(stc.px / pc.mu, ones) * pf.mu
    # the stored X-potential (cost units) is interpolated linearly (R11's
    # interpolate_potential); its validity follows the coarse basic cell
    abar = interpolate_potential(stc.abar, pf.n1, pf.n2)
    warm = np.zeros(nbasic, dtype=bool)
    if stc.warm is not None:
        for b in range(nbasic):
            x1, x2 = basic_rect(pf, b)[:2]
            warm[b] = stc.warm[((x1 // 2) // pc.s1) * pc.nb2 + (x2 // 2) // pc.s2]
    return State(boxes, px, hbar, abar, force_greedy=True, warm=warm)


def interpolate_potential(a_c, n1f: int, n2f: int) -> np.ndarray:
    """Potential of the finer layer from the coarse one (reading R11).

    Coarse point I stands for the fine block {2I, 2I + 1}: its potential is
    taken at the block centre, fine index 2I + 1/2.  Each axis is linear
    between the two nearest coarse points, continued linearly past the first
    and last centres (one coarse point: constant).  Potentials are in cost
    units, so a layer whose eps equals the coarse one's keeps their meaning."""
    a_c = np.asarray(a_c, dtype=np.float64)

    def along(a, axis, nf):
        nc = a.shape[axis]
        if nc == 1:
            return np.repeat(a, nf, axis=axis)
        u = (np.arange(nf) - 0.5) / 2.0
        k = np.clip(np.floor(u).astype(int), 0, nc - 2)
        t = u - k
        lo = np.take(a, k, axis=axis)
        hi = np.take(a, k + 1, axis=axis)
        shape = [1] * a.ndim
        shape[axis] = nf
        t = t.reshape(shape)
        return (1.0 - t) * lo + t * hi

    return along(along(a_c, 0, n1f), 1, n2f)


def init_from_duals(p: Problem, alpha, beta, trunc: float, windows=None) -> State:
    """DD state of the plan pi = exp((alpha + beta - c)/eps) mu x nu (the
    diagonal-scaling form of Sec. 4.1) split by basic cells (reading R11):
    nu_i(y) = sum_{x in X_i} pi(x, y), restricted to the basic cell's scan
    window (default: the whole grid), entries below `trunc` dropped, box =
    bbox of the rest.  The cell plan is pi on X_i x (kept points of the box); P_X pi
    and the tracked pieces Hbar_i (cell_piece) are those of the cell plans.
    The first half-iteration from this state is greedy.  Dense: small grids."""
    C = full_cost(p)
    a = np.ravel(alpha).astype(np.float64)
    b = np.ravel(beta).astype(np.float64)
    pi = uot.plan(a, b, p.mu, p.nu, C, p.eps)
    nbasic = p.nb1 * p.nb2
    nu_tot = p.nu.sum()
    boxes, hbar = [], np.zeros(nbasic)
    px = np.zeros_like(p.mu)
    for bi in range(nbasic):
        rect = basic_rect(p, bi)
        idx = rect_index(rect, p.n2)
        rows = pi[idx]
        nb = rows.sum(0).reshape(p.n1, p.n2)
        inwin = np.zeros((p.n1, p.n2), dtype=bool)
        w1, w2, wl1, wl2 = (0, 0, p.n1, p.n2) if windows is None else windows[bi]
        inwin[w1:w1 + wl1, w2:w2 + wl2] = True
        keep = inwin & (nb >= trunc) & (nb > 0)
        mu_x = p.mu.ravel()[idx]
        if not keep.any():
            boxes.append((rect[0], rect[1], np.zeros((0, 0))))
            hbar[bi] = cell_piece(np.zeros((idx.size, 0)), mu_x, np.zeros(0), nu_tot,
                                  np.zeros((idx.size, 0)), p.eps, p.lam)
            continue
        r1, r2 = np.nonzero(keep)
        o1, o2 = r1.min(), r2.min()
        l1, l2 = r1.max() + 1 - o1, r2.max() + 1 - o2
        yrect = (o1, o2, l1, l2)
        kb = keep[o1:o1 + l1, o2:o2 + l2]
        yidx = rect_index(yrect, p.n2)
        pi_box = rows[:, yidx] * kb.ravel()[None, :]
        boxes.append((o1, o2, np.where(kb, nb[o1:o1 + l1, o2:o2 + l2], 0.0)))
        px.ravel()[idx] = pi_box.sum(1)
        hbar[bi] = cell_piece(pi_box, mu_x, p.nu.ravel()[yidx], nu_tot,
                              rect_cost(p, rect, yrect), p.eps, p.lam)
    return State(boxes, px, hbar, np.asarray(alpha, dtype=np.float64).reshape(p.mu.shape).copy(),
                 force_greedy=True, warm=np.ones(nbasic, dtype=bool))


# --------------------------------------------------------------------------
# certificate (global primal-dual gap of a DD state)
# --------------------------------------------------------------------------
def certificate(p: Problem, abar, polish: int = 0) -> dict:
    """Dual candidate alpha_bar (stitched cell potentials) -> beta_hat by one
    global Y-update with nu_- = 0 (eq. sinkhorn-iters-ot) -> pi_hat; the gap is
    PD = lam KL(P_X pi_hat | exp(-alpha/lam) mu), exact by eq. (PD-gap-KL) with
    J = I.  Dense: for small grids only.  Also returns primal and dual.

    polish: `polish` more global Sinkhorn iterations (X-update, then Y-update,
    eq. sinkhorn-iters-ot) from that pair; every pair k gives a lower bound
    D(alpha_k, beta_k) and an upper bound E(pi_k) of the optimal value
    (weak duality), returned as the best of each (dual_polished,
    primal_polished), the pair 0 included."""
    C = full_cost(p)
    a = np.ravel(abar)
    kappa = p.lam / (p.lam + p.eps)
    z = uot.y_log_integral(a, p.mu, C, p.eps)
    bhat = -p.eps * kappa * z
    pi = uot.plan(a, bhat, p.mu, p.nu, C, p.eps)
    px, py = pi.sum(1), pi.sum(0)
    pd = uot.pd_gap_kl(a, px, p.mu, p.lam)
    D = uot.dual(a, bhat, p.mu, p.nu, C, p.eps, p.lam)
    E = uot.primal(pi, p.mu, p.nu, C, p.eps, p.lam)
    dbest, ebest = D, E
    ak, bk = a, bhat
    for _ in range(polish):
        ak = uot.x_update(bk, p.nu, C, p.eps, p.lam)
        bk = -p.eps * kappa * uot.y_log_integral(ak, p.mu, C, p.eps)
        pik = uot.plan(ak, bk, p.mu, p.nu, C, p.eps)
        dbest = max(dbest, uot.dual(ak, bk, p.mu, p.nu, C, p.eps, p.lam))
        ebest = min(ebest, uot.primal(pik, p.mu, p.nu, C, p.eps, p.lam))
    return dict(pd=pd, dual=D, primal=E, rel=pd / abs(D), beta_hat=bhat.reshape(p.mu.shape),
                px=px.reshape(p.mu.shape), py=py.reshape(p.mu.shape),
                l1_x=float(np.abs(px - np.exp(-a / p.lam) * p.mu.ravel()).sum()),
                dual_polished=dbest, primal_polished=ebest)
