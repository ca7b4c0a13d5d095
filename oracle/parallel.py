"""The contract's LDL^T, first k columns of L^-1, block and eigenvalues at the
benchmark sizes (N = 1024 at 49152 and 98304 bits), rows dealt over worker
processes.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

What is computed is exactly ``contract.factor`` -> ``contract.solve`` ->
``contract.block`` -> ``contract.eigen``, with every rounding point taken by the
same contract functions (``load_entry``, ``pivot_reciprocal``,
``column_factors``, ``linv_diag``, ``linv_entry``, ``block_from_sums``).  Only
the exact integer work is spread out and handed to GMP:

* Distribution.  The paper spreads the matrix over nodes by columns and hands
  every finished column to all of them (Table 1, Algorithms 2 and 3).  Here row r
  of the lower triangle (its entries a_rc, c <= r) lives in worker r mod nproc.
  For column i the owner of row i takes the pivot d_i = a_ii, h_i and w_i, and
  the entries x_im of L^-1's first k columns (Algorithm 4); every worker then
  forms u_r and b_r for its own rows, publishes them, and applies
  a_rc -= b_r u_c to its own rows r >= c > i with mpz_submul.  The update is
  exact, so which process applies which update does not change a bit.
* Algorithm 4's sums.  x_rm = rnd(-(sum_{i=m}^{r-1} b_ri x_im) / 2**h_r) needs
  the whole row r of B; the sum is accumulated while the columns are factored
  (acc_rm += b_ri x_im once column i is done and x_im is known), then rounded
  by ``linv_entry`` when row r becomes the pivot.  The sum is exact, so it is
  the same integer as ``contract.solve``'s.
* Outputs.  Pivots d_i, exponents h_i, w_i, X in full; the multipliers b_ri
  only as one SHA-256 per column (they are 3.2 GB at N = 1024, P = 49152): the
  digest of the column's entries r = i+1 .. N-1, each as P/32 little-endian
  32-bit limbs in two's complement; d_i as 2P/32 limbs.

Errors: ENOTPD at pivot i and EOVERFLOW of a factor at column i stop the run
as ``contract.factor`` does; an EOVERFLOW of L^-1 is reported only when the
factorisation had none (``contract.solve`` runs after the factorisation).

Parity status: pinned in ``tests/test_oracle_gmp.py`` against the
single-process contract bit for bit (d, h, w, every b_ri through its column
digest, X, block, lambda_1) for several beta, N, P, E, k and process counts, on
the leading-columns sample, on a planted wrong-sign update, and on the ENOTPD
and EOVERFLOW paths.
"""

from __future__ import annotations

import hashlib
import multiprocessing as mp
import threading
import time
from dataclasses import dataclass
from typing import List, Optional, Sequence

import numpy as np

from . import contract as C
from .gmp import Mpz


def tc_bytes(v: int, nlimbs: int) -> bytes:
    """v as nlimbs little-endian 32-bit limbs, two's complement."""
    return v.to_bytes(4 * nlimbs, "little", signed=True)


def column_digest(values: Sequence[int], nlimbs: int) -> str:
    h = hashlib.sha256()
    for v in values:
        h.update(tc_bytes(v, nlimbs))
    return h.hexdigest()


@dataclass
class ParallelFactor:
    N: int
    P: int
    E: int
    k: int
    s: List[int]
    d: List[int]
    h: List[int]
    w: List[int]
    b_sha: List[str]              # per column i < N - 1: digest of b_ri, r = i+1 .. N-1
    d_sha: List[str]              # per column: digest of d_i (2P/32 limbs)
    X: List[List[int]]            # X[r][m], m < k
    G: int
    Q: int
    column_seconds: float = 0.0   # wall time of the column loop (after the load), slowest worker

    @property
    def W(self) -> int:
        return 2 * self.P - 4


# shared arrays (numpy views of multiprocessing RawArrays), set before fork
_SH = {}


def _alloc(name, shape, dtype):
    n = int(np.prod(shape)) * np.dtype(dtype).itemsize
    raw = mp.RawArray("b", max(1, n))
    _SH[name] = (raw, shape, dtype)


def _view(name):
    raw, shape, dtype = _SH[name]
    return np.frombuffer(raw, dtype=dtype, count=int(np.prod(shape))).reshape(shape)


def _worker(p: int, nproc: int, mu, N: int, P: int, s: List[int], k: int, ncols: int, barrier, out_q):
    nl, nw, W = P // 32, P // 16, 2 * P - 4
    G, Q = C.solve_exponents(s, k, W)
    Dsh, Hsh, Wsh = _view("d"), _view("h"), _view("w")
    Ush, Usg, Bsh, Xsh, ctrl = _view("u"), _view("usign"), _view("b"), _view("x"), _view("ctrl")
    rows = list(range(p, N, nproc))
    A = {r: [Mpz(C.load_entry(mu, r, c, W, s)) for c in range(r + 1)] for r in rows}
    acc = {r: [Mpz() for _ in range(min(r, k))] for r in rows}   # acc_rm, m < min(r, k)
    digests = []
    solve_err = None
    t_start = None

    def fail(code, idx):
        if ctrl[0] == 0:
            ctrl[0], ctrl[1] = code, idx

    try:
        barrier.wait()   # every worker has loaded its rows: the column loop starts together
        t_start = time.perf_counter()
        for i in range(ncols):
            cur = i & 1
            # -- the pivot row's owner: d_i, h_i, w_i and row i of X
            if i % nproc == p:
                d = A[i][i].get()
                if d <= 0:
                    fail(C.ENOTPD, i)
                else:
                    h, w = C.pivot_reciprocal(d, P)
                    Dsh[i] = np.frombuffer(tc_bytes(d, nw), dtype=np.uint32)
                    Hsh[i] = h
                    Wsh[i] = np.frombuffer(tc_bytes(w, nl + 2), dtype=np.uint32)
                    for m in range(min(i + 1, k)):
                        try:
                            x = C.linv_diag(Q, h, m) if m == i else C.linv_entry(acc[i][m].get(), h, P, i)
                        except C.ContractError as e:
                            solve_err = solve_err or (e.code, e.index)
                            x = 0
                        Xsh[i, m] = np.frombuffer(tc_bytes(x, nl), dtype=np.uint32)
                del A[i], acc[i]
            barrier.wait()
            if ctrl[0]:
                break
            # -- every worker: u_r, b_r of its rows r > i, and the sums of Algorithm 4
            h = int(Hsh[i])
            w = int.from_bytes(Wsh[i].tobytes(), "little", signed=True)
            xs = [Mpz(int.from_bytes(Xsh[i, m].tobytes(), "little", signed=True)) for m in range(min(i + 1, k))]
            bm = {}
            for r in rows:
                if r <= i:
                    continue
                try:
                    u, b = C.column_factors(A[r][i].get(), h, w, P, i)
                except C.ContractError as e:
                    fail(e.code, e.index)
                    break
                A[r][i] = None
                mag = -u if u < 0 else u
                Ush[cur, r] = np.frombuffer(mag.to_bytes(4 * nl, "little"), dtype=np.uint32)
                Usg[cur, r] = 1 if u < 0 else 0
                Bsh[cur, r] = np.frombuffer(tc_bytes(b, nl), dtype=np.uint32)
                bm[r] = Mpz(b)
                for m, xm in enumerate(xs):
                    acc[r][m].addmul(bm[r], xm)
            barrier.wait()
            if ctrl[0]:
                break
            # -- digests of column i (one worker), then the exact trailing update
            if i < N - 1 and (i + nproc // 2) % nproc == p:
                digests.append((i, hashlib.sha256(Dsh[i].tobytes()).hexdigest(),
                                hashlib.sha256(Bsh[cur, i + 1:N].tobytes()).hexdigest()))
            elif i == N - 1 and i % nproc == p:
                digests.append((i, hashlib.sha256(Dsh[i].tobytes()).hexdigest(), None))
            if not bm:
                continue
            top = max(bm)
            base = Ush[cur].ctypes.data
            uc = {}
            for c in range(i + 1, top + 1):
                z = Mpz()
                z.set_bytes(base + 4 * nl * c, 4 * nl, bool(Usg[cur, c]))
                uc[c] = z
            for r, b in bm.items():
                row = A[r]
                for c in range(i + 1, r + 1):
                    row[c].submul(b, uc[c])
    except threading.BrokenBarrierError:
        pass
    out_q.put((p, digests, solve_err, time.perf_counter() - t_start if t_start is not None else 0.0))


def factor_solve(mu, N: int, P: int, E: int, k: int, nproc: int = 8, timeout: float = 6 * 3600,
                 columns: Optional[int] = None) -> ParallelFactor:
    """contract.factor followed by contract.solve, rows over nproc processes.

    ``columns`` stops after that many pivots (a timing sample of the leading
    columns; the result then holds only their d, h, w and digests)."""
    if P % 32 or P < 64:
        raise C.ContractError(C.EINVAL, -1, "P must be a positive multiple of 32")
    if N < 1 or E < 1 or not 1 <= k <= N:
        raise C.ContractError(C.EINVAL, -1, "bad N, E or k")
    nproc = max(1, min(nproc, N))
    nl, nw, W = P // 32, P // 16, 2 * P - 4
    s = C.scales(mu, N, E)
    G, Q = C.solve_exponents(s, k, W)
    _SH.clear()
    _alloc("d", (N, nw), np.uint32)
    _alloc("h", (N,), np.int64)
    _alloc("w", (N, nl + 2), np.uint32)
    _alloc("u", (2, N, nl), np.uint32)
    _alloc("usign", (2, N), np.int8)
    _alloc("b", (2, N, nl), np.uint32)
    _alloc("x", (N, k, nl), np.uint32)
    _alloc("ctrl", (2,), np.int64)
    ctx = mp.get_context("fork")
    barrier = ctx.Barrier(nproc, timeout=timeout)
    q = ctx.Queue()
    ncols = N if columns is None else max(1, min(N, columns))
    procs = [ctx.Process(target=_worker, args=(p, nproc, mu, N, P, s, k, ncols, barrier, q))
             for p in range(nproc)]
    for pr in procs:
        pr.start()
    results = [q.get() for _ in procs]
    for pr in procs:
        pr.join()
    if any(pr.exitcode != 0 for pr in procs):
        raise RuntimeError("an oracle worker failed")
    ctrl = _view("ctrl")
    if ctrl[0]:
        raise C.ContractError(int(ctrl[0]), int(ctrl[1]), "parallel factorisation")
    errs = [e for _, _, e, _ in results if e is not None]
    tcols = max(t for _, _, _, t in results)
    if errs:
        code, idx = min(errs, key=lambda t: t[1])
        raise C.ContractError(code, idx, "L^-1 entry")
    dig = sorted(x for _, ds, _, _ in results for x in ds)
    assert [x[0] for x in dig] == list(range(ncols))
    if ncols < N:
        Dsh, Hsh, Wsh = _view("d"), _view("h"), _view("w")
        out = ParallelFactor(N=N, P=P, E=E, k=k, s=s,
                             d=[int.from_bytes(Dsh[i].tobytes(), "little", signed=True) for i in range(ncols)],
                             h=[int(v) for v in Hsh[:ncols]],
                             w=[int.from_bytes(Wsh[i].tobytes(), "little", signed=True) for i in range(ncols)],
                             b_sha=[x[2] for x in dig], d_sha=[x[1] for x in dig], X=[], G=G, Q=Q,
                             column_seconds=tcols)
        _SH.clear()
        return out
    Dsh, Hsh, Wsh, Xsh = _view("d"), _view("h"), _view("w"), _view("x")
    d = [int.from_bytes(Dsh[i].tobytes(), "little", signed=True) for i in range(N)]
    w = [int.from_bytes(Wsh[i].tobytes(), "little", signed=True) for i in range(N)]
    X = [[int.from_bytes(Xsh[r, m].tobytes(), "little", signed=True) for m in range(k)] for r in range(N)]
    out = ParallelFactor(N=N, P=P, E=E, k=k, s=s, d=d, h=[int(v) for v in Hsh], w=w,
                         b_sha=[x[2] for x in dig[:-1]], d_sha=[x[1] for x in dig], X=X, G=G, Q=Q,
                         column_seconds=tcols)
    _SH.clear()
    return out


def _pair_sum(args):
    X, w, a, b, N = args
    return a, b, C.block_sum(X, w, a, b, N)


def block(pf: ParallelFactor, nproc: int = 8) -> C.Block:
    """contract.block with its k(k+1)/2 exact sums spread over a process pool."""
    k, N = pf.k, pf.N
    Mt = [[0] * k for _ in range(k)]
    pairs = [(a, b) for a in range(k) for b in range(a, k)]
    with mp.get_context("fork").Pool(max(1, nproc)) as pool:
        for a, b, v in pool.imap_unordered(_pair_sum, [(pf.X, pf.w, a, b, N) for a, b in pairs]):
            Mt[a][b] = Mt[b][a] = v
    return C.block_from_sums(Mt, pf.s, k, pf.P, pf.W, pf.Q)


def lambda_min(mu, N: int, k: int, P: int, E: int = 16, nproc: int = 8, prec: Optional[int] = None):
    """The whole path at large N: factor and solve in parallel, block, eigen."""
    pf = factor_solve(mu, N, P, E, k, nproc)
    bl = block(pf, nproc)
    return pf, bl, C.eigen(bl, prec=prec, P=P)
