"""Closed-form kernel properties, derived by hand from the kernel
descriptions (work-item by work-item counting, Sec. 3.2 Alg. 1), valid at
any size.  Used to check counts at sizes no enumeration finishes."""


def cdiv(a, b):
    return -(-a // b)


def bank(e, stride):
    """Bank-stride bin name of an LDS site whose element index moves by
    `stride` elements of e bytes per lane: b0 for a broadcast, else b2^k
    for 2^k the power of two in the word stride, at most 32."""
    w = stride * e // 4
    if w == 0:
        return "b0"
    k = 0
    while w % 2 == 0 and k < 5:
        w //= 2
        k += 1
    return "b%d" % (1 << k)


def matmul(v):
    n, m, l, T = v["n"], v["m"], v["l"], v["T"]
    GX, GY, KT = cdiv(l, T), cdiv(n, T), cdiv(m, T)
    wi = GX * GY * T * T
    if v["op"] == "tiled":
        # As[ly][lx], Bs[ly][lx] stored at lane stride 1; As[ly][k] read by
        # every lane of a row at one word, Bs[k][lx] at lane stride 1
        return {"gld.4.1": n * m * GX + m * l * GY, "gst.4.1": n * l,
                "lst.4": 2 * wi * KT, "lld.4": 2 * wi * KT * T,
                "lst.4.b1": 2 * wi * KT, "lld.4.b0": wi * KT * T, "lld.4.b1": wi * KT * T,
                "fma.f32": wi * KT * T, "bar.wi": 2 * wi * KT,
                "bar.wg": 2 * GX * GY * KT, "wg": GX * GY, "wi": wi}
    return {"gld.4.0": n * m * l, "gld.4.1": n * m * l, "gst.4.1": n * l,
            "fma.f32": n * m * l, "wg": GX * GY, "wi": wi}


def transpose(v):
    n, T = v["n"], v["T"]
    G = cdiv(n, T)
    base = {"wg": G * G, "wi": G * G * T * T}
    strided = "4/>4" if n > 4 else {2: "2/2", 3: "3/3", 4: "4/4"}.get(n, "1")
    if v["op"] == "tiled":
        # tile[ly][lx] stored at lane stride 1, tile[lx][ly] read at T + 1
        base.update({"gld.4.1": n * n, "gst.4.1": n * n, "lst.4": n * n,
                     "lld.4": n * n, "lst.4.b1": n * n, "lld.4." + bank(4, T + 1): n * n,
                     "bar.wi": G * G * T * T, "bar.wg": G * G})
    elif v["op"] == "naive_wc":
        base.update({"gld.4." + strided: n * n, "gst.4.1": n * n})
    else:
        base.update({"gld.4.1": n * n, "gst.4." + strided: n * n})
    out = {}
    for k, x in base.items():
        out[k] = out.get(k, 0) + x
    return out


def stencil(v):
    n, T, dt = v["n"], v["T"], v.get("dtype", "f32")
    e = 4 if dt == "f32" else 8
    G = cdiv(n, T)
    halo = 4 * n * G
    # halo columns written at a fixed column (lane stride 0): the left one
    # in every tile column, the right one in the full tile columns
    col0 = G * n + (n // T) * n
    return {"gld.%d.1" % e: n * n + halo, "lst.%d" % e: n * n + halo,
            "lst.%d.b0" % e: col0, "lst.%d.%s" % (e, bank(e, 1)): n * n + halo - col0,
            "lld.%d" % e: 5 * n * n, "lld.%d.%s" % (e, bank(e, 1)): 5 * n * n,
            "add." + dt: 4 * n * n,
            "mul." + dt: 3 * n * n, "gst.%d.1" % e: n * n,
            "bar.wi": G * G * T * T, "bar.wg": G * G, "wg": G * G,
            "wi": G * G * T * T}


def nbody(v):
    N, G = v["n"], v["wg"]
    B = cdiv(N, G)
    wi = B * G
    # sh[c*G + l] stored at lane stride 1; sh[c*G + jj] read at one word
    return {"gld.4.3/3": 3 * N + 3 * N * B, "gst.4.1": N, "lst.4": 3 * N * B,
            "lld.4": 3 * wi * N, "lst.4.b1": 3 * N * B, "lld.4.b0": 3 * wi * N,
            "add.f32": 6 * wi * N + wi * B, "mul.f32": 3 * wi * N,
            "spec.f32": wi * N, "bar.wi": 2 * wi * B, "bar.wg": 2 * B * B,
            "wg": B, "wi": wi}


def stream(v):
    dt = v.get("dtype", "f32")
    e = 4 if dt == "f32" else 8
    n, wg, s, U, vec = v["n"], v["wg"], v["s"], v.get("U", 1), v.get("vec", 1)
    base = {"wg": n // wg, "wi": n}
    if v["op"] == "filled":
        # c of every s cells read: |F| = c*J cells for J = n*U groups; each
        # read cell opens a run of s cells, so Fill = [0, s*(J-1) + c-1 + s)
        c = v.get("c", s)
        J = n * U
        q = min(s, 4)
        k = min(max(-(-(q * c * J) // (s * J + c - 1)), 1), q)
        cl = "%d/%s" % (k, q if s <= 4 else ">4")
        base.update({"gld.%d.%s" % (e, cl): c * J, "gst.%d.1" % e: n,
                     "add." + dt: c * J})
        return base
    cl = {1: "1", 2: "1/2", 3: "1/3", 4: "1/4"}.get(s, "1/>4")
    key = "%d.%s" % (e * vec, cl)
    if v["op"] == "load":
        base.update({"gld." + key: n * U, "add." + dt: n * U * vec})
    elif v["op"] == "store":
        base["gst." + key] = n * U
    elif v["op"] == "copy":
        base.update({"gld." + key: n * U, "gst." + key: n * U})
    elif v["op"] == "axpby":
        base.update({"gld." + key: 2 * n * U, "gst." + key: n * U,
                     "mul." + dt: 2 * n * U * vec, "add." + dt: n * U * vec})
    else:
        base.update({"gld." + key: 4 * n * U, "gst." + key: n * U,
                     "add." + dt: 3 * n * U * vec})
    return base


def chain(v):
    dt = v.get("dtype", "f32")
    e = 4 if dt == "f32" else 8
    n, F, K = v["n"], v["F"], v["K"]
    out = {"gld.%d.1" % e: n, "gst.%d.1" % e: n, "wg": n // v["wg"], "wi": n}
    if v["family"] == "fma":
        out.update({"fma." + dt: n * F, "add." + dt: n * (K - 1)})
    else:
        out.update({"mul.f32": n * F, "add.f32": n * F + n * (K - 1),
                    "spec.f32": n * F})
    return {k: x for k, x in out.items() if x}


def lds(v):
    G, wg, R, W = v["groups"], v["wg"], v["R"], v["W"]
    out = {"gst.4.1": G * wg, "bar.wi": G * wg, "bar.wg": G, "wg": G, "wi": G * wg}
    b = bank(4, v["b"])  # lds[(l*b + r) mod W]: lane stride b
    if v["op"] == "read":
        out.update({"lst.4": G * W, "lld.4": G * wg * R, "add.f32": G * wg * R,
                    "lst.4.b1": G * W, "lld.4." + b: G * wg * R})
    else:
        out.update({"lst.4": G * wg * R, "lld.4": G * wg,
                    "lst.4." + b: G * wg * R, "lld.4." + b: G * wg})
    return {k: x for k, x in out.items() if x}


def barrier(v):
    G, wg, B = v["groups"], v["wg"], v["B"]
    out = {"bar.wi": G * wg * B, "bar.wg": G * B, "gst.4.1": G * wg, "wg": G,
           "wi": G * wg}
    return {k: x for k, x in out.items() if x}


def empty(v):
    gx, gy = cdiv(v["n"], v["wx"]), cdiv(v["n"], v.get("wy", 1))
    return {"wg": gx * gy, "wi": gx * gy * v["wx"] * v.get("wy", 1)}


def conv(v):
    n, T = v["n"], v["T"]
    P, G, TT = n + 6, cdiv(n, T), T + 6
    rows = sum(min(TT, P - gy * T) for gy in range(G))
    img = 9 * rows * rows * 3
    filt = 9 * G * G * 147
    wi = 9 * G * G * T * T
    # fl[t] (lane stride 1) and tile[r][q][c] (3) stored; per tap the tile
    # read at lane stride 3 and fl at one word for every lane
    return {"gld.4.1": filt, "gld.4.3/3": img, "lst.4": img + filt,
            "lld.4": 9 * n * n * 294, "lst.4.b1": img + filt,
            "lld.4.b1": 9 * n * n * 147, "lld.4.b0": 9 * n * n * 147,
            "fma.f32": 9 * n * n * 147,
            "gst.4.1": 9 * n * n, "bar.wi": wi, "bar.wg": 9 * G * G,
            "wg": 9 * G * G, "wi": wi}


def arith(v):
    dt = v.get("dtype", "f32")
    e = 4 if dt == "f32" else 8
    n, F, K = v["n"], v["F"], v["K"]
    out = {"gld.%d.1" % e: n, "gst.%d.1" % e: n, "mul." + dt: n * F,
           "wg": n // v["wg"], "wi": n}
    if v["op"] == "div":
        out.update({"div." + dt: n * F, "add." + dt: n * F + n * (K - 1)})
    else:
        out.update({"exp." + dt: n * F, "add." + dt: n * (K - 1)})
    return {k: x for k, x in out.items() if x}


FORMS = {"matmul": matmul, "transpose": transpose, "stencil": stencil,
         "nbody": nbody, "stream": stream, "fma": chain, "rsqrt": chain,
         "lds": lds, "barrier": barrier, "empty": empty, "conv": conv,
         "arith": arith}


def counts(v):
    return FORMS[v["family"]](v)
