"""The asm loops of Steps IV and VI (`pair16_loop_r6_f32`, `pair16_loop_r4_f32`
and their exact-k variants `pair16_loop_r6x_f32`, `pair16_loop_r4x_f32` in
kde_device.hip) read back from the source and executed instruction by
instruction on the CPU.

Each loop runs the 16-column step of its stage, written out as gfx950 assembly
(equations (6)-(7) with the Gaussian kernel's sixth and fourth derivatives,
He6 in the depressed form (Z^2 - 30) Z - 40 with Z = u^2 - 5, He4(u) =
u^4 - 6u^2 + 3, and exp(-u^2/2) = 2^(-k u^2)).  This test checks their data flow
without a GPU: every operand it reads holds the value the per-pair formula
says it should, the four column accumulators take their terms in read order,
and the fold into the FP64 total is (a0 + a1) + (a2 + a3).  Both sides use the
same FP32 arithmetic model (exact products rounded once, 2^x rounded to FP32),
so any dropped term, wrong register or misordered accumulation fails it.
The loop control is modelled too (64 bytes of LDS per group, cnt groups,
nothing read past the last one).  It also checks the one wait state gfx950
needs between a transcendental result and a VALU op that reads it in the next
instruction, and where each loop's first VALU op lands within 64 bytes.
"""
import os
import re
from fractions import Fraction

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "paper_1505_02100_amd", "csrc", "kde_device.hip")

f32 = np.float32


def block_lines(name):
    text = open(SRC).read()
    start = text.index(f"void {name}(")
    body = text[text.index("asm volatile(", start):]
    body = body[:body.index("\n        :")]
    return [m.group(1) for m in re.finditer(r'"([^"]*)\\n"', body)]


def operand(tok):
    """Register-file key of an operand: %[name] or a physical VGPR (range)."""
    m = re.fullmatch(r"%\[(\w+)\]", tok)
    if m:
        return m.group(1)
    if re.fullmatch(r"v\d+|v\[\d+:\d+\]", tok):
        return tok
    return None


def fma32(a, b, c):
    # one rounding of the exact a*b + c (through a correctly rounded double)
    return f32(float(Fraction(float(a)) * Fraction(float(b)) + Fraction(float(c))))


def exp2_32(a):
    return f32(2.0 ** float(a))


def literal(tok):
    if tok.startswith("0x"):
        return np.frombuffer(int(tok, 16).to_bytes(4, "little"), dtype=np.float32)[0]
    return f32(float(tok))


def execute(lines, x, ui, k, tot, cnt=None, k_lo=0.0):
    """Run a block on one lane.  x is the LDS tile (FP32 values from byte
    address 0); a whole-loop block runs cnt groups of 16 columns from there."""
    reg = {f"x{j}": f32(x[j]) for j in range(min(16, len(x)))}
    reg.update(ui=f32(ui), k=f32(k), khi=f32(k), klo=f32(k_lo), tot=float(tot), addr=0, cnt=cnt, scc=0)
    labels = {l[:-1]: i for i, l in enumerate(lines) if l.endswith(":")}

    def val(tok):
        neg = tok.startswith("-")
        tok = tok.lstrip("-")
        key = operand(tok)
        v = reg[key] if key else literal(tok)
        return -v if neg else v

    pc, steps = 0, 0
    while pc < len(lines):
        line = lines[pc]
        pc += 1
        steps += 1
        assert steps < 100000
        op, _, rest = line.partition(" ")
        t = [a.strip() for a in rest.split(",")]
        if op.endswith(":") or op in ("s_nop", "s_waitcnt", ".p2align"):
            continue
        if op == "s_add_u32":
            reg[operand(t[0])] = int(reg[operand(t[1])]) + int(t[2])
        elif op == "s_sub_u32":
            reg[operand(t[0])] = int(reg[operand(t[1])]) - int(t[2])
        elif op == "s_cmp_lg_u32":
            reg["scc"] = int(reg[operand(t[0])] != int(t[1]))
        elif op == "s_cbranch_scc1":
            if reg["scc"]:
                pc = labels[t[0][:-1]]
        elif op == "v_mov_b32_e32" and t[1] == "%[addr]":
            reg[t[0]] = reg["addr"]
        elif op == "ds_read_b128":
            # four consecutive values at the address register plus the offset
            m = re.fullmatch(r"v\[(\d+):(\d+)\], (v\d+)(?: offset:(\d+))?", rest.strip())
            first, byte = int(m.group(1)), reg[m.group(3)] + int(m.group(4) or 0)
            assert byte % 16 == 0
            for c in range(4):
                reg[f"v{first + c}"] = f32(x[byte // 4 + c])
        else:
            d = operand(t[0])
            if op.startswith("v_sub_f32"):
                reg[d] = f32(val(t[1]) - val(t[2]))
            elif op.startswith("v_add_f32"):
                reg[d] = f32(val(t[1]) + val(t[2]))
            elif op.startswith("v_mul_f32"):
                reg[d] = f32(val(t[1]) * val(t[2]))
            elif op.startswith("v_fmaak_f32") or op.startswith("v_fma_f32"):
                reg[d] = fma32(val(t[1]), val(t[2]), val(t[3]))
            elif op.startswith("v_fmac_f32"):
                reg[d] = fma32(val(t[1]), val(t[2]), reg[d])
            elif op.startswith("v_exp_f32"):
                reg[d] = exp2_32(val(t[1]))
            elif op.startswith("v_cvt_f64_f32"):
                reg[d] = float(val(t[1]))
            elif op.startswith("v_add_f64"):
                reg[d] = val(t[1]) + val(t[2])
            else:
                raise AssertionError(f"unexpected instruction {op}")
    assert cnt is None or reg["cnt"] == 0
    return reg["tot"]


def step_vi_reference(x, ui, k, tot):
    acc = [None] * 4
    for j in range(16):
        d = f32(f32(ui) - f32(x[j]))
        y = f32(d * d)
        q = fma32(d, d, f32(-6.0))
        p = fma32(q, y, f32(3.0))
        e = exp2_32(f32(y * f32(-k)))
        c = j % 4
        acc[c] = f32(p * e) if acc[c] is None else fma32(p, e, acc[c])
    return float(tot) + float(f32(f32(acc[0] + acc[1]) + f32(acc[2] + acc[3])))


def step_iv_reference(x, ui, k, tot):
    acc = [None] * 4
    for j in range(16):
        d = f32(f32(ui) - f32(x[j]))
        z = fma32(d, d, f32(-5.0))
        q = fma32(z, z, f32(-30.0))
        p = fma32(q, z, f32(-40.0))
        e = exp2_32(f32(z * f32(-k)))
        c = j % 4
        acc[c] = fma32(p, e, f32(0.0)) if acc[c] is None else fma32(p, e, acc[c])
    return float(tot) + float(f32(f32(acc[0] + acc[1]) + f32(acc[2] + acc[3])))


def exact_k_reference(r):
    def ref(x, ui, k, tot, k_lo):
        acc = [None] * 4
        for j in range(16):
            d = f32(f32(ui) - f32(x[j]))
            y = f32(d * d)
            a = fma32(y, f32(k), f32(y * f32(k_lo)))
            e = exp2_32(f32(-a))
            # Y - c is contracted with the product: fma(d, d, -c)
            if r == 6:
                q = fma32(d, d, f32(-15.0))
                q = fma32(q, y, f32(45.0))
                p = fma32(q, y, f32(-15.0))
            else:
                q = fma32(d, d, f32(-6.0))
                p = fma32(q, y, f32(3.0))
            c = j % 4
            acc[c] = fma32(p, e, f32(0.0)) if acc[c] is None else fma32(p, e, acc[c])
        return float(tot) + float(f32(f32(acc[0] + acc[1]) + f32(acc[2] + acc[3])))
    return ref


R6, R4 = "pair16_loop_r6_f32", "pair16_loop_r4_f32"
R6X, R4X = "pair16_loop_r6x_f32", "pair16_loop_r4x_f32"
K = f32(np.log2(np.e) / 2)
K_LO = f32(np.log2(np.e) / 2 - float(K))


def run_groups(ref, x, ui, k, tot, cnt):
    for g in range(cnt):
        tot = ref(x[16 * g:16 * g + 16], ui, k, tot)
    return tot


@pytest.mark.parametrize("name,r,seed", [(R6X, 6, 9), (R4X, 4, 11)])
def test_exact_k_loop_computes_the_pair_terms(name, r, seed):
    lines = block_lines(name)
    assert sum(l.startswith("v_exp_f32") for l in lines) == 16
    ref = exact_k_reference(r)
    rng = np.random.default_rng(seed)
    for trial in range(60):
        cnt = 1 + trial % 3
        x = np.concatenate([rng.normal(0.0, 2.0, 16 * cnt), np.full(16, np.nan)]).astype(np.float32)
        ui = f32(rng.normal(0.0, 2.0))
        tot = rng.normal()
        want = tot
        for g in range(cnt):
            want = ref(x[16 * g:16 * g + 16], ui, K, want, K_LO)
        assert execute(lines, x, ui, K, tot, cnt, K_LO) == want


@pytest.mark.parametrize("name,ref,seed", [(R6, step_iv_reference, 5), (R4, step_vi_reference, 7)])
def test_loop_computes_the_pair_terms(name, ref, seed):
    lines = block_lines(name)
    assert sum(l.startswith("v_exp_f32") for l in lines) == 16
    assert sum(l.startswith("ds_read_b128") for l in lines) == 4
    rng = np.random.default_rng(seed)
    for trial in range(120):
        cnt = 1 + trial % 4
        # values past the last group are NaN: a read beyond it would show
        x = np.concatenate([rng.normal(0.0, 2.0, 16 * cnt), np.full(16, np.nan)]).astype(np.float32)
        ui = f32(rng.normal(0.0, 2.0))
        tot = rng.normal()
        assert execute(lines, x, ui, K, tot, cnt) == run_groups(ref, x, ui, K, tot, cnt)


def test_step_vi_loop_detects_a_planted_error():
    # the check above is not vacuous: reading the wrong register changes the result
    lines = block_lines(R4)
    i = next(i for i, l in enumerate(lines) if l.startswith("v_fmac_f32"))
    op, _, rest = lines[i].partition(" ")
    d, a, b = [t.strip() for t in rest.split(",")]
    same = lines[:i] + [f"{op} {d}, {b}, {a}"] + lines[i + 1:]     # product is commutative
    wrong = lines[:i] + [f"{op} {d}, {a}, {a}"] + lines[i + 1:]    # one factor read twice
    rng = np.random.default_rng(1)
    x = rng.normal(0.0, 1.0, 32).astype(np.float32)
    ref = run_groups(step_vi_reference, x, f32(0.3), K, 0.0, 2)
    assert execute(same, x, f32(0.3), K, 0.0, 2) == ref
    assert execute(wrong, x, f32(0.3), K, 0.0, 2) != ref


@pytest.mark.parametrize("name", [R6, R4, R6X, R4X])
def test_transcendental_results_are_not_read_in_the_next_instruction(name):
    lines = block_lines(name)
    body = [l for l in lines if not l.endswith(":") and not l.startswith(".")]
    for a, b in zip(body, body[1:] + body[:1]):     # the loop's back edge included
        if not a.startswith("v_exp_f32") or b.startswith(("v_exp_f32", "s_nop")):
            continue
        dst = a.split()[1].rstrip(",")
        ops = [t.strip().lstrip("-") for t in b.partition(" ")[2].split(",")]
        reads = ops[1:] + (ops[:1] if b.startswith("v_fmac") else [])
        assert dst not in reads, (a, b)


# encoded sizes (bytes) of the instructions that precede the first VALU op
HEAD_BYTES = {"v_mov_b32_e32": 4, "ds_read_b128": 8, "s_add_u32": 4, "s_sub_u32": 4, "s_waitcnt": 4}


@pytest.mark.parametrize("name,mod64", [(R6, 60), (R4, 0), (R6X, 60), (R4X, 60)])
def test_loop_body_placement(name, mod64):
    # the block starts on a 64-byte boundary; the padding before the loop
    # label runs once per call, and the first VALU op of the body lands where
    # each order was timed fastest
    lines = block_lines(name)
    assert lines[0] == ".p2align 6"
    label = lines.index("1:")
    assert all(l == "s_nop 0" for l in lines[1:label])
    off = 4 * (label - 1)
    for l in lines[label + 1:]:
        op = l.split()[0]
        if op.startswith("v_") and op != "v_mov_b32_e32":
            break
        assert op in HEAD_BYTES, l
        assert op != "s_add_u32" or l.endswith(", 64")     # inline constant, no literal
        off += HEAD_BYTES[op]
    assert off % 64 == mod64


@pytest.mark.parametrize("name", [R6, R4, R6X, R4X])
def test_block_operands_are_declared(name):
    text = open(SRC).read()
    start = text.index(f"void {name}(")
    end = text.index("\n}\n", start)
    fn = text[start:end]
    used = set(re.findall(r"%\[(\w+)\]", fn))
    declared = set(re.findall(r"\[(\w+)\] \"", fn))
    assert used <= declared, used - declared
    # operands the block writes are read-write
    lines = block_lines(name)
    for l in lines:
        m = re.match(r"[sv]_\w+ %\[(\w+)\],", l)
        if m and not l.startswith("s_cmp"):
            assert re.search(rf'\[{m.group(1)}\] "\+', fn), l
    # physical registers the block writes are clobbered, or are its pinned operands
    pinned = set(re.findall(r'"\+?\{(v\d+|v\[\d+:\d+\])\}"', fn))
    for line in lines:
        op, _, rest = line.partition(" ")
        if not op.startswith(("v_", "ds_read")):
            continue
        dst = rest.split(",")[0].strip()
        m = re.fullmatch(r"v(\d+)|v\[(\d+):(\d+)\]", dst)
        if not m:
            continue
        regs = [int(m.group(1))] if m.group(1) else list(range(int(m.group(2)), int(m.group(3)) + 1))
        for r in regs:
            assert f'"v{r}"' in fn or dst in pinned, (name, line)
    assert '"scc"' in fn


if __name__ == "__main__":
    pytest.main([__file__, "-q"])
