"""Constants of the table-driven exponential in rg_prelude.h (Tang's method:
P. T. P. Tang, "Table-driven implementation of the exponential function in
IEEE floating-point arithmetic", ACM TOMS 15 (1989) 144-157), computed in
60-digit decimal arithmetic and rounded once to double.

    x = (N m + j) ln2/N + r,  |r| <= ln2/(2N),  e^x = 2^m 2^(j/N) e^r

with N = 2^BITS table entries.

Prints the C block that rg_prelude.h holds between its RG_EXP_TABLE
markers; tests check that the two agree."""
from decimal import Decimal, getcontext

getcontext().prec = 60

BITS = 8
N = 1 << BITS


def hexd(v) -> str:
    return float(v).hex()


def block() -> str:
    ln2 = Decimal(2).ln()
    step = ln2 / N
    # high part with 32 significant bits: n * L1 is exact for |n| < 2^21
    e = 0
    while step * (2 ** e) < 2 ** 31:
        e += 1
    l1 = Decimal(int((step * (2 ** e)).to_integral_value())) / (2 ** e)
    l2 = step - l1
    lines = ["// RG_EXP_TABLE begin (written by gen_exp_table.py)",
             f"#define RG_EXP_BITS {BITS}",
             f"#define RG_EXP_N {N}",
             f"#define RG_EXP_INV_L ({hexd(N / ln2)})  /* {N} / ln 2 */",
             f"#define RG_EXP_L1 ({hexd(l1)})  /* ln2/{N}, high 32 bits */",
             f"#define RG_EXP_L2 ({hexd(l2)})  /* ln2/{N} - L1 */",
             "#define RG_EXP_TABLE_VALUES \\"]
    vals = [hexd(Decimal(2) ** (Decimal(j) / N)) for j in range(N)]
    for i in range(0, N, 4):
        lines.append("    " + ", ".join(vals[i:i + 4]) + (", \\" if i + 4 < N else ""))
    lines.append("// RG_EXP_TABLE end")
    return "\n".join(lines) + "\n"


if __name__ == "__main__":
    print(block(), end="")
