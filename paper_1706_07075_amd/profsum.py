"""Condense a rocprofv3 ``--stats --output-format csv`` kernel table into a
short Markdown table (kernel, calls, average / total milliseconds, share).

    python -m paper_1706_07075_amd.profsum <run>_kernel_stats.csv
"""
import csv
import re
import sys


def short_name(name: str) -> str:
    name = name.replace("void ", "").replace("lmtof::(anonymous namespace)::", "")
    m = re.match(r"([A-Za-z_0-9:]+(?:<[^>]*>)?)", name)
    return m.group(1) if m else name


def table(path: str) -> str:
    with open(path) as fh:
        rows = list(csv.DictReader(fh))
    out = ["| kernel | calls | avg ms | total ms | % of GPU time |", "|---|---|---|---|---|"]
    for r in rows:
        out.append(f"| `{short_name(r['Name'])}` | {r['Calls']} | {float(r['AverageNs']) / 1e6:.3f} | "
                   f"{float(r['TotalDurationNs']) / 1e6:.2f} | {float(r['Percentage']):.2f} |")
    return "\n".join(out)


if __name__ == "__main__":
    print(table(sys.argv[1]))
