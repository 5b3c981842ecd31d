"""Aggregate the parity report the GPU tests write (GS_PARITY_REPORT=path.jsonl
pytest -m gpu): one forward table (per configuration: pixels compared strictly,
under the order bound, excluded; max-abs / RMS / rel-L2 of C, D, A) and one
gradient table (rel-L2 and element-wise violation fraction per tensor).
Usage: python tests/parity_table.py path.jsonl"""
import json, collections, math, sys


def main(path):
    rows = [json.loads(l) for l in open(path)]
    fw = collections.OrderedDict(); gr = collections.OrderedDict()
    for d in rows:
        if d["kind"] == "forward":
            a = fw.setdefault(d["config"], {"pixels": 0, "strict": 0, "bounded": 0, "excluded": 0, "views": 0,
                                            "C": [0.0, 0.0, 0.0, 0], "D": [0.0, 0.0, 0.0, 0], "A": [0.0, 0.0, 0.0, 0],
                                            "bmax": [0.0, 0.0, 0.0], "ex_share_max": 0.0})
            a["views"] += 1
            a["pixels"] += d["pixels"]; a["strict"] += d["strict"]; a["bounded"] += d["order_bounded"]; a["excluded"] += d["excluded"]
            a["ex_share_max"] = max(a["ex_share_max"], d["excluded_share"] if d["pixels"] >= 100 else 0.0)
            for k in "CDA":
                st = d[k]
                a[k][0] = max(a[k][0], st["max_abs"])
                a[k][1] += st["rms"] ** 2 * d["strict"] * (3 if k == "C" else 1)
                a[k][2] = max(a[k][2], st["rel_l2"])
                a[k][3] += d["strict"] * (3 if k == "C" else 1)
            if d.get("bounded_max_abs"):
                a["bmax"] = [max(x, y) for x, y in zip(a["bmax"], d["bounded_max_abs"])]
        else:
            name = d["output"] if not d["output"].startswith("pose[") else "pose (worst view)"
            key = (d["config"], name)
            g = gr.get(key)
            if g is None or d["rel_l2"] > g["rel_l2"]:
                gr[key] = {"rel_l2": d["rel_l2"], "viol": d["violation_fraction"], "n": d["elements"]}
            else:
                g["viol"] = max(g["viol"], d["violation_fraction"])
    print("| configuration | views | pixels | strict / order-bounded / excluded | worst excluded share of a view | C max-abs / RMS / rel-L2 | D max-abs / RMS / rel-L2 | A max-abs / RMS / rel-L2 | order-bounded max-abs C, D, A |")
    print("|---|---:|---:|---|---:|---|---|---|---|")
    for cfg, a in fw.items():
        def f(k):
            m, s2, r, n = a[k]
            return f"{m:.1e} / {math.sqrt(s2 / n) if n else 0:.1e} / {r:.1e}"
        print(f"| {cfg} | {a['views']} | {a['pixels']} | {a['strict']} / {a['bounded']} / {a['excluded']} | {a['ex_share_max']:.3f} | {f('C')} | {f('D')} | {f('A')} | {a['bmax'][0]:.1e}, {a['bmax'][1]:.1e}, {a['bmax'][2]:.1e} |")
    print()
    cfgs = collections.OrderedDict()
    for (cfg, name), g in gr.items():
        cfgs.setdefault(cfg, {})[name] = g
    names = ["means", "log_scales", "log_radius", "quats", "opacity_logits", "colors", "pose (worst view)"]
    print("| configuration | " + " | ".join(names) + " |")
    print("|---|" + "---|" * len(names))
    for cfg, d in cfgs.items():
        cells = []
        for n in names:
            g = d.get(n)
            cells.append("—" if g is None else f"{g['rel_l2']:.1e} ({g['viol']:.0e})")
        print(f"| {cfg} | " + " | ".join(cells) + " |")


if __name__ == "__main__":
    main(sys.argv[1])
