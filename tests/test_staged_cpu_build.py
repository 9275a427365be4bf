"""The staged g g -> t t~ g g g diagram kernels built for the CPU.

The FP64 chunk kernels of g g -> t t~ g g g once returned wrong values on
gfx950 (relative errors 4e-4 to 5e-2 on every checked event) in a variant
that passed each external wavefunction through an empty volatile asm
statement before every use (fresh()/fresh_pol() in helamp.h).  These tests
settle where that defect was:

  - the variant differs from the generated sources only by those identity
    barriers (it is rebuilt here from the current sources by wrapping every
    use of an external wavefunction, and unwrapping it gives the current
    sources back character for character);
  - both variants, compiled for the host CPU from the same generated bodies
    and helamp.h (with the two gfx950 builtins replaced by their exact
    meaning: a reciprocal, and a scheduling hint), give |M|^2 within 1e-12
    of the oracle on the same 67 events that failed on the GPU.

So the generated program is exact with and without the barriers; the wrong
values came from the device compilation of the barrier variant, not from
the code generator.  The generator no longer emits that variant, and the
first test fails if it ever does again.

The host build includes each chunk's prologue that fills the kinematics
rows (momentum sums and denominators the chunk reads from LDS), run for the
one event of column 0, so the rows' assignment and contents are checked
against the oracle too.
"""
import concurrent.futures as cf
import os
import re
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2303_18244_amd", "csrc")
SEED = 230318244
N_EVENTS = 67
GLUON_LEGS = (0, 1, 4, 5, 6)
EXT_DECL = re.compile(r"^\s*(const )?wf<T> x\d+ = ")
EXT_USE = re.compile(r"\bx(\d+)\b")
BARRIER = re.compile(r"\bfresh(_pol)?\((x\d+)\)")


def _staged_meta():
    from paper_2303_18244_amd.build import PROCESSES, STAGED
    from paper_2303_18244_amd.codegen.emit import emit_gg_staged

    nch, budget, inplace, lds = STAGED["gg_ttggg"]
    return emit_gg_staged("gg_ttggg", PROCESSES["gg_ttggg"], nch, budget, inplace=inplace, lds=lds)


def barrier_variant(body: str) -> str:
    """Every use of an external wavefunction x<i> (not its declaration)
    wrapped in the identity barrier of its kind."""
    out = []
    for line in body.split("\n"):
        if not EXT_DECL.match(line):
            line = EXT_USE.sub(lambda m: (f"fresh_pol(x{m.group(1)})" if int(m.group(1)) in GLUON_LEGS
                                          else f"fresh(x{m.group(1)})"), line)
        out.append(line)
    return "\n".join(out)


@pytest.fixture(scope="module")
def meta():
    return _staged_meta()


def test_staged_generator_passes_no_external_through_a_barrier(meta):
    for c, body in enumerate(meta["chunk_bodies"]):
        assert not BARRIER.search(body), f"chunk {c} passes an external wavefunction through a barrier"


def test_barrier_variant_differs_only_by_identity_barriers(meta):
    n_wrapped = 0
    for body in meta["chunk_bodies"]:
        var = barrier_variant(body)
        n_wrapped += len(BARRIER.findall(var))
        assert BARRIER.sub(r"\2", var) == body
    assert n_wrapped > 1000


CHUNK_UNIT = r"""// chunk {c} of g g -> t t~ g g g, {variant}, for the host CPU
#define __builtin_amdgcn_rcp(x) (1.0 / (x))
#define __builtin_amdgcn_sched_barrier(x) ((void)0)
#include "{csrc}/helamp.h"
#include "{csrc}/me_kernel.h"
namespace mgme {{
void {variant}_chunk{c}(const double (&q)[7][4], int hc, double mt, cx<double>* Jc, cx<double>* Ov, long long ldp) {{
  using T = double;
  constexpr int NEXT = 7;
  (void)Ov;
  // the kernel's LDS rows, for the one event of column 0
  constexpr int EV = 64;
  constexpr int HB = 4;
  const int lane = 0;
  static double smom[NEXT * 4 * EV];
  for (int i = 0; i < NEXT; ++i)
    for (int mu = 0; mu < 4; ++mu) smom[(i * 4 + mu) * EV] = q[i][mu];
{rows_decl}
  static T skin[NKIN * 4 * EV];
  static T sden[NDEN * EV];
  for (int slot = 0; slot < HB; ++slot) {{
{rows_fill}
  }}
{body}
}}
}}  // namespace mgme
"""

DRIVER = r"""// host driver: |M|^2 of events read from stdin-named file with every chunk
// in order, then the colour sum from the upper doubled numerators
#include <cstdio>
#include <vector>
#define __builtin_amdgcn_rcp(x) (1.0 / (x))
#define __builtin_amdgcn_sched_barrier(x) ((void)0)
#include "{csrc}/helamp.h"
namespace mgme {{
{decls}
}}
using namespace mgme;
static const double kCud[{ncol}][{ncol}] = {{{cud}}};
int main(int argc, char** argv) {{
  FILE* f = std::fopen(argv[1], "rb");
  int n = 0;
  if (!f || std::fread(&n, sizeof n, 1, f) != 1) return 1;
  std::vector<double> mom((size_t)n * 28);
  if (std::fread(mom.data(), sizeof(double), mom.size(), f) != mom.size()) return 2;
  std::fclose(f);
  const double factor = {factor!r};
  for (int e = 0; e < n; ++e) {{
    double q[7][4];
    for (int i = 0; i < 7; ++i)
      for (int mu = 0; mu < 4; ++mu) q[i][mu] = mom[(size_t)e * 28 + i * 4 + mu];
    double total = 0.0;
    for (int hc = 0; hc < 128; ++hc) {{
      cx<double> J[{ncol}], Ov[{nov}];
      for (auto& j : J) j = mk<double>(0.0, 0.0);
      for (auto& o : Ov) o = mk<double>(0.0, 0.0);
{calls}
{overflow}
      double me = 0.0;
      for (int s = 0; s < {ncol}; ++s) {{
        double yr = 0.0, yi = 0.0;
        for (int t = s; t < {ncol}; ++t) {{ yr += kCud[s][t] * J[t].re; yi += kCud[s][t] * J[t].im; }}
        me += J[s].re * yr + J[s].im * yi;
      }}
      total += me;
    }}
    std::printf("%.17g\n", total * factor);
  }}
  return 0;
}}
"""


def _compile(args):
    src, obj = args
    r = subprocess.run(["g++", "-std=c++17", "-O1", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include", "-c", src,
                        "-o", obj], capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(r.stderr[-3000:])
    return obj


@pytest.mark.slow
def test_cpu_build_of_both_variants_matches_oracle(meta, oracle_mod, tmp_path):
    import math

    from paper_2303_18244_amd.build import PROCESSES

    pdg = PROCESSES["gg_ttggg"]
    ncol, nov = meta["ncol"], max(1, meta["n_overflow"])
    nchunk = len(meta["chunk_bodies"])
    cden = meta["cden"]
    num = meta["colour_num"]
    cud = [0.0 if t < s else (num[s * ncol + t] if t == s else 2.0 * num[s * ncol + t])
           for s in range(ncol) for t in range(ncol)]
    gs = math.sqrt(4.0 * math.pi * 0.118)
    factor = gs ** meta["gs_power"] / (meta["spin_colour_avg"] * meta["ident"]) / cden
    overflow = "\n".join(
        f"      J[{fl}].re += {' + '.join(f'Ov[{k}].re' for k in sl)}; "
        f"J[{fl}].im += {' + '.join(f'Ov[{k}].im' for k in sl)};"
        for fl, sl in enumerate(meta["overflow_of"]) if sl)
    host, _ = oracle_mod.rambo([173.0 if abs(x) == 6 else 0.0 for x in pdg[2:]], 1500.0, SEED, 0, N_EVENTS)
    evfile = tmp_path / "events.bin"
    with open(evfile, "wb") as f:
        f.write(np.int32(N_EVENTS).tobytes())
        f.write(np.ascontiguousarray(host, dtype=np.float64).tobytes())
    O = oracle_mod.Process(oracle_mod.PROCESSES["gg_ttggg"])
    ref = O.me(host, nthreads=max(1, min(8, os.cpu_count() or 1)))
    units = []
    for variant in ("plain", "barrier"):
        for c, body in enumerate(meta["chunk_bodies"]):
            decl, fill = meta["chunk_prologues"][c].split("\n", 2)[:2], meta["chunk_prologues"][c].split("\n", 2)[2]
            text = CHUNK_UNIT.format(c=c, variant=variant, csrc=CSRC, rows_decl="\n".join(decl), rows_fill=fill,
                                     body=body if variant == "plain" else barrier_variant(body))
            src = tmp_path / f"{variant}_chunk{c}.cpp"
            src.write_text(text)
            units.append((str(src), str(tmp_path / f"{variant}_chunk{c}.o")))
        decls = "\n".join(f"void {variant}_chunk{c}(const double (&)[7][4], int, double, cx<double>*, cx<double>*, "
                          f"long long);" for c in range(nchunk))
        calls = "\n".join(f"      {variant}_chunk{c}(q, hc, 173.0, J, Ov, 1);" for c in range(nchunk))
        drv = tmp_path / f"{variant}_driver.cpp"
        drv.write_text(DRIVER.format(csrc=CSRC, decls=decls, ncol=ncol, nov=nov,
                                     cud=", ".join(repr(v) for v in cud), factor=factor, calls=calls,
                                     overflow=overflow))
        units.append((str(drv), str(tmp_path / f"{variant}_driver.o")))
    with cf.ThreadPoolExecutor(max(1, min(8, os.cpu_count() or 1))) as ex:
        objs = list(ex.map(_compile, units))
    results = {}
    for variant in ("plain", "barrier"):
        exe = str(tmp_path / variant)
        subprocess.run(["g++", "-o", exe] + [o for o in objs if os.path.basename(o).startswith(variant)],
                       check=True)
        r = subprocess.run([exe, str(evfile)], capture_output=True, text=True, check=True, timeout=600)
        results[variant] = np.array([float(x) for x in r.stdout.split()])
    for variant, me in results.items():
        rel = np.abs(me / ref - 1.0)
        bad = np.nonzero(rel > 1e-12)[0]
        if len(bad):
            ld = O.me(host[bad], precision=1)
            assert np.all(np.abs(me[bad] / ld - 1.0) <= 1e-12), (variant, bad, rel[bad])
        print(f"{variant}: {N_EVENTS} events, max rel deviation from the oracle {rel.max():.2e}")
    # the barrier is an identity on the CPU: bit for bit the same program
    assert np.array_equal(results["plain"], results["barrier"])
