"""The oracle and the HIP path share no code: the package (Python binding and
HIP sources) never imports, includes or loads the oracle, the oracle never
touches the package or its headers, and the seeded input generator, which
both sides use, depends on neither."""
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _sources(sub, exts):
    base = os.path.join(ROOT, sub)
    for dirpath, dirnames, files in os.walk(base):
        dirnames[:] = [d for d in dirnames if not d.startswith(("_", "."))]
        for f in files:
            if f.endswith(exts):
                yield os.path.join(dirpath, f), open(os.path.join(dirpath, f), errors="replace").read()


def _code(text):
    """Text without comments and docstrings (C and Python), so that prose
    naming the other side does not count."""
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    text = re.sub(r"//[^\n]*", "", text)
    text = re.sub(r'"""(.*?)"""', "", text, flags=re.S)
    return re.sub(r"#[^\n]*", lambda m: m.group(0) if m.group(0).startswith("#include") else "", text)


def test_package_never_uses_the_oracle():
    for path, text in _sources("paper_2410_02314_amd", (".py", ".hip", ".h", ".cpp")):
        code = _code(text)
        assert not re.search(r"\boracle\b", code), path


def test_oracle_never_uses_the_package():
    for path, text in _sources("oracle", (".py", ".c", ".h")):
        code = _code(text)
        assert "paper_2410_02314_amd" not in code and "dloc" not in code, path


def test_input_generator_uses_neither():
    for path, text in _sources("smlm_synth", (".py",)):
        if os.path.basename(path) == "make_calibration.py":
            continue            # writes stored constants with the oracle, by design
        code = _code(text)
        assert not re.search(r"import\s+oracle|from\s+oracle", code), path
        assert "paper_2410_02314_amd" not in code, path
